"""MI355X-native single-temperature MCMC decoder for the planar surface code
(Hutter, Wootton, Loss, arXiv:1302.2669).

Python face of libmcmcdec.so.  Functions take and return torch tensors on a
HIP device and run on the current torch stream; they only marshal arguments.
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import (MCMC_INIT_CANONICAL, MCMC_INIT_MATCHING, MCMC_INIT_MWPM, MCMC_L_MAX,
                   MCMC_L_MIN,
                   MCMC_NOISE_BITPHASE, MCMC_NOISE_DEPOLARIZING, MCMC_RANDOM_SCAN, MCMC_RESUME,
                   MCMC_TRACE, McmcError, Params)

__all__ = ["Params", "McmcError", "geometry", "lattice", "acceptance_table", "workspace_size",
           "chain_state_size", "decode_batch", "sample_errors", "init_representatives",
           "start_weights", "unpack_chain_state", "MCMC_TRACE", "MCMC_RESUME",
           "MCMC_RANDOM_SCAN", "MCMC_L_MIN", "MCMC_L_MAX",
           "MCMC_INIT_CANONICAL", "MCMC_INIT_MATCHING", "MCMC_INIT_MWPM", "MCMC_NOISE_DEPOLARIZING",
           "MCMC_NOISE_BITPHASE", "params_table", "MixedPlan", "spacetime_params",
           "spacetime_tables", "sample_spacetime", "decode_spacetime"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_GEOMETRY = {}


def geometry(L):
    """(n_qubits, n_stab) of a distance-L code."""
    L = int(L)
    if L not in _GEOMETRY:
        nq, ns = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib._lib().mcmc_geometry(L, ctypes.byref(nq), ctypes.byref(ns)),
                   "mcmc_geometry")
        _GEOMETRY[L] = (nq.value, ns.value)
    return _GEOMETRY[L]


def lattice(L):
    """(supports [n_stab, 4] (-1 padded), colour [n_stab], draw [n_stab]) as numpy."""
    _, ns = geometry(L)
    sup = np.zeros((ns, 4), dtype=np.int32)
    col = np.zeros(ns, dtype=np.int32)
    drw = np.zeros(ns, dtype=np.int32)
    _lib.check(_lib._lib().mcmc_lattice(L, sup.ctypes.data, col.ctypes.data, drw.ctypes.data),
               "mcmc_lattice")
    return sup, col, drw


def acceptance_table(p, n_temps=1):
    out = np.zeros((n_temps, 4), dtype=np.uint32)
    _lib.check(_lib._lib().mcmc_acceptance_table(float(p), int(n_temps), out.ctypes.data),
               "mcmc_acceptance_table")
    return out


def make_params(L, p, sweeps, seed, chains=1, n_temps=1, burn=0, sweep_begin=0, flags=0,
                init=MCMC_INIT_MATCHING, noise=MCMC_NOISE_DEPOLARIZING, beta_scale=0.0):
    """beta_scale 0 selects the noise model's default beta*/beta_bar."""
    return Params(L=int(L), n_temps=int(n_temps), chains=int(chains), burn=int(burn),
                  sweeps=int(sweeps), sweep_begin=int(sweep_begin), p=float(p),
                  seed=int(seed) & ((1 << 64) - 1), flags=int(flags), init=int(init),
                  noise=int(noise), reserved=0, beta_scale=float(beta_scale))


def params_table(prm):
    """[n_temps, 4] uint32 thresholds a decode with these Params uses."""
    out = np.zeros((prm.n_temps, 4), dtype=np.uint32)
    _lib.check(_lib._lib().mcmc_params_table(ctypes.byref(prm), out.ctypes.data),
               "mcmc_params_table")
    return out


def workspace_size(prm, n):
    b = ctypes.c_size_t()
    _lib.check(_lib._lib().mcmc_workspace_size(ctypes.byref(prm), int(n), ctypes.byref(b)),
               "mcmc_workspace_size")
    return b.value


def chain_state_size(prm, n):
    b = ctypes.c_size_t()
    _lib.check(_lib._lib().mcmc_chain_state_size(ctypes.byref(prm), int(n), ctypes.byref(b)),
               "mcmc_chain_state_size")
    return b.value


def decode_batch(syndromes, L, p, sweeps, seed, chains=1, n_temps=1, burn=0, syndrome_ids=None,
                 want_sums=False, want_correction=True, trace=False, chain_state=None,
                 resume_from=None, workspace=None, init=MCMC_INIT_MATCHING,
                 noise=MCMC_NOISE_DEPOLARIZING, beta_scale=0.0, random_scan=False):
    """Decode a [n, n_stab] uint8 device tensor of syndromes.  `noise` picks
    the error model p refers to (depolarizing, or independent bit/phase flips
    of rate p per part); `beta_scale` sets beta*/beta_bar for n_temps = 1
    (0: the model's default); `random_scan` runs Sec. IV's one-random-
    stabilizer-per-step chains instead of the colour-phased sweeps.

    Returns a dict of device tensors: class_prob [n,4] f64, mean_n [n,4] f64,
    chosen [n] u8, and when requested correction [n,n_q] u8, sum_n/accepts
    [n,4,K,chains] i64, trace [n,4,K,chains,4*(burn+sweeps-begin)] i16,
    chain_state (uint8 buffer).  `resume_from=(state_buffer, sweep_begin)`
    continues earlier chains (MCMC_RESUME).
    """
    torch = _torch()
    dev = syndromes.device
    n = int(syndromes.shape[0])
    nq, ns = geometry(L)
    if syndromes.dtype != torch.uint8 or syndromes.dim() != 2 or syndromes.shape[1] != ns:
        raise ValueError(f"syndromes must be uint8 [n, {ns}]")
    syndromes = syndromes.contiguous()
    flags = ((_lib.MCMC_TRACE if trace else 0) | (_lib.MCMC_RESUME if resume_from is not None else 0)
             | (_lib.MCMC_RANDOM_SCAN if random_scan else 0))
    begin = 0 if resume_from is None else int(resume_from[1])
    prm = make_params(L, p, sweeps, seed, chains, n_temps, burn, begin, flags, init, noise,
                      beta_scale)
    out = {
        "class_prob": torch.empty((n, 4), dtype=torch.float64, device=dev),
        "mean_n": torch.empty((n, 4), dtype=torch.float64, device=dev),
        "chosen": torch.empty((n,), dtype=torch.uint8, device=dev),
    }
    if want_correction:
        out["correction"] = torch.empty((n, nq), dtype=torch.uint8, device=dev)
    if want_sums:
        out["sum_n"] = torch.empty((n, 4, n_temps, chains), dtype=torch.int64, device=dev)
        out["accepts"] = torch.empty((n, 4, n_temps, chains), dtype=torch.int64, device=dev)
    if trace:
        out["trace"] = torch.empty((n, 4, n_temps, chains, 4 * (burn + sweeps - begin)),
                                   dtype=torch.int16, device=dev)
    cs = None
    if resume_from is not None:
        cs = resume_from[0]
    elif chain_state:
        cs = torch.empty((chain_state_size(prm, n),), dtype=torch.uint8, device=dev)
    if cs is not None:
        out["chain_state"] = cs
    if workspace is None:
        workspace = torch.empty((max(workspace_size(prm, n), 1),), dtype=torch.uint8, device=dev)
    ids = None
    if syndrome_ids is not None:
        ids = syndrome_ids.to(device=dev, dtype=torch.int32).contiguous()
    st = _lib._lib().mcmc_decode_batch(
        _ptr(syndromes), _ptr(ids), n, ctypes.byref(prm), _ptr(out["class_prob"]),
        _ptr(out["mean_n"]), _ptr(out.get("sum_n")), _ptr(out.get("accepts")), _ptr(out["chosen"]),
        _ptr(out.get("correction")), _ptr(cs), _ptr(out.get("trace")), _ptr(workspace),
        workspace.numel(), _stream(dev))
    _lib.check(st, "mcmc_decode_batch")
    return out


def sample_errors(L, p, seed, n, device="cuda", id_base=0, sample_ids=None, want_errors=False,
                  noise=MCMC_NOISE_DEPOLARIZING):
    """Samples of the noise model: (syndromes [n,n_stab] u8, true_class [n] u8,
    errors [n,n_q] u8 or None)."""
    torch = _torch()
    nq, ns = geometry(L)
    syn = torch.empty((n, ns), dtype=torch.uint8, device=device)
    cls = torch.empty((n,), dtype=torch.uint8, device=device)
    err = torch.empty((n, nq), dtype=torch.uint8, device=device) if want_errors else None
    ids = None if sample_ids is None else sample_ids.to(device=device, dtype=torch.int32).contiguous()
    st = _lib._lib().mcmc_sample_errors_model(int(L), int(noise), float(p),
                                              int(seed) & ((1 << 64) - 1), _ptr(ids), int(id_base),
                                              int(n), _ptr(syn), _ptr(cls), _ptr(err),
                                              _stream(syn.device))
    _lib.check(st, "mcmc_sample_errors_model")
    return syn, cls, err


def init_representatives(syndromes, L, init=MCMC_INIT_MATCHING):
    torch = _torch()
    nq, ns = geometry(L)
    n = int(syndromes.shape[0])
    reps = torch.empty((n, 4, nq), dtype=torch.uint8, device=syndromes.device)
    st = _lib._lib().mcmc_init_representatives(int(L), int(init), _ptr(syndromes.contiguous()), n,
                                               _ptr(reps), _stream(syndromes.device))
    _lib.check(st, "mcmc_init_representatives")
    return reps


def start_weights(syndromes, L, init=MCMC_INIT_MATCHING):
    """int32 [n][4]: the weights of the four class starts (mcmc_start_weights)."""
    torch = _torch()
    n = int(syndromes.shape[0])
    w = torch.empty((n, 4), dtype=torch.int32, device=syndromes.device)
    st = _lib._lib().mcmc_start_weights(int(L), int(init), _ptr(syndromes.contiguous()), n,
                                        _ptr(w), _stream(syndromes.device))
    _lib.check(st, "mcmc_start_weights")
    return w


def unpack_chain_state(chain_state, n, L, p, sweeps, seed, chains=1, n_temps=1, burn=0,
                       noise=MCMC_NOISE_DEPOLARIZING):
    torch = _torch()
    nq, _ = geometry(L)
    prm = make_params(L, p, sweeps, seed, chains, n_temps, burn, noise=noise)
    states = torch.empty((n, 4, n_temps, chains, nq), dtype=torch.uint8, device=chain_state.device)
    weights = torch.empty((n, 4, n_temps, chains), dtype=torch.int32, device=chain_state.device)
    st = _lib._lib().mcmc_unpack_chain_state(ctypes.byref(prm), int(n), _ptr(chain_state),
                                             _ptr(states), _ptr(weights),
                                             _stream(chain_state.device))
    _lib.check(st, "mcmc_unpack_chain_state")
    return states, weights


def spacetime_params(L, rounds, p, p_m, sweeps, seed, chains=1, burn=0):
    return _lib.SpaceTimeParams(L=int(L), rounds=int(rounds), chains=int(chains), burn=int(burn),
                                sweeps=int(sweeps), reserved=0, p=float(p), p_m=float(p_m),
                                seed=int(seed) & ((1 << 64) - 1))


def spacetime_tables(prm):
    """(spatial [4], time [5, 5] indexed (dn+2, dm+2), always [5, 5] bool, xi)."""
    sp = np.zeros(4, dtype=np.uint32)
    tt = np.zeros(25, dtype=np.uint32)
    al = ctypes.c_uint32()
    xi = ctypes.c_double()
    _lib.check(_lib._lib().mcmc_spacetime_tables(ctypes.byref(prm), sp.ctypes.data,
                                                 tt.ctypes.data, ctypes.byref(al),
                                                 ctypes.byref(xi)), "mcmc_spacetime_tables")
    always = np.array([(al.value >> e) & 1 for e in range(25)], dtype=bool).reshape(5, 5)
    return sp, tt.reshape(5, 5), always, xi.value


def sample_spacetime(L, rounds, p, p_m, seed, n, device="cuda", id_base=0):
    """(observations [n, rounds, n_stab] u8, true_class [n] u8) of the
    imperfect-measurement model."""
    torch = _torch()
    _, ns = geometry(L)
    obs = torch.empty((n, rounds, ns), dtype=torch.uint8, device=device)
    cls = torch.empty((n,), dtype=torch.uint8, device=device)
    st = _lib._lib().mcmc_sample_spacetime(int(L), int(rounds), float(p), float(p_m),
                                           int(seed) & ((1 << 64) - 1), int(id_base), int(n),
                                           _ptr(obs), _ptr(cls), _stream(obs.device))
    _lib.check(st, "mcmc_sample_spacetime")
    return obs, cls


def decode_spacetime(obs, L, p, p_m, sweeps, seed, chains=1, burn=0, syndrome_ids=None,
                     want_sums=False, want_correction=True, workspace=None):
    """Decode observation histories obs [n, rounds, n_stab] u8 (device) under
    imperfect measurements.  Returns class_prob, mean_n, mean_m, chosen and
    optionally correction, sum_n, sum_m, accepts ([n, 4, chains])."""
    torch = _torch()
    dev = obs.device
    n, T = int(obs.shape[0]), int(obs.shape[1])
    nq, ns = geometry(L)
    if obs.dtype != torch.uint8 or obs.dim() != 3 or obs.shape[2] != ns:
        raise ValueError(f"observations must be uint8 [n, rounds, {ns}]")
    obs = obs.contiguous()
    prm = spacetime_params(L, T, p, p_m, sweeps, seed, chains, burn)
    b = ctypes.c_size_t()
    _lib.check(_lib._lib().mcmc_spacetime_workspace_size(ctypes.byref(prm), n, ctypes.byref(b)),
               "mcmc_spacetime_workspace_size")
    out = {"class_prob": torch.empty((n, 4), dtype=torch.float64, device=dev),
           "mean_n": torch.empty((n, 4), dtype=torch.float64, device=dev),
           "mean_m": torch.empty((n, 4), dtype=torch.float64, device=dev),
           "chosen": torch.empty((n,), dtype=torch.uint8, device=dev)}
    if want_correction:
        out["correction"] = torch.empty((n, nq), dtype=torch.uint8, device=dev)
    if want_sums:
        for k in ("sum_n", "sum_m", "accepts"):
            out[k] = torch.empty((n, 4, chains), dtype=torch.int64, device=dev)
    if workspace is None:
        workspace = torch.empty((max(b.value, 1),), dtype=torch.uint8, device=dev)
    ids = None if syndrome_ids is None else \
        syndrome_ids.to(device=dev, dtype=torch.int32).contiguous()
    st = _lib._lib().mcmc_decode_spacetime(
        _ptr(obs), _ptr(ids), n, ctypes.byref(prm), _ptr(out["class_prob"]), _ptr(out["mean_n"]),
        _ptr(out["mean_m"]), _ptr(out.get("sum_n")), _ptr(out.get("sum_m")),
        _ptr(out.get("accepts")), _ptr(out["chosen"]), _ptr(out.get("correction")),
        _ptr(workspace), workspace.numel(), _stream(dev))
    _lib.check(st, "mcmc_decode_spacetime")
    return out


# numpy twin of the C mcmc_item struct (natural alignment, 64 bytes)
_ITEM_DTYPE = np.dtype([("L", "<i4"), ("sweeps", "<i4"), ("burn", "<i4"), ("chains", "<i4"),
                        ("n_temps", "<i4"), ("syndrome_id", "<u4"), ("p", "<f8"),
                        ("syn_offset", "<i8"), ("corr_offset", "<i8"), ("noise", "<u4"),
                        ("reserved", "<u4"), ("beta_scale", "<f8")], align=True)
assert _ITEM_DTYPE.itemsize == ctypes.sizeof(_lib.Item)


class MixedPlan:
    """A mixed batch: syndromes of different L, p, budgets and chain counts
    decoded by one plan (see mcmc_plan_* in the C header).

    `items` is a sequence of dicts with keys L, p, sweeps and optionally burn
    (0), chains (1), n_temps (1), syndrome_id (position), noise (depolarizing)
    and beta_scale (0: the model's default).  Syndromes are passed
    as one flat uint8 device tensor: item i's n_stab(L_i) bytes after those of
    items 0..i-1; corrections come back the same way (n_q(L_i) bytes each).
    """

    def __init__(self, items, seed, init=MCMC_INIT_MATCHING):
        n = len(items)
        cols = {k: np.asarray([it.get(k, d) if k != "syndrome_id" else it.get(k, i)
                               for i, it in enumerate(items)])
                for k, d in (("L", 0), ("p", 0.0), ("sweeps", 0), ("burn", 0), ("chains", 1),
                             ("n_temps", 1), ("syndrome_id", 0), ("noise", 0),
                             ("beta_scale", 0.0))} if n else {}
        self._build(n, cols, seed, init)

    @classmethod
    def from_arrays(cls, L, p, sweeps, seed, chains=1, n_temps=1, burn=0, syndrome_ids=None,
                    init=MCMC_INIT_MATCHING, noise=MCMC_NOISE_DEPOLARIZING, beta_scale=0.0):
        """Same as the constructor, from per-item arrays (scalars broadcast)."""
        p = np.asarray(p, dtype=np.float64).reshape(-1)
        n = p.size
        bc = lambda v: np.broadcast_to(np.asarray(v), (n,))  # noqa: E731
        cols = dict(L=bc(L), p=p, sweeps=bc(sweeps), burn=bc(burn), chains=bc(chains),
                    n_temps=bc(n_temps), noise=bc(noise), beta_scale=bc(beta_scale),
                    syndrome_id=np.arange(n) if syndrome_ids is None else bc(syndrome_ids))
        self = cls.__new__(cls)
        self._build(n, cols, seed, init)
        return self

    def _build(self, n, cols, seed, init):
        arr = np.zeros(max(n, 1), dtype=_ITEM_DTYPE)
        self.L = np.zeros(n, dtype=np.int32)
        self.syn_offsets = np.zeros(n + 1, dtype=np.int64)
        self.corr_offsets = np.zeros(n + 1, dtype=np.int64)
        self.chain_offsets = np.zeros(n + 1, dtype=np.int64)
        if n:
            L = cols["L"].astype(np.int32)
            geo = {int(v): geometry(int(v)) for v in np.unique(L)}
            nq = np.asarray([geo[int(v)][0] for v in L], dtype=np.int64)
            ns = np.asarray([geo[int(v)][1] for v in L], dtype=np.int64)
            np.cumsum(ns, out=self.syn_offsets[1:])
            np.cumsum(nq, out=self.corr_offsets[1:])
            arr = arr[:n]
            arr["L"] = L
            arr["sweeps"] = cols["sweeps"]
            arr["burn"] = cols["burn"]
            arr["chains"] = cols["chains"]
            arr["n_temps"] = cols["n_temps"]
            arr["syndrome_id"] = cols["syndrome_id"].astype(np.int64) & 0xFFFFFFFF
            arr["p"] = cols["p"]
            arr["syn_offset"] = self.syn_offsets[:-1]
            arr["corr_offset"] = self.corr_offsets[:-1]
            arr["noise"] = cols["noise"]
            arr["beta_scale"] = cols["beta_scale"]
            self.L[:] = L
            np.cumsum(4 * arr["n_temps"].astype(np.int64) * arr["chains"],
                      out=self.chain_offsets[1:])
        self.n = n
        self.syn_bytes, self.corr_bytes = int(self.syn_offsets[-1]), int(self.corr_offsets[-1])
        h = ctypes.c_void_p()
        _lib.check(_lib._lib().mcmc_plan_create(arr.ctypes.data_as(ctypes.POINTER(_lib.Item)), n,
                                                int(seed) & ((1 << 64) - 1), int(init),
                                                ctypes.byref(h)), "mcmc_plan_create")
        self._h = h
        tc, wb, tu = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_int64()
        _lib.check(_lib._lib().mcmc_plan_info(h, ctypes.byref(tc), ctypes.byref(wb),
                                              ctypes.byref(tu)), "mcmc_plan_info")
        self.total_chains, self.workspace_bytes, self.total_updates = tc.value, wb.value, tu.value
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            _lib._lib().mcmc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _outputs(self, dev, want_sums, want_correction):
        torch = _torch()
        out = {
            "class_prob": torch.empty((self.n, 4), dtype=torch.float64, device=dev),
            "mean_n": torch.empty((self.n, 4), dtype=torch.float64, device=dev),
            "chosen": torch.empty((self.n,), dtype=torch.uint8, device=dev),
        }
        if want_correction:
            out["correction"] = torch.empty((max(self.corr_bytes, 1),), dtype=torch.uint8, device=dev)
        if want_sums:
            out["sum_n"] = torch.empty((max(self.total_chains, 1),), dtype=torch.int64, device=dev)
            out["accepts"] = torch.empty((max(self.total_chains, 1),), dtype=torch.int64, device=dev)
        return out

    def _args(self, syndromes, out):
        torch = _torch()
        if self._ws is None or self._ws.device != syndromes.device:
            self._ws = torch.empty((max(self.workspace_bytes, 1),), dtype=torch.uint8,
                                   device=syndromes.device)
        return (self._h, _ptr(syndromes), _ptr(out["class_prob"]), _ptr(out["mean_n"]),
                _ptr(out.get("sum_n")), _ptr(out.get("accepts")), _ptr(out["chosen"]),
                _ptr(out.get("correction")), _ptr(self._ws), self._ws.numel(),
                _stream(syndromes.device))

    def _check_input(self, syndromes):
        torch = _torch()
        if syndromes.dtype != torch.uint8 or syndromes.dim() != 1 or \
                syndromes.numel() < self.syn_bytes:
            raise ValueError(f"syndromes must be a flat uint8 tensor of {self.syn_bytes} bytes")
        return syndromes.contiguous()

    def execute(self, syndromes, want_sums=False, want_correction=True, graph=False, out=None):
        syndromes = self._check_input(syndromes)
        if out is None:
            out = self._outputs(syndromes.device, want_sums, want_correction)
        fn = _lib._lib().mcmc_plan_graph_launch if graph else _lib._lib().mcmc_plan_execute
        _lib.check(fn(*self._args(syndromes, out)),
                   "mcmc_plan_graph_launch" if graph else "mcmc_plan_execute")
        return out

    def sample(self, seed, device="cuda"):
        """Samples of every item under its own noise model and rate: (flat
        syndromes, true classes)."""
        torch = _torch()
        syn = torch.empty((max(self.syn_bytes, 1),), dtype=torch.uint8, device=device)
        cls = torch.empty((max(self.n, 1),), dtype=torch.uint8, device=device)
        _lib.check(_lib._lib().mcmc_plan_sample(self._h, int(seed) & ((1 << 64) - 1), _ptr(syn),
                                                _ptr(cls), _stream(syn.device)), "mcmc_plan_sample")
        return syn[:self.syn_bytes], cls[:self.n]

    def autotune(self, syndromes, cache_path=None):
        syndromes = self._check_input(syndromes)
        out = self._outputs(syndromes.device, False, True)
        res = _lib.Tuning()
        path = None if cache_path is None else str(cache_path).encode()
        _lib.check(_lib._lib().mcmc_plan_autotune(*self._args(syndromes, out), path,
                                                  ctypes.byref(res)), "mcmc_plan_autotune")
        return {k: getattr(res, k) for k, _ in _lib.Tuning._fields_}

    @property
    def tuning(self):
        t = _lib.Tuning()
        _lib.check(_lib._lib().mcmc_plan_get_tuning(self._h, ctypes.byref(t)), "mcmc_plan_get_tuning")
        return {k: getattr(t, k) for k, _ in _lib.Tuning._fields_}

    @tuning.setter
    def tuning(self, values):
        t = _lib.Tuning(**values)
        _lib.check(_lib._lib().mcmc_plan_set_tuning(self._h, ctypes.byref(t)), "mcmc_plan_set_tuning")
