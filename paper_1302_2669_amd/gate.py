"""Learned gate in front of the Metropolis decoder (not part of the paper's
method): a small convolutional network over the syndrome planes that predicts
the four class probabilities and a sweep budget, trained by the library's own
forward/backward kernels on class probabilities the decoder itself produces.

Argument marshalling only: the network, its gradients, the optimizer, the
gate and the decodes run in libmcmcdec.so.  See the gate-network section of
include/mcmcdec.h for the layouts.
"""

import ctypes

import numpy as np

from . import _lib
from . import MCMC_INIT_MATCHING, MixedPlan, geometry, _ptr, _stream, _torch

BUDGET_NAMES = ("none", "short", "full")


def param_count(L):
    n = ctypes.c_int64()
    _lib.check(_lib._lib().mcmc_cnn_param_count(int(L), ctypes.byref(n)), "mcmc_cnn_param_count")
    return n.value


def workspace_size(L, batch):
    b = ctypes.c_size_t()
    _lib.check(_lib._lib().mcmc_cnn_workspace_size(int(L), int(batch), ctypes.byref(b)),
               "mcmc_cnn_workspace_size")
    return b.value


def workspace_offsets(L, batch):
    """Byte offsets of x0, a1, a2, a3, dpre3, dpre2, dpre1 in the workspace."""
    arr = (ctypes.c_int64 * 7)()
    _lib.check(_lib._lib().mcmc_cnn_workspace_offsets(int(L), int(batch), arr),
               "mcmc_cnn_workspace_offsets")
    return dict(zip(("x0", "a1", "a2", "a3", "dp3", "dp2", "dp1"), list(arr)))


def forward(L, params, syndromes, p, workspace=None):
    """logits [B][8] fp32 (entries 0..6 meaningful) and the workspace holding
    the activations."""
    torch = _torch()
    B = syndromes.shape[0]
    dev = syndromes.device
    if workspace is None:
        workspace = torch.empty((max(workspace_size(L, B), 1),), dtype=torch.uint8, device=dev)
    logits = torch.zeros((B, 8), dtype=torch.float32, device=dev)
    syndromes = syndromes.contiguous()
    p = p.to(dtype=torch.float32).contiguous()
    _lib.check(_lib._lib().mcmc_cnn_forward(int(L), B, _ptr(params), _ptr(syndromes), _ptr(p),
                                            _ptr(logits), _ptr(workspace), workspace.numel(),
                                            _stream(dev)), "mcmc_cnn_forward")
    return logits, workspace


def infer(L, params, syndromes, p, workspace=None):
    """logits [B][8] of the fused inference kernel (identical to forward's)."""
    torch = _torch()
    B = syndromes.shape[0]
    dev = syndromes.device
    if workspace is None:
        b = ctypes.c_size_t()
        _lib.check(_lib._lib().mcmc_cnn_infer_workspace_size(int(L), ctypes.byref(b)),
                   "mcmc_cnn_infer_workspace_size")
        workspace = torch.empty((max(b.value, 1),), dtype=torch.uint8, device=dev)
    logits = torch.zeros((B, 8), dtype=torch.float32, device=dev)
    syndromes = syndromes.contiguous()
    p = p.to(dtype=torch.float32).contiguous()
    _lib.check(_lib._lib().mcmc_cnn_infer(int(L), B, _ptr(params), _ptr(syndromes), _ptr(p),
                                          _ptr(logits), _ptr(workspace), workspace.numel(),
                                          _stream(dev)), "mcmc_cnn_infer")
    return logits, workspace


def backward(L, params, logits, class_target, budget, workspace, budget_weight=0.5,
             want_loss=True):
    """(grads [param_count] fp32, per-sample loss [B] or None) of the batch
    whose forward pass left its activations in `workspace`."""
    torch = _torch()
    B = logits.shape[0]
    dev = logits.device
    grads = torch.empty_like(params)
    loss = torch.empty((B,), dtype=torch.float32, device=dev) if want_loss else None
    tgt = class_target.to(dtype=torch.float32).contiguous()
    bud = budget.to(dtype=torch.int32).contiguous()
    _lib.check(_lib._lib().mcmc_cnn_backward(int(L), B, _ptr(params), _ptr(logits), _ptr(tgt),
                                             _ptr(bud), float(budget_weight), _ptr(grads),
                                             _ptr(loss), _ptr(workspace), workspace.numel(),
                                             _stream(dev)), "mcmc_cnn_backward")
    return grads, loss


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _lib.check(_lib._lib().mcmc_cnn_step(params.numel(), int(step), float(lr), float(beta1),
                                         float(beta2), float(eps), _ptr(params), _ptr(grads),
                                         _ptr(m), _ptr(v), _stream(params.device)),
               "mcmc_cnn_step")


def gate(logits, threshold=0.99, class_route=False):
    """(route [B] u8, class [B] u8, confidence [B][3] fp32): the route, the
    argmax class, and (q0, q0 + q1, c): the predicted probabilities that no
    sweep / at most the short budget reaches the full-budget decision, and
    the class head's largest softmax entry (with class_route, c >= threshold
    also gives route 0)."""
    torch = _torch()
    B = logits.shape[0]
    dev = logits.device
    route = torch.empty((B,), dtype=torch.uint8, device=dev)
    cls = torch.empty((B,), dtype=torch.uint8, device=dev)
    conf = torch.empty((B, 3), dtype=torch.float32, device=dev)
    _lib.check(_lib._lib().mcmc_cnn_gate(B, _ptr(logits.contiguous()), float(threshold),
                                         1 if class_route else 0, _ptr(route), _ptr(cls),
                                         _ptr(conf), _stream(dev)), "mcmc_cnn_gate")
    return route, cls, conf


GAP_BINS = 50
GAP_NEVER = 255


def fit_gap_table(p, weights, budget, max_miss, min_count=50):
    """uint8 [GAP_BINS] host array: the start-weight gap route's thresholds
    per rate bin (mcmc_gate_fit_gap_table), from host rates p [n], device
    class start weights [n][4] (start_weights) and budget labels [n]."""
    torch = _torch()
    n = len(p)
    h_p = np.ascontiguousarray(p, dtype=np.float64)
    table = np.zeros(GAP_BINS, dtype=np.uint8)
    w = weights.contiguous()
    b = budget.to(torch.int32).contiguous()
    _lib.check(_lib._lib().mcmc_gate_fit_gap_table(
        int(n), h_p.ctypes.data, _ptr(w), _ptr(b), float(max_miss), int(min_count),
        table.ctypes.data, _stream(w.device)), "mcmc_gate_fit_gap_table")
    return table


def init_params(L, seed, device="cuda"):
    """Initial parameters [param_count] fp32 on the device (mcmc_cnn_init:
    He-normal weights from the library's Philox stream, zero biases)."""
    torch = _torch()
    prm = torch.empty((param_count(L),), dtype=torch.float32, device=device)
    _lib.check(_lib._lib().mcmc_cnn_init(int(L), int(seed) & ((1 << 64) - 1), _ptr(prm),
                                         _stream(prm.device)), "mcmc_cnn_init")
    return prm


def permutation(n, seed, epoch, device="cuda"):
    """The keyed shuffle of one training epoch, int32 [n] on the device."""
    torch = _torch()
    perm = torch.empty((n,), dtype=torch.int32, device=device)
    _lib.check(_lib._lib().mcmc_cnn_permutation(int(n), int(seed) & ((1 << 64) - 1), int(epoch),
                                                _ptr(perm), _stream(perm.device)),
               "mcmc_cnn_permutation")
    return perm


def budget_labels(d_zero, d_short, d_full):
    """int32 [n]: 0 if the no-sweep decision equals the full one, else 1 if
    the short one does, else 2 (mcmc_gate_budget_labels)."""
    torch = _torch()
    n = d_full.shape[0]
    out = torch.empty((n,), dtype=torch.int32, device=d_full.device)
    _lib.check(_lib._lib().mcmc_gate_budget_labels(
        n, _ptr(d_zero.contiguous()), _ptr(d_short.contiguous()), _ptr(d_full.contiguous()),
        _ptr(out), _stream(d_full.device)), "mcmc_gate_budget_labels")
    return out


def relative_targets(start_class, class_prob):
    """float32 [n][4]: class probabilities read relative to each syndrome's
    start decision, out[i][k] = class_prob[i][k ^ start_class[i]]
    (mcmc_gate_relative_targets)."""
    torch = _torch()
    n = class_prob.shape[0]
    prob = class_prob.to(torch.float32).contiguous()
    out = torch.empty((n, 4), dtype=torch.float32, device=prob.device)
    _lib.check(_lib._lib().mcmc_gate_relative_targets(
        n, _ptr(start_class.to(torch.uint8).contiguous()), _ptr(prob), _ptr(out),
        _stream(prob.device)), "mcmc_gate_relative_targets")
    return out


class GateNet:
    """Parameters and Adam state of one network on the device; init_params is
    a host array or a device tensor of the initial parameters."""

    def __init__(self, L, init_params, device="cuda"):
        torch = _torch()
        self.L = int(L)
        if isinstance(init_params, torch.Tensor):
            if init_params.numel() != param_count(L):
                raise ValueError(f"expected {param_count(L)} parameters")
            self.params = init_params.detach().to(device=device, dtype=torch.float32).clone()
        else:
            init = np.asarray(init_params, dtype=np.float32)
            if init.size != param_count(L):
                raise ValueError(f"expected {param_count(L)} parameters, got {init.size}")
            self.params = torch.from_numpy(init.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        self._ws = None
        self._ws_batch = -1

    def _workspace(self, B, dev):
        torch = _torch()
        if self._ws is None or self._ws_batch < B or self._ws.device != dev:
            self._ws = torch.empty((max(workspace_size(self.L, B), 1),), dtype=torch.uint8,
                                   device=dev)
            self._ws_batch = B
        return self._ws

    def forward(self, syndromes, p):
        B = syndromes.shape[0]
        ws = self._workspace(B, syndromes.device)[:max(workspace_size(self.L, B), 1)]
        return forward(self.L, self.params, syndromes, p, ws)

    def train_step(self, syndromes, p, class_target, budget, lr=1e-3, budget_weight=0.5):
        logits, ws = self.forward(syndromes, p)
        grads, loss = backward(self.L, self.params, logits, class_target, budget, ws,
                               budget_weight)
        self.step_count += 1
        adam_step(self.params, grads, self.m, self.v, self.step_count, lr)
        return loss

    def predict(self, syndromes, p, threshold=0.99, batch=65536):
        """(class_prob [B][4] fp32 from the class logits, route, class)."""
        torch = _torch()
        outs = []
        for s in range(0, syndromes.shape[0], batch):
            logits, _ = self.forward(syndromes[s:s + batch], p[s:s + batch])
            route, cls, _ = gate(logits, threshold)
            outs.append((torch.softmax(logits[:, :4], dim=1), route, cls))
        return tuple(torch.cat([o[i] for o in outs]) for i in range(3))


def sample_dataset(L, p, seed, id_base=0, device="cuda"):
    """Depolarizing samples of distance L with per-sample rates p (host
    array): (syndromes [n][n_stab] u8, true classes [n] u8, ids [n]) on the
    device, sample ids id_base + i."""
    n = len(p)
    ids = (id_base + np.arange(n, dtype=np.int64)) & 0xFFFFFFFF
    plan = MixedPlan.from_arrays(L, p, 0, seed, syndrome_ids=ids)
    syn, cls = plan.sample(seed, device)
    plan.close()
    return syn.reshape(n, -1), cls, ids


def mcmc_labels(L, syndromes, p, ids, seed, sweeps_short=None, sweeps_full=None, chains=4,
                label_temps=20, label_chains=1, init=MCMC_INIT_MATCHING, relative=False):
    """Training targets made by the decoder itself, for n syndromes of
    distance L ([n][n_stab] device tensor), rates p (host float array) and ids
    (host int array):

    * class_target [n][4]: the class probabilities of thermodynamic
      integration over `label_temps` temperatures (Simpson's rule),
      `sweeps_full` sweeps, `label_chains` chains; with `relative`, read
      relative to the no-sweep decision (relative_targets);
    * budget [n]: the smallest of (0, sweeps_short, sweeps_full) counted
      sweeps whose decision (the plain decoder: one temperature, `chains`
      chains) equals the one at sweeps_full (0 sweeps: the decision from the
      class starts alone);
    * decision [n]: that full-budget decision.
    """
    torch = _torch()
    n = len(p)
    sweeps_short = L if sweeps_short is None else sweeps_short
    sweeps_full = L * L if sweeps_full is None else sweeps_full
    flat = syndromes.reshape(-1).contiguous()

    def run(sweeps, K, C):
        plan = MixedPlan.from_arrays(L, p, sweeps, seed, chains=C, n_temps=K, syndrome_ids=ids,
                                     init=init)
        out = plan.execute(flat, want_correction=False)
        plan.close()
        return out

    soft = run(sweeps_full, label_temps, label_chains)["class_prob"].to(torch.float32)
    d_full = run(sweeps_full, 1, chains)["chosen"]
    d_short = run(sweeps_short, 1, chains)["chosen"]
    d_zero = run(0, 1, chains)["chosen"]
    if relative:
        soft = relative_targets(d_zero, soft)
    return soft, budget_labels(d_zero, d_short, d_full), d_full


def train(net, syndromes, p, class_target, budget, epochs=2, batch=512, lr=1e-3, seed=0,
          budget_weight=0.5, lr_final=None, log=None):
    """Adam over shuffled mini-batches, one mcmc_cnn_train_epoch call per
    epoch (the last partial batch of an epoch is dropped); the learning rate
    falls linearly from lr to lr_final (lr/10 by default) over the run.
    Returns the mean loss of each epoch."""
    torch = _torch()
    n = syndromes.shape[0]
    dev = syndromes.device
    L = net.L
    cfg = _lib.TrainConfig(lr=float(lr), lr_final=float(lr / 10.0 if lr_final is None else lr_final),
                           beta1=0.9, beta2=0.999, eps=1e-8, budget_weight=float(budget_weight),
                           batch=int(batch), total_steps=max(1, epochs * (n // batch)),
                           seed=int(seed) & ((1 << 64) - 1))
    b = ctypes.c_size_t()
    _lib.check(_lib._lib().mcmc_cnn_train_workspace_size(L, n, int(batch), ctypes.byref(b)),
               "mcmc_cnn_train_workspace_size")
    ws = torch.empty((max(b.value, 1),), dtype=torch.uint8, device=dev)
    syn = syndromes.contiguous()
    pp = p.to(device=dev, dtype=torch.float32).contiguous()
    tgt = class_target.to(device=dev, dtype=torch.float32).contiguous()
    bud = budget.to(device=dev, dtype=torch.int32).contiguous()
    loss_sum = torch.zeros((1,), dtype=torch.float64, device=dev)
    step = ctypes.c_int64(net.step_count)
    history = []
    for e in range(epochs):
        _lib.check(_lib._lib().mcmc_cnn_train_epoch(
            L, n, ctypes.byref(cfg), e, ctypes.byref(step), _ptr(net.params), _ptr(net.m),
            _ptr(net.v), _ptr(syn), _ptr(pp), _ptr(tgt), _ptr(bud), _ptr(loss_sum), _ptr(ws),
            ws.numel(), _stream(dev)), "mcmc_cnn_train_epoch")
        history.append(float(loss_sum.item()) / max(1, (n // batch) * batch))
        if log:
            log(f"epoch {e}: mean loss {history[-1]:.4f}")
    net.step_count = step.value
    return history


class GatedDecoder:
    """The gated decoder of include/mcmcdec.h (mcmc_gated_*)."""

    def __init__(self, L, p, seed, max_batch, sweeps_short=None, sweeps_full=None, chains=4,
                 n_temps=1, burn=0, threshold=0.99, escalate=0.0, init=MCMC_INIT_MATCHING,
                 class_route=False, gap_table=None, device="cuda"):
        torch = _torch()
        cfg = _lib.GateConfig()
        cfg.L = int(L)
        cfg.n_temps = int(n_temps)
        cfg.chains = int(chains)
        cfg.burn = int(burn)
        cfg.sweeps_short = int(L if sweeps_short is None else sweeps_short)
        cfg.sweeps_full = int(L * L if sweeps_full is None else sweeps_full)
        cfg.p = float(p)
        cfg.seed = int(seed) & ((1 << 64) - 1)
        cfg.init = int(init)
        cfg.threshold = float(threshold)
        cfg.escalate = float(escalate)
        cfg.max_batch = int(max_batch)
        cfg.class_route = 1 if class_route else 0
        self.cfg = cfg
        self.L = int(L)
        self.nq, self.ns = geometry(L)
        h = ctypes.c_void_p()
        _lib.check(_lib._lib().mcmc_gated_create(ctypes.byref(cfg), ctypes.byref(h)),
                   "mcmc_gated_create")
        self._h = h
        b = ctypes.c_size_t()
        _lib.check(_lib._lib().mcmc_gated_workspace_size(h, ctypes.byref(b)),
                   "mcmc_gated_workspace_size")
        self.workspace = torch.empty((max(b.value, 1),), dtype=torch.uint8, device=device)
        self.set_gap_table(gap_table)

    def set_gap_table(self, table):
        """The start-weight gap route's thresholds (uint8 [GAP_BINS]), or None
        to switch the route off (mcmc_gated_set_gap_table)."""
        if table is None:
            _lib.check(_lib._lib().mcmc_gated_set_gap_table(self._h, None),
                       "mcmc_gated_set_gap_table")
            self.gap_table = None
            return
        t = np.ascontiguousarray(table, dtype=np.uint8)
        if t.shape != (GAP_BINS,):
            raise ValueError(f"gap table needs {GAP_BINS} entries")
        _lib.check(_lib._lib().mcmc_gated_set_gap_table(self._h, t.ctypes.data),
                   "mcmc_gated_set_gap_table")
        self.gap_table = t

    def close(self):
        if getattr(self, "_h", None):
            _lib._lib().mcmc_gated_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def decode(self, params, syndromes, p=None, ids=None, want_correction=False):
        """dict with chosen [n], route [n] (0 none, 1 short, 2 full, 3 short
        then full), logits [n][8], counts (4 ints, per route) and optionally
        correction [n][n_q]."""
        torch = _torch()
        n = syndromes.shape[0]
        dev = syndromes.device
        syndromes = syndromes.contiguous()
        chosen = torch.empty((n,), dtype=torch.uint8, device=dev)
        route = torch.empty((n,), dtype=torch.uint8, device=dev)
        logits = torch.zeros((n, 8), dtype=torch.float32, device=dev)
        corr = torch.empty((n, self.nq), dtype=torch.uint8, device=dev) if want_correction \
            else None
        h_p = None if p is None else np.ascontiguousarray(p, dtype=np.float64)
        h_ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
        counts = (ctypes.c_int64 * 4)()
        _lib.check(_lib._lib().mcmc_gated_decode(
            self._h, _ptr(params), _ptr(syndromes),
            None if h_ids is None else h_ids.ctypes.data_as(ctypes.c_void_p),
            None if h_p is None else h_p.ctypes.data_as(ctypes.c_void_p), n, _ptr(chosen),
            _ptr(route), _ptr(logits), _ptr(corr), counts, _ptr(self.workspace),
            self.workspace.numel(), _stream(dev)), "mcmc_gated_decode")
        out = dict(chosen=chosen, route=route, logits=logits, counts=list(counts))
        if corr is not None:
            out["correction"] = corr
        return out
