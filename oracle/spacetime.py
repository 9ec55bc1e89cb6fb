"""Imperfect stabilizer measurements (Sec. VI): space-time hypotheses and
their Metropolis chains.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model.  Stabilizers are measured in rounds t = 0 .. T-1.  Before round t the
data qubits suffer the depolarizing error E_t (interval t); round t reports
s_t = syn(C_t) xor M_t, with C_t = E_0 E_1 ... E_t the accumulated error and
M_t the set of wrong measurement outcomes (each stabilizer outcome wrong with
probability p_M).  The last round is taken to be perfect (M_{T-1} = 0), so
that the hypotheses close in time and the logical class is that of C_{T-1}.
A hypothesis (E_0..E_{T-1}, M_0..M_{T-2}) with n data-qubit errors and m
wrong outcomes has relative probability ((p/3)/(1-p))^n (p_M/(1-p_M))^m =
exp(-beta_bar (n + xi m)), xi = log((1-p_M)/p_M) / beta_bar (Sec. VI).

Moves keep the observations and the class:
  spatial (t, k): apply stabilizer k to E_t (C_t .. C_{T-1} change by a
      stabilizer: no syndrome changes);
  time (t, q, P), t < T-1: apply the Pauli P (X or Z) to qubit q in E_t and
      in E_{t+1} (only C_t changes, by P) and toggle M_t on the stabilizers
      that anticommute with P on q (the plaquettes of q for X, its stars for
      Z), which keeps s_t (Sec. VI's deformation).
Delta n of a time move is the sum over the two intervals of the single-qubit
change, (1-z)(1-2x) for X and (1-x)(1-2z) for Z; Delta m is the sum over the
toggled outcomes of (1 - 2 M).  A move with E = Delta n + xi Delta m <= 0 is
taken; otherwise with probability exp(-beta E), as u < floor(2^32 exp(-beta E)).

Sweep (absolute index s): first every spatial move, t = 0..T-1 and k in site
order; then every time move, t = 0..T-2, q = 0..n_q-1, X before Z.  Move
(t, k) uses draw d = t n_stab + k, move (t, q, P) draw
d = T n_stab + 2 t (n_q + 1) + 2 q + (P==Z) (two draws per round are left
unused so that every round starts a Philox block: n_stab and 2 (n_q + 1) are
multiples of 4); draw d is word d & 3 of Philox at counter
(d >> 2, sweep, syndrome_id, 3<<30 | cls<<28 | 1<<20 | chain).
After the spatial half and after the time half of a counted sweep, n is added
to S_n and m to S_m.

Class starts (Sec. VI names none): every flipped outcome before the last
round is blamed on the measurement, M_t = s_t for t < T-1, with no data error
before the last interval, and E_{T-1} is the class-c matching start of the
perfect last round's syndrome s_{T-1} (the single-round decoder's start).
Each true data error is then relaxed back to its interval by time moves that
remove two wrong outcomes each, all downhill; explaining every syndrome
change by data strings instead (canonical strings per interval) leaves the
chains stuck far above the true energy at beta_bar.

Sampling: interval t's data errors use the depolarizing rule with counter
word 1 = 1 + t (the single-round sampler uses 0); round t's outcome k
(t < T-1) is wrong iff word k & 3 of Philox at (k >> 2, 0x80000000 | t,
sample_id, 1<<30) is below floor(p_M 2^32).

Estimator (single temperature, beta* = beta_bar, the decision rule of
Sec. IV.A with energy n + xi m): key_E = S_n + xi S_m (float64, this order);
the class with the smallest key wins (ties to the lowest class).  Class
probabilities by Eq. (main) with the trapezoid on [0, beta_bar]:
log Z_E = const - (beta_bar / 2)(f0 + key_E / (chains * 2 * sweeps)), where
f0 = 3/4 n_q T + xi n_stab (T - 1) / 2 is <n + xi m> at beta = 0 (every data
part and every outcome bit is uniform there).  With no counted sweep the
chains' final n + xi m stands in for the mean.
"""

import math

import numpy as np

from . import geometry, init, philox, tables
from .chains import apply_site, delta_n

DOMAIN_SPACETIME = 3


def xi_of(p, p_m):
    if not (0.0 < p_m < 0.5):
        raise ValueError("measurement error rate must satisfy 0 < p_M < 0.5")
    return math.log((1.0 - p_m) / p_m) / tables.beta_bar(p)


def time_table(beta, xi):
    """(thr [5, 5] uint32, always [5, 5] bool) indexed by (dn + 2, dm + 2)."""
    thr = np.zeros((5, 5), dtype=np.uint32)
    always = np.zeros((5, 5), dtype=bool)
    for dn in range(-2, 3):
        for dm in range(-2, 3):
            e = float(dn) + xi * float(dm)
            if e <= 0.0:
                always[dn + 2, dm + 2] = True
            else:
                thr[dn + 2, dm + 2] = int(math.floor(math.ldexp(math.exp(-(beta * e)), 32)))
    return thr, always


def anticommuting(lat):
    """Per qubit: (plaquettes containing it, stars containing it)."""
    plaq = [[] for _ in range(lat.n_qubits)]
    star = [[] for _ in range(lat.n_qubits)]
    for s in range(lat.n_stab):
        for q in lat.supports[s]:
            (star if lat.site_is_star[s] else plaq)[q].append(s)
    return plaq, star


def sample(lat, p, p_m, T, seed, sample_ids):
    """(observed [n, T, n_stab] uint8, true_class [n], E [n, T, n_q], M [n, T, n_stab])."""
    ids = np.asarray(sample_ids, dtype=np.uint64)
    n = ids.size
    k0, k1 = philox.seed_key(seed)
    q = np.arange(lat.n_qubits, dtype=np.uint64)
    E = np.zeros((n, T, lat.n_qubits), dtype=np.uint8)
    thr_d = np.uint64(tables.error_threshold(p))
    code = np.array([1, 3, 2], dtype=np.uint8)
    for t in range(T):
        w = np.stack(philox.philox4x32_10(q[None, :] >> np.uint64(1), 1 + t, ids[:, None],
                                          philox.sampler_ctr3(), k0, k1), -1).astype(np.uint64)
        half = (q & np.uint64(1)).astype(np.int64) * 2
        u0 = np.take_along_axis(w, half[None, :, None], axis=-1)[..., 0]
        u1 = np.take_along_axis(w, half[None, :, None] + 1, axis=-1)[..., 0]
        typ = ((u1 * np.uint64(3)) >> np.uint64(32)).astype(np.int64)
        E[:, t] = np.where(u0 < thr_d, code[typ], 0)
    M = np.zeros((n, T, lat.n_stab), dtype=np.uint8)
    thr_m = np.uint64(int(math.floor(math.ldexp(float(p_m), 32))))
    k = np.arange(lat.n_stab, dtype=np.uint64)
    for t in range(T - 1):
        w = np.stack(philox.philox4x32_10(k[None, :] >> np.uint64(2),
                                          np.uint64(0x80000000 | t), ids[:, None],
                                          philox.sampler_ctr3(), k0, k1), -1).astype(np.uint64)
        u = np.take_along_axis(w, (k & np.uint64(3)).astype(np.int64)[None, :, None], -1)[..., 0]
        M[:, t] = (u < thr_m).astype(np.uint8)
    C = np.bitwise_xor.accumulate(E, axis=1)
    obs = geometry.syndrome(lat, C) ^ M
    return obs, geometry.class_index(lat, C[:, T - 1]), E, M


def observations(lat, E, M):
    """Observed syndromes of hypotheses E [..., T, n_q], M [..., T, n_stab]."""
    C = np.bitwise_xor.accumulate(E, axis=-2)
    return geometry.syndrome(lat, C) ^ M


def hyp_class(lat, E):
    return geometry.class_index(lat, np.bitwise_xor.reduce(E, axis=-2))


def starts(lat, obs):
    """Class starts of one observation history [T, n_stab]: (E [4, T, n_q],
    M [4, T, n_stab])."""
    T = obs.shape[0]
    E = np.zeros((4, T, lat.n_qubits), dtype=np.uint8)
    E[:, T - 1] = init.matching_representatives(lat, obs[T - 1])
    M = np.zeros((4, T, lat.n_stab), dtype=np.uint8)
    M[:, :T - 1] = obs[:T - 1]
    return E, M


def run(lat, E, M, syndrome_id, cls, chain, beta, xi, seed, sweep_begin, sweep_end, burn,
        n=None, m=None, Sn=None, Sm=None, A=None, check_invariants=False, obs=None):
    """Advance chains (rows of E [C, T, n_q], M [C, T, n_stab]) over absolute
    sweeps [sweep_begin, sweep_end).  Returns dict(E, M, n, m, Sn, Sm, A)."""
    E = np.array(E, dtype=np.uint8, copy=True)
    M = np.array(M, dtype=np.uint8, copy=True)
    C, T = E.shape[0], E.shape[1]
    rows = np.arange(C)
    sid = np.asarray(syndrome_id, dtype=np.uint64).reshape(C)
    ctr3 = philox.chain_ctr3(np.asarray(cls).reshape(C), np.ones(C),
                             np.asarray(chain).reshape(C), DOMAIN_SPACETIME)
    k0, k1 = philox.seed_key(seed)
    sp_thr = tables.acceptance_table(beta).astype(np.uint64)
    t_thr, t_always = time_table(beta, xi)
    plaq_of, star_of = anticommuting(lat)
    n = geometry.weight(E).sum(axis=1).astype(np.int64) if n is None else np.array(n, np.int64)
    m = M.sum(axis=(1, 2)).astype(np.int64) if m is None else np.array(m, np.int64)
    Sn = np.zeros(C, np.int64) if Sn is None else np.array(Sn, np.int64)
    Sm = np.zeros(C, np.int64) if Sm is None else np.array(Sm, np.int64)
    A = np.zeros(C, np.int64) if A is None else np.array(A, np.int64)
    n_draws = T * lat.n_stab + 2 * (T - 1) * (lat.n_qubits + 1)
    if check_invariants:
        cls_arr = np.asarray(cls).reshape(C)
        obs = np.broadcast_to(obs, (C,) + obs.shape[-2:])

    def words(sweep):
        blocks = np.arange((n_draws + 3) // 4, dtype=np.uint64)
        w = philox.philox4x32_10(blocks[None, :], np.uint64(sweep), sid[:, None], ctr3[:, None],
                                 k0, k1)
        return np.stack(w, -1).astype(np.uint64).reshape(C, -1)

    for sweep in range(sweep_begin, sweep_end):
        u = words(sweep)
        for t in range(T):
            Et = E[:, t, :]
            for k in range(lat.n_stab):
                dn = delta_n(lat, Et, k)
                acc = (dn <= 0) | (u[:, t * lat.n_stab + k] < sp_thr[np.clip(dn, 1, 4) - 1])
                apply_site(lat, Et, k, acc)
                n += np.where(acc, dn, 0)
                A += acc
            E[:, t, :] = Et
        if sweep >= burn:
            Sn += n
            Sm += m
        for t in range(T - 1):
            for q in range(lat.n_qubits):
                for kind in (0, 1):              # 0: X (x part, plaquettes), 1: Z
                    d = T * lat.n_stab + 2 * t * (lat.n_qubits + 1) + 2 * q + kind
                    dn = np.zeros(C, np.int64)
                    for tt in (t, t + 1):
                        c = E[:, tt, q].astype(np.int64)
                        x, z = c & 1, c >> 1
                        dn += (1 - z) * (1 - 2 * x) if kind == 0 else (1 - x) * (1 - 2 * z)
                    stabs = plaq_of[q] if kind == 0 else star_of[q]
                    dm = np.zeros(C, np.int64)
                    for a in stabs:
                        dm += 1 - 2 * M[:, t, a].astype(np.int64)
                    acc = t_always[dn + 2, dm + 2] | \
                        (u[:, d] < t_thr[dn + 2, dm + 2].astype(np.uint64))
                    bit = np.uint8(1 if kind == 0 else 2)
                    E[acc, t, q] ^= bit
                    E[acc, t + 1, q] ^= bit
                    for a in stabs:
                        M[acc, t, a] ^= np.uint8(1)
                    n += np.where(acc, dn, 0)
                    m += np.where(acc, dm, 0)
                    A += acc
        if sweep >= burn:
            Sn += n
            Sm += m
        if check_invariants:
            assert np.array_equal(observations(lat, E, M), obs), "observations changed"
            assert np.array_equal(hyp_class(lat, E), cls_arr), "class changed"
            assert np.array_equal(geometry.weight(E).sum(axis=1), n), "n != recount"
            assert np.array_equal(M.sum(axis=(1, 2)), m), "m != recount"
            assert not M[:, T - 1].any(), "last round must stay perfect"
    return dict(E=E, M=M, n=n, m=m, Sn=Sn, Sm=Sm, A=A)


def estimate(Sn, Sm, n_final, m_final, chains, sweeps, beta_bar, xi, n_q, n_stab, T):
    """Sn, Sm, n_final, m_final: int64 [4, chains] of one observation history.
    Returns (class_prob [4], mean_n [4], mean_m [4], key [4] float, chosen)."""
    Sn, Sm = np.asarray(Sn, np.int64), np.asarray(Sm, np.int64)
    counted = sweeps > 0
    an = Sn.sum(axis=1) if counted else np.asarray(n_final, np.int64).sum(axis=1)
    am = Sm.sum(axis=1) if counted else np.asarray(m_final, np.int64).sum(axis=1)
    denom = float(chains * 2 * sweeps) if counted else float(chains)
    key = [float(an[e]) + xi * float(am[e]) for e in range(4)]
    f0 = 0.75 * n_q * T + xi * (0.5 * n_stab * (T - 1))
    logz = [-((beta_bar / 2.0) * (f0 + key[e] / denom)) for e in range(4)]
    mx = max(logz)
    ex = [math.exp(v - mx) for v in logz]
    tot = ((ex[0] + ex[1]) + ex[2]) + ex[3]
    prob = np.array([v / tot for v in ex])
    chosen = min(range(4), key=lambda e: (key[e], e))
    return (prob, np.array([float(an[e]) / denom for e in range(4)]),
            np.array([float(am[e]) / denom for e in range(4)]), np.array(key), chosen)


def decode(L, obs, p, p_m, sweeps, seed, chains_per_class=1, burn=0, syndrome_ids=None,
           check_invariants=False):
    """Decode observation histories obs [n, T, n_stab].  Returns class_prob,
    mean_n, mean_m, key, chosen, sum_n, sum_m, accepts, n_final, m_final
    ([n, 4, chains]) and correction (C_{T-1} of chain 0 of the chosen class)."""
    lat = geometry.Lattice(L)
    obs = (np.asarray(obs, dtype=np.uint8) != 0).astype(np.uint8)
    n, T = obs.shape[0], obs.shape[1]
    ids = np.arange(n, dtype=np.uint64) if syndrome_ids is None else \
        np.asarray(syndrome_ids, dtype=np.uint64)
    Cc = int(chains_per_class)
    bb = tables.beta_bar(p)
    xi = xi_of(p, p_m)
    out = {k: [] for k in ("class_prob", "mean_n", "mean_m", "key", "chosen", "sum_n", "sum_m",
                           "accepts", "n_final", "m_final", "correction")}
    for i in range(n):
        E0, M0 = starts(lat, obs[i])
        ci = np.repeat(np.arange(4), Cc)
        hi = np.tile(np.arange(Cc), 4)
        res = run(lat, E0[ci], M0[ci], np.full(4 * Cc, ids[i]), ci, hi, bb, xi, seed, 0,
                  burn + sweeps, burn, check_invariants=check_invariants, obs=obs[i])
        shape = (4, Cc)
        pr, mn, mm, key, ch = estimate(res["Sn"].reshape(shape), res["Sm"].reshape(shape),
                                       res["n"].reshape(shape), res["m"].reshape(shape), Cc,
                                       sweeps, bb, xi, lat.n_qubits, lat.n_stab, T)
        for k, v in (("class_prob", pr), ("mean_n", mn), ("mean_m", mm), ("key", key),
                     ("chosen", ch), ("sum_n", res["Sn"].reshape(shape)),
                     ("sum_m", res["Sm"].reshape(shape)), ("accepts", res["A"].reshape(shape)),
                     ("n_final", res["n"].reshape(shape)), ("m_final", res["m"].reshape(shape))):
            out[k].append(v)
        out["correction"].append(np.bitwise_xor.reduce(res["E"][ch * Cc], axis=0))
    return {k: np.array(v) for k, v in out.items()}
