"""Colour-phased Metropolis chains over one class's stabilizer-equivalent
configurations (Sec. IV, Sec. IV.A, Sec. V).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A move applies one stabilizer to the configuration (Sec. IV): a star flips the
x part of its 3-4 qubits, a plaquette the z part.  Moves never change the
syndrome or the class.  Delta n, the change in the number of non-identity
qubits, is a sum over the support of
    star:      (1 - z)(1 - 2x)      (a qubit with a z part stays non-identity)
    plaquette: (1 - x)(1 - 2z)
The move is taken if Delta n <= 0, else with probability exp(-beta Delta n),
realised as u < A[Delta n] with u a uniform 32-bit Philox word.

Under independent bit/phase-flip noise (noise = 1) the energy is m, the
number of x parts plus the number of z parts, and a move flips one part per
qubit of its support, so
    star:      Delta m = sum (1 - 2x)
    plaquette: Delta m = sum (1 - 2z)
with the same acceptance rule.

Scan order (the paper draws a random stabilizer per step; its parallel version,
Sec. V, probes one stabilizer in every region of group i mod 4 at step i): one
sweep visits colour 0, 1, 2, 3 in turn and, within a colour, every site once in
ascending site index.  Sites of one colour share no qubit, so the order within
a colour does not change the result; each single-site Metropolis update leaves
exp(-beta n) invariant, so the whole sweep does too.

Sampling (Sec. IV: sum n over the steps; Sec. V: per group step): after every
colour phase of a counted sweep (absolute sweep index >= burn) the current n is
added to S.  A counts every accepted move of the call (burn-in included).

Randomness: draw d of a sweep (d = colour * L(L-1)/2 + rank of the site within
its colour) is word d & 3 of Philox4x32-10 at counter
(d >> 2, sweep, syndrome_id, cls << 28 | temp << 20 | chain).
"""

import numpy as np

from . import geometry, philox


def delta_n(lat, state, s, noise=0):
    """int64 [T]: change in energy if site s were applied to each row of
    `state` (uint8 [T, n_q])."""
    codes = state[:, lat.supports[s]].astype(np.int64)
    x, z = codes & 1, codes >> 1
    if noise == 1:
        part = x if lat.site_is_star[s] else z
        return (1 - 2 * part).sum(axis=1)
    if lat.site_is_star[s]:
        return ((1 - z) * (1 - 2 * x)).sum(axis=1)
    return ((1 - x) * (1 - 2 * z)).sum(axis=1)


def apply_site(lat, state, s, mask):
    """Apply stabilizer s in place to the rows of `state` selected by `mask`."""
    flip = np.uint8(1) if lat.site_is_star[s] else np.uint8(2)
    for q in lat.supports[s]:
        state[mask, q] ^= flip


def _sweep_uniforms(lat, sweep, sid, ctr3, k0, k1):
    """uint64 [T, n_stab] uniforms of one sweep, indexed by draw number."""
    blocks = np.arange(lat.n_stab // 4, dtype=np.uint64)
    w = philox.philox4x32_10(blocks[None, :], np.uint64(sweep), sid[:, None],
                             ctr3[:, None], k0, k1)
    w = np.stack(w, axis=-1).astype(np.uint64)       # [T, n_stab/4, 4]
    return w.reshape(w.shape[0], lat.n_stab)


def run(lat, state, syndrome_id, cls, temp, chain, table, seed,
        sweep_begin, sweep_end, burn, n=None, S=None, A=None,
        trace=False, check_invariants=False, syndromes=None, noise=0):
    """Advance T independent chains over absolute sweeps [sweep_begin, sweep_end).

    state      uint8 [T, n_q] Pauli codes (modified copy is returned)
    syndrome_id, cls, temp, chain   [T] logical coordinates of each chain
    table      uint32 [T, 4] acceptance thresholds A[1..4] of each chain
    n, S, A    carried-in energy / energy sum / accept count (None = fresh start)
    noise      0 depolarizing (energy = weight), 1 bit/phase flips (x + z parts)
    Returns dict(state, n, S, A, trace) with trace int64 [T, 4*(end-begin)]
    (n after every phase) when requested.
    """
    state = np.array(state, dtype=np.uint8, copy=True)
    T = state.shape[0]
    sid = np.asarray(syndrome_id, dtype=np.uint64).reshape(T)
    ctr3 = philox.chain_ctr3(np.asarray(cls).reshape(T), np.asarray(temp).reshape(T),
                             np.asarray(chain).reshape(T))
    k0, k1 = philox.seed_key(seed)
    thr = np.asarray(table, dtype=np.uint64).reshape(T, 4)
    n = geometry.energy(state, noise).astype(np.int64) if n is None else \
        np.array(n, dtype=np.int64)
    S = np.zeros(T, dtype=np.int64) if S is None else np.array(S, dtype=np.int64)
    A = np.zeros(T, dtype=np.int64) if A is None else np.array(A, dtype=np.int64)
    rows = np.arange(T)
    tr = []
    if check_invariants:
        cls_arr = np.asarray(cls).reshape(T)
        syn_ref = np.asarray(syndromes, dtype=np.uint8).reshape(T, lat.n_stab)

    for sweep in range(sweep_begin, sweep_end):
        u = _sweep_uniforms(lat, sweep, sid, ctr3, k0, k1)
        for phase in range(4):
            for s in lat.phase_sites[phase]:
                delta = delta_n(lat, state, s, noise)
                ud = u[:, lat.draw_index[s]]
                a_of_delta = thr[rows, np.clip(delta, 1, 4) - 1]
                accept = (delta <= 0) | (ud < a_of_delta)
                apply_site(lat, state, s, accept)
                n += np.where(accept, delta, 0)
                A += accept
            if sweep >= burn:
                S += n
            if trace:
                tr.append(n.copy())
            if check_invariants:
                assert np.array_equal(geometry.syndrome(lat, state), syn_ref), "syndrome changed"
                assert np.array_equal(geometry.class_index(lat, state), cls_arr), "class changed"
                assert np.array_equal(geometry.energy(state, noise), n), \
                    "incremental n != recount"

    out = dict(state=state, n=n, S=S, A=A)
    if trace:
        out["trace"] = (np.stack(tr, axis=1) if tr else np.zeros((T, 0), dtype=np.int64))
    return out


# ---------------------------------------------------------------------------
# Random scan (Sec. IV as written): every step picks one stabilizer uniformly
# at random among all n_stab and applies the Metropolis rule to it; the
# energy n is summed after every step.  A "sweep" is n_stab steps, so budgets
# compare with the colour-phased scan.  Step t of a sweep draws block t >> 1
# at counter (t >> 1, sweep, syndrome_id, 2<<30 | cls<<28 | temp<<20 | chain)
# and uses its words 2(t&1) (site: floor(u * n_stab / 2^32)) and 2(t&1)+1
# (acceptance).
# ---------------------------------------------------------------------------
def _padded_supports(lat):
    sup = np.full((lat.n_stab, 4), -1, dtype=np.int64)
    for s in range(lat.n_stab):
        sup[s, :len(lat.supports[s])] = lat.supports[s]
    return sup


def run_random(lat, state, syndrome_id, cls, temp, chain, table, seed,
               sweep_begin, sweep_end, burn, n=None, S=None, A=None,
               check_invariants=False, syndromes=None, noise=0):
    """Advance T independent random-scan chains over absolute sweeps
    [sweep_begin, sweep_end); arguments and result as `run` (no trace)."""
    state = np.array(state, dtype=np.uint8, copy=True)
    T = state.shape[0]
    sid = np.asarray(syndrome_id, dtype=np.uint64).reshape(T)
    ctr3 = philox.chain_ctr3(np.asarray(cls).reshape(T), np.asarray(temp).reshape(T),
                             np.asarray(chain).reshape(T), philox.DOMAIN_RANDOM_SCAN)
    k0, k1 = philox.seed_key(seed)
    thr = np.asarray(table, dtype=np.uint64).reshape(T, 4)
    n = geometry.energy(state, noise).astype(np.int64) if n is None else \
        np.array(n, dtype=np.int64)
    S = np.zeros(T, dtype=np.int64) if S is None else np.array(S, dtype=np.int64)
    A = np.zeros(T, dtype=np.int64) if A is None else np.array(A, dtype=np.int64)
    rows = np.arange(T)
    sup = _padded_supports(lat)
    is_star = lat.site_is_star
    n_stab = np.uint64(lat.n_stab)
    if check_invariants:
        cls_arr = np.asarray(cls).reshape(T)
        syn_ref = np.asarray(syndromes, dtype=np.uint8).reshape(T, lat.n_stab)

    for sweep in range(sweep_begin, sweep_end):
        blocks = np.arange(lat.n_stab // 2, dtype=np.uint64)
        w = philox.philox4x32_10(blocks[None, :], np.uint64(sweep), sid[:, None],
                                 ctr3[:, None], k0, k1)
        w = np.stack(w, axis=-1).astype(np.uint64)           # [T, n_stab/2, 4]
        for t in range(lat.n_stab):
            u_site = w[:, t >> 1, 2 * (t & 1)]
            u_acc = w[:, t >> 1, 2 * (t & 1) + 1]
            site = ((u_site * n_stab) >> np.uint64(32)).astype(np.int64)
            q = sup[site]                                       # [T, 4], -1 padded
            valid = q >= 0
            codes = np.where(valid, state[rows[:, None], np.where(valid, q, 0)], 0).astype(np.int64)
            x, z = codes & 1, codes >> 1
            star = is_star[site][:, None]
            if noise == 1:
                part = np.where(star, x, z)
                delta = np.where(valid, 1 - 2 * part, 0).sum(axis=1)
            else:
                other, own = np.where(star, z, x), np.where(star, x, z)
                delta = np.where(valid, (1 - other) * (1 - 2 * own), 0).sum(axis=1)
            accept = (delta <= 0) | (u_acc < thr[rows, np.clip(delta, 1, 4) - 1])
            flip = np.where(is_star[site], 1, 2).astype(np.uint8)
            for k in range(4):
                m = accept & valid[:, k]
                state[rows[m], q[m, k]] ^= flip[m]
            n += np.where(accept, delta, 0)
            A += accept
            if sweep >= burn:
                S += n
        if check_invariants:
            assert np.array_equal(geometry.syndrome(lat, state), syn_ref), "syndrome changed"
            assert np.array_equal(geometry.class_index(lat, state), cls_arr), "class changed"
            assert np.array_equal(geometry.energy(state, noise), n), "incremental n != recount"

    return dict(state=state, n=n, S=S, A=A)
