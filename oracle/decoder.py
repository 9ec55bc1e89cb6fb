"""The whole decode of a batch of syndromes (Sec. IV.A), composed from the
oracle's steps: representatives per class -> Metropolis chains per
(class, temperature, chain) -> estimator and decision -> correction.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The correction is the final configuration of chain 0 of the chosen class at
the highest inverse temperature (any member of a class is an equally valid
correction, Sec. II).
"""

import numpy as np

from . import chains, estimator, geometry, init, matching, tables


INIT_CANONICAL = 0
INIT_MATCHING = 1
INIT_MWPM = 2       # exact minimum-weight matching per type and parity (Sec. III)
SCAN_COLOUR = 0      # colour-phased systematic sweeps (Sec. V's grouping)
SCAN_RANDOM = 1      # one uniformly random stabilizer per step (Sec. IV)


def decode(L, syndromes, p, sweeps, seed, chains_per_class=1, n_temps=1, burn=0,
           syndrome_ids=None, trace=False, check_invariants=False, init_mode=INIT_MATCHING,
           noise=tables.DEPOLARIZING, beta_scale=None, scan=SCAN_COLOUR):
    """noise: tables.DEPOLARIZING (p = depolarizing rate) or tables.BITPHASE
    (p = flip rate q of each part); beta_scale: beta*/beta_bar for K = 1
    (None = the model's default); scan: SCAN_COLOUR or SCAN_RANDOM (no
    trace)."""
    if scan == SCAN_RANDOM and trace:
        raise ValueError("the random scan keeps no trace")
    lat = geometry.Lattice(L)
    syn = np.asarray(syndromes, dtype=np.uint8).reshape(-1, lat.n_stab)
    syn = (syn != 0).astype(np.uint8)
    n = syn.shape[0]
    ids = np.arange(n, dtype=np.uint64) if syndrome_ids is None else \
        np.asarray(syndrome_ids, dtype=np.uint64)
    K, C = int(n_temps), int(chains_per_class)
    if K != 1 and K % 2 != 0:
        raise ValueError("n_temps must be 1 or even")
    tab = tables.tables(p, K, noise, beta_scale)              # [K, 4]
    start = {INIT_CANONICAL: init.representatives, INIT_MATCHING: init.matching_representatives,
             INIT_MWPM: matching.mwpm_representatives}[init_mode]
    reps = np.stack([start(lat, syn[i]) for i in range(n)]) \
        if n else np.zeros((0, 4, lat.n_qubits), np.uint8)

    # task order: ((syndrome * 4 + class) * K + (k - 1)) * chains + chain
    si, ci, ki, hi = np.meshgrid(np.arange(n), np.arange(4), np.arange(K), np.arange(C),
                                 indexing="ij")
    si, ci, ki, hi = (a.reshape(-1) for a in (si, ci, ki, hi))
    state0 = reps[si, ci] if n else np.zeros((0, lat.n_qubits), np.uint8)
    if scan == SCAN_RANDOM:
        res = chains.run_random(lat, state0, ids[si] if n else ids, ci, ki + 1, hi, tab[ki],
                                seed, 0, burn + sweeps, burn,
                                check_invariants=check_invariants,
                                syndromes=syn[si] if n else None, noise=noise)
    else:
        res = chains.run(lat, state0, ids[si] if n else ids, ci, ki + 1, hi, tab[ki], seed,
                         0, burn + sweeps, burn, trace=trace,
                         check_invariants=check_invariants,
                         syndromes=syn[si] if n else None, noise=noise)

    shape = (n, 4, K, C)
    S = res["S"].reshape(shape)
    A = res["A"].reshape(shape)
    nf = res["n"].reshape(shape)
    states = res["state"].reshape(shape + (lat.n_qubits,))
    bb = tables.beta_bar(p, noise)
    bs = tables.ladder(p, K, noise, beta_scale)[0] if K == 1 else bb
    prob = np.zeros((n, 4))
    mean = np.zeros((n, 4))
    key = np.zeros((n, 4), dtype=np.int64)
    chosen = np.zeros(n, dtype=np.int64)
    for i in range(n):
        prob[i], mean[i], key[i], chosen[i] = estimator.estimate(
            S[i], nf[i], C, sweeps, bb, lat.n_qubits, lat.n_stab, noise, bs,
            lat.n_stab if scan == SCAN_RANDOM else 4)
    correction = states[np.arange(n), chosen, K - 1, 0] if n else \
        np.zeros((0, lat.n_qubits), np.uint8)
    out = dict(class_prob=prob, mean_n=mean, sum_n=S, accepts=A, n_final=nf, key=key,
               chosen=chosen, correction=correction, states=states, init=reps)
    if trace:
        out["trace"] = res["trace"].reshape(shape + (-1,))
    return out
