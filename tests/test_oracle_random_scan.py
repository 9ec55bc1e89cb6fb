"""Pins for the oracle's random-scan chains (Sec. IV: one stabilizer chosen
uniformly at random per Metropolis step, n summed after every step)."""

import math

import numpy as np
import pytest

from oracle import chains, decoder, estimator, geometry, init, philox, sampler, tables
from oracle import enumerate as en


def _tasks(lat, syn, C, p, noise=0):
    reps = init.representatives(lat, syn)
    ci, hi = np.meshgrid(np.arange(4), np.arange(C), indexing="ij")
    ci, hi = ci.ravel(), hi.ravel()
    tab = np.broadcast_to(tables.tables(p, 1, noise)[0], (ci.size, 4))
    return reps[ci], ci, np.ones_like(ci), hi, tab


def test_single_steps_follow_the_definition():
    """Replays the first sweep of one chain step by step with the scalar
    pieces (Philox call, site rule, delta_n and apply_site of the systematic
    oracle) and compares the state after every step count."""
    L, p, seed = 4, 0.12, 0xABC
    lat = geometry.Lattice(L)
    rng = np.random.default_rng(1)
    st0 = rng.integers(0, 4, size=(1, lat.n_qubits)).astype(np.uint8)
    thr = tables.tables(p, 1)[0]
    k0, k1 = philox.seed_key(seed)
    ctr3 = (2 << 30) | (3 << 28) | (1 << 20) | 5
    ref = st0.copy()
    n_ref = int(geometry.weight(ref)[0])
    S_ref = 0
    for t in range(lat.n_stab):
        w = [int(v) for v in philox.philox4x32_10(t >> 1, 0, 9, ctr3, k0, k1)]
        u_site, u_acc = w[2 * (t & 1)], w[2 * (t & 1) + 1]
        s = (u_site * lat.n_stab) >> 32
        d = int(chains.delta_n(lat, ref, s)[0])
        if d <= 0 or u_acc < int(thr[min(max(d, 1), 4) - 1]):
            chains.apply_site(lat, ref, s, np.array([True]))
            n_ref += d
        S_ref += n_ref
    res = chains.run_random(lat, st0, [9], [3], [1], [5], thr[None], seed, 0, 1, 0)
    assert np.array_equal(res["state"], ref)
    assert int(res["n"][0]) == n_ref == int(geometry.weight(ref)[0])
    assert int(res["S"][0]) == S_ref


def test_sites_are_uniform():
    """The site rule floor(u n_stab / 2^32) spreads steps evenly over the
    stabilizers (chi-square at 20 sweeps x 64 chains)."""
    L = 5
    lat = geometry.Lattice(L)
    k0, k1 = philox.seed_key(77)
    counts = np.zeros(lat.n_stab, dtype=np.int64)
    ctr3 = philox.chain_ctr3(np.zeros(64), np.ones(64), np.arange(64), philox.DOMAIN_RANDOM_SCAN)
    for sweep in range(20):
        blocks = np.arange(lat.n_stab // 2, dtype=np.uint64)
        w = np.stack(philox.philox4x32_10(blocks[None, :], sweep, 3, ctr3[:, None], k0, k1), -1)
        u = w[:, :, [0, 2]].astype(np.uint64).reshape(-1)
        counts += np.bincount(((u * np.uint64(lat.n_stab)) >> np.uint64(32)).astype(np.int64),
                              minlength=lat.n_stab)
    e = counts.sum() / lat.n_stab
    chi2 = ((counts - e) ** 2 / e).sum()
    dof = lat.n_stab - 1
    assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof)


@pytest.mark.parametrize("noise", [0, 1])
def test_invariants(noise):
    lat = geometry.Lattice(4)
    syn = sampler.sample(lat, 0.1, 5, [2], noise=noise)[0][0]
    st, ci, ki, hi, tab = _tasks(lat, syn, 2, 0.1, noise)
    T = st.shape[0]
    chains.run_random(lat, st, np.full(T, 2), ci, ki, hi, tab, 3, 0, 4, 1, check_invariants=True,
                      syndromes=np.broadcast_to(syn, (T, lat.n_stab)), noise=noise)


def test_zero_temperature_never_increases_weight():
    lat = geometry.Lattice(5)
    syn = sampler.sample(lat, 0.15, 3, [0])[0][0]
    st, ci, ki, hi, _ = _tasks(lat, syn, 4, 0.15)
    T = st.shape[0]
    w0 = geometry.weight(st)
    res = chains.run_random(lat, st, np.zeros(T), ci, ki, hi, np.zeros((T, 4), np.uint32), 1,
                            0, 10, 0)
    assert (res["n"] <= w0).all()
    assert (res["S"] <= w0 * 10 * lat.n_stab).all()


@pytest.mark.parametrize("noise,p", [(0, 0.10), (1, 0.08)])
def test_chain_mean_matches_enumeration(noise, p):
    """L = 3: the random-scan average of n over 1000 sweeps agrees with the
    exact <n>_{beta*,E} within statistical error, under both noise models."""
    L, C, sweeps, burn = 3, 8, 1000, 100
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, p, 0x1302266900000001, [4], noise=noise)[0][0]
    beta = tables.ladder(p, 1, noise)[0]
    exact = en.mean_n(en.class_histograms(lat, syn, noise=noise), beta)
    st, ci, ki, hi, tab = _tasks(lat, syn, C, p, noise)
    T = st.shape[0]
    res = chains.run_random(lat, st, np.full(T, 4), ci, ki, hi, tab, 0xBEEF, 0, burn + sweeps,
                            burn, noise=noise)
    per_chain = (res["S"] / (lat.n_stab * float(sweeps))).reshape(4, C)
    est = per_chain.mean(axis=1)
    se = per_chain.std(axis=1, ddof=1) / np.sqrt(C)
    assert (np.abs(est - exact) < 6 * se + 2e-3 * exact).all(), (est, exact, se)


def test_decoder_random_scan_estimator_denominator():
    """The random-scan decoder divides S by chains * n_stab * sweeps."""
    L = 3
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, 0.1, 1, np.arange(3))[0]
    out = decoder.decode(L, syn, 0.1, 7, 5, chains_per_class=2, scan=decoder.SCAN_RANDOM)
    S = out["sum_n"].sum(axis=3)[:, :, 0]
    assert np.allclose(out["mean_n"], S / (2 * lat.n_stab * 7), rtol=1e-15)
    with pytest.raises(ValueError):
        decoder.decode(L, syn, 0.1, 7, 5, scan=decoder.SCAN_RANDOM, trace=True)
    pr, mean, key, chosen = estimator.estimate(out["sum_n"][0], out["n_final"][0], 2, 7,
                                               tables.beta_bar(0.1), lat.n_qubits, lat.n_stab,
                                               samples_per_sweep=lat.n_stab)
    assert np.allclose(pr, out["class_prob"][0], rtol=0, atol=0) and chosen == out["chosen"][0]
