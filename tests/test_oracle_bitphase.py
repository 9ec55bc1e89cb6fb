"""Pins for the oracle's independent bit/phase-flip model (Eq. pauliChannel
with p_b = p_p = q; Sec. IV.A's last paragraph).

Each check reaches the model from a different side than the oracle code
does: the channel's own Pauli probabilities, recounts of flipped parts,
exhaustive enumeration of all errors, exact partition functions and
closed-form integrals."""

import math

import numpy as np
import pytest

from oracle import chains, decoder, estimator, geometry, init, sampler, tables
from oracle import enumerate as en

BP = tables.BITPHASE


def _channel(q):
    """(p_I, p_x, p_y, p_z) of Eq. pauliChannel for independent flips."""
    return ((1 - q) * (1 - q), q * (1 - q), q * q, (1 - q) * q)


@pytest.mark.parametrize("q", [0.02, 0.08, 0.1, 0.3, 0.49])
def test_beta_bar_from_the_channel(q):
    """Probability ratios of whole error configurations under the channel
    equal exp(-beta_bar * difference in flip count)."""
    rng = np.random.default_rng(7)
    pI, px, py, pz = _channel(q)
    logp = np.log(np.array([pI, px, pz, py]))        # by Pauli code 0, 1, 2, 3
    bb = tables.beta_bar(q, BP)
    for _ in range(20):
        e1, e2 = rng.integers(0, 4, size=(2, 13))
        lr = logp[e1].sum() - logp[e2].sum()
        m1, m2 = geometry.flip_count(e1), geometry.flip_count(e2)
        assert lr == pytest.approx(-bb * (m1 - m2), rel=1e-12, abs=1e-12)


def test_flip_count_per_code():
    assert geometry.flip_count(np.array([0, 1, 2, 3])[:, None]).tolist() == [0, 1, 1, 2]
    assert geometry.energy(np.array([[3, 3, 1]]), BP)[0] == 5
    assert geometry.energy(np.array([[3, 3, 1]]), tables.DEPOLARIZING)[0] == 3


def test_rate_range_and_ladder():
    with pytest.raises(ValueError):
        tables.beta_bar(0.5, BP)
    with pytest.raises(ValueError):
        tables.beta_bar(0.0, BP)
    assert tables.beta_bar(1.0 / (1.0 + math.e), BP) == pytest.approx(1.0, rel=1e-14)
    assert tables.ladder(0.1, 1, BP) == [0.85 * math.log(9.0)]
    assert tables.ladder(0.1, 1, BP, 1.0) == [math.log(9.0)]
    assert tables.ladder(0.1, 4, BP)[-1] == pytest.approx(math.log(9.0), rel=1e-15)
    with pytest.raises(ValueError):
        tables.ladder(0.1, 4, BP, 0.85)


@pytest.mark.parametrize("L", [3, 5])
def test_delta_matches_recount(L):
    """Delta m of every site equals the change of a full recount of x and z
    parts after the stabilizer is applied."""
    lat = geometry.Lattice(L)
    rng = np.random.default_rng(L)
    st = rng.integers(0, 4, size=(64, lat.n_qubits)).astype(np.uint8)
    for s in range(lat.n_stab):
        d = chains.delta_n(lat, st, s, BP)
        after = st.copy()
        chains.apply_site(lat, after, s, np.ones(64, bool))
        assert np.array_equal(d, geometry.flip_count(after) - geometry.flip_count(st))
        assert d.min() >= -4 and d.max() <= 4


def test_sampler_rates_and_independence():
    """x and z parts are each set with rate q and independently: the four
    Pauli frequencies match the channel within 5 standard errors."""
    q, L = 0.1, 5
    lat = geometry.Lattice(L)
    e = sampler.sample_errors(lat, q, 0x5EED, np.arange(4000), noise=BP).reshape(-1)
    n = e.size
    want = dict(zip((0, 1, 3, 2), _channel(q)))
    for code, pr in want.items():
        f = (e == code).mean()
        assert abs(f - pr) < 5 * math.sqrt(pr * (1 - pr) / n), (code, f, pr)


def test_sampled_syndrome_and_class_consistent():
    lat = geometry.Lattice(5)
    syn, cls, e = sampler.sample(lat, 0.1, 3, np.arange(50), noise=BP)
    assert np.array_equal(syn, geometry.syndrome(lat, e))
    assert np.array_equal(cls, geometry.class_index(lat, e))
    for i in range(50):
        reps = init.representatives(lat, syn[i])
        assert np.array_equal(geometry.syndrome(lat, reps), np.broadcast_to(syn[i], (4, lat.n_stab)))


@pytest.mark.parametrize("L", [2, 3])
def test_enumeration_routes_agree(L):
    """Class histograms from representatives times stabilizer span equal those
    of running over every one of the 4^n_q errors (L = 2) / a sample of
    syndromes (L = 3 uses the span route only, checked against its total)."""
    lat = geometry.Lattice(L)
    if L == 2:
        brute = en.brute_force_histograms(lat, noise=BP)
        for idx in range(1 << lat.n_stab):
            syn = np.array([(idx >> s) & 1 for s in range(lat.n_stab)], np.uint8)
            assert np.array_equal(en.class_histograms(lat, syn, noise=BP), brute[idx])
    else:
        syn = sampler.sample(lat, 0.1, 9, [1], noise=BP)[0][0]
        h = en.class_histograms(lat, syn, noise=BP)
        assert (h.sum(axis=1) == 1 << lat.n_stab).all()


@pytest.mark.parametrize("L", [2, 3])
def test_beta_zero_endpoint_is_n_q(L):
    """<m>_{0,E} = n_q exactly for every class and syndrome."""
    lat = geometry.Lattice(L)
    for idx in range(6):
        syn = sampler.sample(lat, 0.2, 77, [idx], noise=BP)[0][0]
        h = en.class_histograms(lat, syn, noise=BP)
        assert np.allclose(en.mean_n(h, 0.0), lat.n_qubits, rtol=0, atol=1e-12)


def test_chain_mean_matches_enumeration():
    """L = 3, q = 0.10 at beta* = 0.85 beta_bar: the pooled chain average of m
    agrees with the exact <m>_{beta*,E} within statistical error."""
    L, q, C, sweeps, burn = 3, 0.10, 8, 2000, 200
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, q, 0x1302266900000001, [4], noise=BP)[0][0]
    bs = tables.ladder(q, 1, BP)[0]
    exact = en.mean_n(en.class_histograms(lat, syn, noise=BP), bs)
    reps = init.representatives(lat, syn)
    ci, hi = np.meshgrid(np.arange(4), np.arange(C), indexing="ij")
    ci, hi = ci.ravel(), hi.ravel()
    tab = np.broadcast_to(tables.tables(q, 1, BP)[0], (ci.size, 4))
    res = chains.run(lat, reps[ci], np.full(ci.size, 4), ci, np.ones_like(ci), hi, tab, 0xBEEF,
                     0, burn + sweeps, burn, noise=BP)
    per_chain = (res["S"] / (4.0 * sweeps)).reshape(4, C)
    est = per_chain.mean(axis=1)
    se = per_chain.std(axis=1, ddof=1) / np.sqrt(C)
    assert (np.abs(est - exact) < 6 * se + 2e-3 * exact).all(), (est, exact, se)


def test_chain_invariants():
    lat = geometry.Lattice(4)
    syn = sampler.sample(lat, 0.12, 11, [3], noise=BP)[0][0]
    reps = init.matching_representatives(lat, syn)
    T = 8
    ci = np.arange(T) % 4
    tab = np.broadcast_to(tables.tables(0.12, 1, BP)[0], (T, 4))
    chains.run(lat, reps[ci], np.full(T, 3), ci, np.ones(T, int), np.arange(T) // 4, tab, 5,
               0, 6, 2, check_invariants=True,
               syndromes=np.broadcast_to(syn, (T, lat.n_stab)), noise=BP)


def test_simpson_recovers_exact_log_z():
    """With the exact <m>_{beta_k} of a K = 20 ladder plugged in, the
    estimator's log Z_E (closed-form endpoint f0 = n_q included) equals the
    exact log Z_E(beta_bar) up to Simpson's error.  The depolarizing endpoint
    (3/4 n_q) would shift every class by (n_q / 4) * h / 3, h = beta_bar / K,
    well above that error."""
    L, q, K = 3, 0.1, 20
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, q, 0x1302266900000001, [2], noise=BP)[0][0]
    h = en.class_histograms(lat, syn, noise=BP)
    bb = tables.beta_bar(q, BP)
    exact = en.log_z(h, bb)
    means = np.array([en.mean_n(h, b) for b in tables.ladder(q, K, BP)]).T      # [4, K]
    sweeps = 10**6
    S = np.rint(means[:, :, None] * 4 * sweeps).astype(np.int64)
    _, _, _, chosen, logz = estimator.estimate_log_z(S, S, 1, sweeps, bb, lat.n_qubits,
                                                     lat.n_stab, noise=BP)
    assert np.abs(logz - exact).max() < 2e-3
    _, _, _, _, wrong = estimator.estimate_log_z(S, S, 1, sweeps, bb, lat.n_qubits, lat.n_stab)
    assert np.abs(wrong - exact).min() > 0.05
    assert chosen == int(np.argmax(exact))


def test_single_temperature_integral_closed_form():
    """K = 1 below beta_bar: trapezoid on [0, beta*] plus <m> held on
    [beta*, beta_bar].  With <m> = f0 = n_q constant the integral is
    n_q * beta_bar; at beta* = beta_bar it is the plain trapezoid."""
    n_q, n_stab, sweeps = 13, 12, 1000
    bb = tables.beta_bar(0.1, BP)
    bs = 0.85 * bb
    S = np.full((4, 1, 1), n_q * 4 * sweeps, dtype=np.int64)
    logz = estimator.estimate_log_z(S, S, 1, sweeps, bb, n_q, n_stab, BP, bs)[4]
    assert np.allclose(logz, n_stab * math.log(2) - n_q * bb, rtol=0, atol=1e-12)
    S2 = np.array([7, 8, 9, 10], dtype=np.int64).reshape(4, 1, 1) * 4 * sweeps
    lz = estimator.estimate_log_z(S2, S2, 1, sweeps, bb, n_q, n_stab, BP, bs)[4]
    for e, m in enumerate([7, 8, 9, 10]):
        want = bs / 2 * (n_q + m) + (bb - bs) * m
        assert lz[e] == pytest.approx(n_stab * math.log(2) - want, abs=1e-12)
    lz1 = estimator.estimate_log_z(S2, S2, 1, sweeps, bb, n_q, n_stab, BP, bb)[4]
    for e, m in enumerate([7, 8, 9, 10]):
        assert lz1[e] == pytest.approx(n_stab * math.log(2) - bb / 2 * (n_q + m), abs=1e-12)


def test_decoder_recovers_ml_class_at_low_rate():
    """L = 3, q = 0.05: with ample sweeps the decoder's class agrees with the
    exact most likely class (enumeration at beta_bar) on syndromes where that
    class is clearly ahead."""
    L, q = 3, 0.05
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, q, 0xC0DE, np.arange(12), noise=BP)
    out = decoder.decode(L, syn, q, 300, 0xFACE, chains_per_class=2, burn=30, noise=BP)
    checked = 0
    for i in range(12):
        pr = en.class_probabilities(en.class_histograms(lat, syn[i], noise=BP),
                                    tables.beta_bar(q, BP))
        top = np.sort(pr)[::-1]
        if top[0] > 2 * top[1]:
            assert out["chosen"][i] == int(np.argmax(pr)), (i, pr)
            checked += 1
    assert checked >= 6
