"""Pins for the oracle's imperfect-measurement model (Sec. VI): sampler,
class starts, chain invariants, and exact space-time enumeration at L = 2."""

import math

import numpy as np
import pytest

from oracle import geometry, spacetime as stm, tables
from oracle import enumerate as en


def _all_paulis(nq):
    """codes [4^nq, nq]: index i has qubit k's code in bits 2k, 2k+1."""
    idx = np.arange(4 ** nq)
    return ((idx[:, None] >> (2 * np.arange(nq))[None, :]) & 3).astype(np.uint8)


def exact_histograms(lat, obs, T=2):
    """[4, 2 n_q + 1, n_stab + 1] counts of consistent hypotheses (E_0, E_1,
    M_0) by class, n and m, for one T = 2 observation history (plain
    definition: run over all pairs of data errors; M_0 is then fixed)."""
    assert T == 2
    codes = _all_paulis(lat.n_qubits)
    syn = geometry.syndrome(lat, codes).astype(np.int64)
    sidx = (syn << np.arange(lat.n_stab)).sum(axis=1)
    w = geometry.weight(codes).astype(np.int64)
    cls = geometry.class_index(lat, codes)
    s0 = int((obs[0].astype(np.int64) << np.arange(lat.n_stab)).sum())
    s1 = int((obs[1].astype(np.int64) << np.arange(lat.n_stab)).sum())
    i0 = np.arange(codes.shape[0])[:, None]
    i1 = np.arange(codes.shape[0])[None, :]
    c = i0 ^ i1                                  # accumulated error C_1
    valid = sidx[c] == s1
    m = np.bitwise_count((s0 ^ sidx[i0]).astype(np.uint64)).astype(np.int64)
    n = w[i0] + w[i1]
    h = np.zeros((4, 2 * lat.n_qubits + 1, lat.n_stab + 1), dtype=np.int64)
    np.add.at(h, (np.broadcast_to(cls[c], valid.shape)[valid],
                  np.broadcast_to(n, valid.shape)[valid],
                  np.broadcast_to(m, valid.shape)[valid]), 1)
    return h


def mean_energy(h, beta, xi):
    nn = np.arange(h.shape[1])[:, None]
    mm = np.arange(h.shape[2])[None, :]
    e = nn + xi * mm
    out = []
    for hc in h:
        wgt = hc * np.exp(-beta * (e - e[hc > 0].min()))
        out.append(float((wgt * e).sum() / wgt.sum()))
    return np.array(out)


def class_probs(h, beta, xi):
    nn = np.arange(h.shape[1])[:, None]
    mm = np.arange(h.shape[2])[None, :]
    z = np.array([(hc * np.exp(-beta * (nn + xi * mm))).sum() for hc in h])
    return z / z.sum()


def test_sampler_rates_and_perfect_last_round():
    L, T, p, pm = 5, 4, 0.09, 0.06
    lat = geometry.Lattice(L)
    obs, cls, E, M = stm.sample(lat, p, pm, T, 0x51, np.arange(3000))
    for code in (1, 2, 3):
        f = (E == code).mean()
        assert abs(f - p / 3) < 5 * math.sqrt(p / 3 / E.size)
    fm = M[:, :T - 1].mean()
    assert abs(fm - pm) < 5 * math.sqrt(pm / M[:, :T - 1].size)
    assert not M[:, T - 1].any()
    # observations recomputed by an explicit loop over rounds
    C = np.zeros_like(E[:, 0])
    for t in range(T):
        C = C ^ E[:, t]
        assert np.array_equal(obs[:, t], geometry.syndrome(lat, C) ^ M[:, t])
    assert np.array_equal(cls, geometry.class_index(lat, C))


@pytest.mark.parametrize("L,T", [(2, 1), (3, 3), (5, 2)])
def test_starts_are_consistent(L, T):
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, 0.1, 0.1, T, 3, np.arange(6))
    for i in range(6):
        E, M = stm.starts(lat, obs[i])
        assert np.array_equal(stm.observations(lat, E, M), np.broadcast_to(obs[i], (4,) + obs[i].shape))
        assert stm.hyp_class(lat, E).tolist() == [0, 1, 2, 3]
        assert not M[:, T - 1].any() and not E[:, :T - 1].any()


@pytest.mark.parametrize("L,T", [(2, 2), (3, 3), (4, 2)])
def test_chain_invariants(L, T):
    """Observations, class, the perfect last round and both energies (against
    recounts) after every sweep."""
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, 0.12, 0.1, T, 8, [5])
    stm.decode(L, obs, 0.12, 0.1, 3, 2, chains_per_class=2, burn=1, check_invariants=True)


def test_time_table():
    thr, always = stm.time_table(2.0, 0.5)
    for dn in range(-2, 3):
        for dm in range(-2, 3):
            e = dn + 0.5 * dm
            assert always[dn + 2, dm + 2] == (e <= 0)
            if e > 0:
                assert thr[dn + 2, dm + 2] == math.floor(math.exp(-2.0 * e) * 2**32)


def test_beta_zero_endpoint():
    """Enumeration at beta = 0: <n + xi m> = 3/4 n_q T + xi n_stab (T-1) / 2."""
    lat = geometry.Lattice(2)
    obs, _, _, _ = stm.sample(lat, 0.2, 0.2, 2, 17, np.arange(4))
    xi = stm.xi_of(0.2, 0.2)
    for i in range(4):
        h = exact_histograms(lat, obs[i])
        assert (h.sum(axis=(1, 2)) == h.sum() // 4).all()      # classes equally large
        f0 = 0.75 * lat.n_qubits * 2 + xi * 0.5 * lat.n_stab * 1
        assert np.allclose(mean_energy(h, 0.0, xi), f0, rtol=0, atol=1e-9)


def test_chain_means_match_enumeration():
    """L = 2, T = 2: pooled chain averages of n + xi m agree with the exact
    averages at beta_bar within statistical error."""
    L, p, pm, C, sweeps, burn = 2, 0.15, 0.1, 8, 1500, 100
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, p, pm, 2, 0xE7, [3])
    xi = stm.xi_of(p, pm)
    bb = tables.beta_bar(p)
    exact = mean_energy(exact_histograms(lat, obs[0]), bb, xi)
    out = stm.decode(L, obs, p, pm, sweeps, 0xF00, chains_per_class=C, burn=burn)
    per = (out["sum_n"][0] + xi * out["sum_m"][0]) / (2.0 * sweeps)       # [4, C]
    est = per.mean(axis=1)
    se = per.std(axis=1, ddof=1) / np.sqrt(C)
    assert (np.abs(est - exact) < 6 * se + 2e-3 * exact).all(), (est, exact, se)


def test_decision_matches_exact_ml_class():
    """L = 2, T = 2: with ample sweeps the decision equals the class with the
    largest exact probability wherever that class is clearly ahead."""
    L, p, pm = 2, 0.1, 0.08
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, p, pm, 2, 0xD1, np.arange(16))
    xi = stm.xi_of(p, pm)
    out = stm.decode(L, obs, p, pm, 400, 0xACE, chains_per_class=2, burn=40)
    checked = 0
    for i in range(16):
        pr = class_probs(exact_histograms(lat, obs[i]), tables.beta_bar(p), xi)
        top = np.sort(pr)[::-1]
        if top[0] > 2 * top[1]:
            assert out["chosen"][i] == int(np.argmax(pr)), (i, pr)
            checked += 1
    assert checked >= 6


def test_single_round_is_the_perfect_measurement_model():
    """T = 1: no time moves and no outcome errors; the chain samples the
    perfect-measurement class distribution (exact means from the
    single-round enumeration)."""
    L, p, C, sweeps, burn = 3, 0.1, 8, 1500, 100
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, p, 0.1, 1, 0x1A, [2])
    exact = en.mean_n(en.class_histograms(lat, obs[0, 0]), tables.beta_bar(p))
    out = stm.decode(L, obs, p, 0.1, sweeps, 0xB0B, chains_per_class=C, burn=burn)
    assert (out["sum_m"] == 0).all()
    per = out["sum_n"][0] / (2.0 * sweeps)
    est = per.mean(axis=1)
    se = per.std(axis=1, ddof=1) / np.sqrt(C)
    assert (np.abs(est - exact) < 6 * se + 2e-3 * exact).all(), (est, exact, se)
