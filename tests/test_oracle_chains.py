"""Pins for the oracle's Metropolis chains (Sec. IV, Sec. IV.A, Sec. V)."""

import json
import os

import numpy as np
import pytest

from oracle import chains, decoder, estimator, geometry, init, sampler, tables
from oracle import enumerate as en

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
CODE = {"I": 0, "X": 1, "Z": 2, "Y": 3}


def test_minimal_example():
    """Fig. minimalExample: Z_a X_b X_c on one star's qubits {a, b, c, d};
    applying that sigma^x stabilizer gives Y_a X_d, lowering n from 3 to 2."""
    g = GOLDEN["minimal_example"]
    lat = geometry.Lattice(5)
    s = next(s for s in range(lat.n_stars) if len(lat.supports[s]) == 4)
    a, b, c, d = lat.supports[s]
    st = np.zeros((1, lat.n_qubits), dtype=np.uint8)
    for q, name in zip((a, b, c, d), "abcd"):
        st[0, q] = CODE[g["before"][name]]
    assert geometry.weight(st)[0] == g["weight_before"]
    assert chains.delta_n(lat, st, s)[0] == g["delta_n"]
    chains.apply_site(lat, st, s, np.array([True]))
    for q, name in zip((a, b, c, d), "abcd"):
        assert st[0, q] == CODE[g["after"][name]]
    assert geometry.weight(st)[0] == g["weight_after"]


def _tasks(lat, syn, K, C, p):
    reps = init.representatives(lat, syn)
    ci, ki, hi = np.meshgrid(np.arange(4), np.arange(K), np.arange(C), indexing="ij")
    ci, ki, hi = ci.ravel(), ki.ravel(), hi.ravel()
    tab = tables.tables(p, K)
    return reps[ci], ci, ki + 1, hi, tab[ki]


@pytest.mark.parametrize("L,p", [(2, 0.1), (3, 0.15), (4, 0.05), (5, 0.3)])
def test_invariants(L, p):
    """Sec. IV: stabilizer moves keep the syndrome and the class; the running n
    equals a recount after every phase."""
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, p, 11, [L])[0][0]
    st, ci, ki, hi, tab = _tasks(lat, syn, 2, 2, p)
    T = st.shape[0]
    chains.run(lat, st, np.full(T, 5), ci, ki, hi, tab, 42, 0, 6, 2,
               check_invariants=True, syndromes=np.broadcast_to(syn, (T, lat.n_stab)))


def test_zero_temperature_never_increases_weight():
    """Sec. IV.A: for beta* -> infinity no move raises the weight."""
    lat = geometry.Lattice(5)
    syn = sampler.sample(lat, 0.15, 3, [0])[0][0]
    st, ci, ki, hi, _ = _tasks(lat, syn, 1, 4, 0.15)
    T = st.shape[0]
    res = chains.run(lat, st, np.zeros(T), ci, ki, hi, np.zeros((T, 4), np.uint32), 1, 0, 30, 0,
                     trace=True)
    tr = np.concatenate([geometry.weight(st)[:, None], res["trace"]], axis=1)
    assert (np.diff(tr, axis=1) <= 0).all()


def test_resume_is_exact():
    lat = geometry.Lattice(4)
    syn = sampler.sample(lat, 0.12, 9, [1])[0][0]
    st, ci, ki, hi, tab = _tasks(lat, syn, 1, 3, 0.12)
    T = st.shape[0]
    sid = np.full(T, 77)
    full = chains.run(lat, st, sid, ci, ki, hi, tab, 5, 0, 40, 10, trace=True)
    a = chains.run(lat, st, sid, ci, ki, hi, tab, 5, 0, 17, 10, trace=True)
    b = chains.run(lat, a["state"], sid, ci, ki, hi, tab, 5, 17, 40, 10,
                   n=a["n"], S=a["S"], A=a["A"], trace=True)
    for k in ("state", "n", "S", "A"):
        assert np.array_equal(full[k], b[k])
    assert np.array_equal(full["trace"], np.concatenate([a["trace"], b["trace"]], axis=1))


@pytest.mark.parametrize("p", [0.1, 0.18])
def test_exact_stationarity_L2(p):
    """The whole colour-phased sweep, with the quantised acceptance, keeps
    exp(-beta n)/Z_E stationary on every class (L = 2: 16 configurations per
    class, one site per colour).  The transition matrix is built from the
    oracle's own Delta-n rule and table; the target comes from enumeration."""
    lat = geometry.Lattice(2)
    beta = tables.beta_bar(p)
    tab = tables.acceptance_table(beta).astype(np.float64) / 2.0**32
    syn = np.array([1, 0, 0, 1], dtype=np.uint8)
    reps = init.representatives(lat, syn)
    for e in range(4):
        configs = []
        for m in range(16):
            c = reps[e:e + 1].copy()
            for s in range(4):
                if (m >> s) & 1:
                    chains.apply_site(lat, c, s, np.array([True]))
            configs.append(c[0])
        configs = np.array(configs)
        key = {bytes(c): i for i, c in enumerate(configs)}
        M = np.eye(16)
        for ph in range(4):
            (s,) = lat.phase_sites[ph]
            Tm = np.zeros((16, 16))
            d = chains.delta_n(lat, configs, s)
            moved = configs.copy()
            chains.apply_site(lat, moved, s, np.ones(16, dtype=bool))
            for i in range(16):
                pa = 1.0 if d[i] <= 0 else tab[d[i] - 1]
                Tm[i, key[bytes(moved[i])]] += pa
                Tm[i, i] += 1.0 - pa
            M = M @ Tm
        w = geometry.weight(configs)
        target = np.exp(-beta * w)
        target /= target.sum()
        vals, vecs = np.linalg.eig(M.T)
        pi = np.real(vecs[:, np.argmin(np.abs(vals - 1.0))])
        pi /= pi.sum()
        assert np.allclose(pi, target, rtol=2e-3, atol=1e-12)


def test_chain_mean_matches_enumeration():
    """Config-1 scale (L = 3, p = 0.10, 2000 sweeps): the pooled chain average
    of n agrees with the exact <n>_{beta_bar,E} within statistical error."""
    L, p, C, sweeps, burn = 3, 0.10, 8, 2000, 200
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, p, 0x1302266900000001, [4])[0][0]
    exact = en.mean_n(en.class_histograms(lat, syn), tables.beta_bar(p))
    st, ci, ki, hi, tab = _tasks(lat, syn, 1, C, p)
    T = st.shape[0]
    res = chains.run(lat, st, np.full(T, 4), ci, ki, hi, tab, 0xBEEF, 0, burn + sweeps, burn)
    per_chain = (res["S"] / (4.0 * sweeps)).reshape(4, C)
    est = per_chain.mean(axis=1)
    se = per_chain.std(axis=1, ddof=1) / np.sqrt(C)
    assert (np.abs(est - exact) < 6 * se + 2e-3 * exact).all(), (est, exact, se)


def test_ti_probabilities_match_enumeration():
    """K = 20 Simpson integration (Sec. IV.A) recovers the exact class
    probabilities at L = 3; the Simpson rule's own error is computed from the
    exact <n>_beta and added to the tolerance."""
    L, p, C, K, sweeps, burn = 3, 0.10, 4, 20, 400, 100
    lat = geometry.Lattice(L)
    syn = sampler.sample(lat, p, 0x1302266900000001, [2])[0][0]
    h = en.class_histograms(lat, syn)
    bb = tables.beta_bar(p)
    exact_p = en.class_probabilities(h, bb)
    # exact Simpson: plug exact means into the estimator
    exact_means = np.array([en.mean_n(h, b) for b in tables.ladder(p, K)]).T   # [4, K]
    T = 4 * sweeps
    S_exact = np.rint(exact_means[:, :, None] * T * 1e6).astype(np.int64)
    simpson_p = estimator.estimate(S_exact, S_exact, 1, sweeps * 10**6 // 1, bb,
                                   lat.n_qubits, lat.n_stab)[0]
    out = decoder.decode(L, syn[None], p, sweeps, 0xFACE, chains_per_class=C, n_temps=K,
                         burn=burn, syndrome_ids=[2])
    assert np.abs(simpson_p - exact_p).max() < 5e-3
    assert np.abs(out["class_prob"][0] - exact_p).max() < 0.03 + np.abs(simpson_p - exact_p).max()
    assert int(np.argmax(exact_p)) == int(out["chosen"][0])


def test_decision_rules():
    """K = 1 decides by the smallest pooled <n> (Sec. IV.A); with no counted
    sweep it compares the starting weights (the matching-only limit)."""
    S = np.array([[[50]], [[40]], [[40]], [[90]]], dtype=np.int64)
    prob, mean, key, chosen = estimator.estimate(S, S, 1, 3, 2.0, 13, 12)
    assert chosen == 1 and key.tolist() == [50, 40, 40, 90]
    assert np.argmax(prob) == 1 and prob[1] == prob[2]
    nf = np.array([[[7]], [[5]], [[9]], [[6]]], dtype=np.int64)
    prob, mean, key, chosen = estimator.estimate(np.zeros_like(nf), nf, 1, 0, 2.0, 13, 12)
    assert chosen == 1 and mean.tolist() == [7.0, 5.0, 9.0, 6.0]


@pytest.mark.parametrize("mode", [decoder.INIT_CANONICAL, decoder.INIT_MATCHING])
def test_decoder_zero_sweeps_is_min_weight_of_starts(mode):
    """With no sweep the decision compares the class starts' weights, which
    for the matching start is Sec. III's enhanced-matching rule."""
    lat = geometry.Lattice(5)
    syn, _, _ = sampler.sample(lat, 0.1, 3, np.arange(20))
    out = decoder.decode(5, syn, 0.1, 0, 1, chains_per_class=1, init_mode=mode)
    start = init.matching_representatives if mode == decoder.INIT_MATCHING else init.representatives
    for i in range(20):
        w = geometry.weight(start(lat, syn[i]))
        assert out["chosen"][i] == int(np.argmin(w))


@pytest.mark.parametrize("K", [1, 2, 4, 20])
def test_quadrature_exact_on_polynomials(K):
    """Simpson's rule is exact for cubics and the trapezoid for straight
    lines: with <n>_beta such a polynomial (and f(0) = 3/4 n_q, the closed-form
    endpoint), the estimator's log Z must equal n_stab log 2 minus the
    closed-form integral (Eq. main)."""
    n_q, n_stab = 13, 12
    f0 = 0.75 * n_q
    bb = tables.beta_bar(0.1)
    c = [-1.5, 0.25, -0.02] if K > 1 else [-1.5, 0.0, 0.0]
    sweeps = 2**20
    T = 4 * sweeps
    S = np.zeros((4, K, 1), dtype=np.int64)
    exact = []
    for e in range(4):
        a1 = c[0] - 0.05 * e                 # one polynomial per class
        f = lambda b: f0 + a1 * b + c[1] * b**2 + c[2] * b**3
        for k, b in enumerate(tables.ladder(0.1, K)):
            S[e, k, 0] = int(round(f(b) * T))
        exact.append(f0 * bb + a1 * bb**2 / 2 + c[1] * bb**3 / 3 + c[2] * bb**4 / 4)
    prob, mean, key, chosen, logz = estimator.estimate_log_z(S, S, 1, sweeps, bb, n_q, n_stab)
    for e in range(4):
        assert logz[e] == pytest.approx(n_stab * np.log(2) - exact[e], abs=1e-5)
    assert chosen == 3 and np.argmax(prob) == 3
