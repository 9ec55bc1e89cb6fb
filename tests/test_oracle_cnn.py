"""Pins for the gate network's float64 reference: analytic gradients against
central finite differences, the bf16 rounding helper against its definition,
Adam against a closed-form first step, and the layout against the shapes."""

import numpy as np
import pytest

from oracle import cnn
from paper_1302_2669_amd.inputs import cnn_init, uniform_syndromes


def test_bf16_rounding():
    """bfloat16 keeps 8 significant bits: the spacing above 1 is 2^-7."""
    u = 2.0 ** -7
    cases = [(1.0, 1.0), (1 + u, 1 + u), (1 + u / 2, 1.0),            # tie -> even
             (1 + 3 * u / 2, 1 + 2 * u),                                # tie -> even
             (1 + u / 2 + 1e-9, 1 + u), (-(1 + 0.7 * u), -(1 + u)),
             (3.0, 3.0), (0.0, 0.0), (2.0 ** -20 * (1 + u / 4), 2.0 ** -20)]
    for x, want in cases:
        assert cnn.to_bf16(x) == want, x
    # agrees with truncating the float32 bit pattern when the dropped bits are 0
    rng = np.random.default_rng(3)
    v = rng.standard_normal(1000).astype(np.float32)
    exact = (v.view(np.uint32) & 0xFFFF0000).view(np.float32).astype(np.float64)
    assert np.array_equal(cnn.to_bf16(exact), exact)


def test_layout_matches_init():
    L = 5
    flat = cnn_init(L, 1)
    n = sum(int(np.prod(s)) for _, s in cnn.param_shapes(L))
    assert flat.size == n
    P = cnn.unflatten(L, flat)
    assert np.array_equal(cnn.flatten(L, P), flat.astype(np.float64))
    assert not P["b1"].any() and P["W2"].std() > 0


@pytest.mark.parametrize("L", [3, 4])
def test_gradients_against_finite_differences(L):
    B = 3
    flat = cnn_init(L, 7).astype(np.float64)
    syn = uniform_syndromes(L, B, seed=L, density=0.4)
    p = np.array([0.05, 0.11, 0.17])
    rng = np.random.default_rng(0)
    t = rng.dirichlet(np.ones(4), size=B)
    y = rng.integers(0, 3, size=B)
    # move biases off zero so that every ReLU is away from its kink
    flat = flat + 0.01 * rng.standard_normal(flat.size)
    P = cnn.unflatten(L, flat)
    loss, _, g, _ = cnn.backward(L, P, syn, p, t, y, 0.7, bf16=False)
    gflat = cnn.flatten(L, g)

    def f(v):
        return cnn.backward(L, cnn.unflatten(L, v), syn, p, t, y, 0.7, bf16=False)[0]

    eps = 1e-6
    idx = np.concatenate([rng.choice(flat.size, 40, replace=False),
                          [0, 864 + 3, flat.size - 1, flat.size - 8]])
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = eps
        fd = (f(flat + e) - f(flat - e)) / (2 * eps)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])
    d = rng.standard_normal(flat.size)
    d /= np.linalg.norm(d)
    fd = (f(flat + eps * d) - f(flat - eps * d)) / (2 * eps)
    assert abs(fd - gflat @ d) <= 1e-6 * max(1.0, abs(fd))


def test_loss_closed_form():
    """Uniform logits: loss = log 4 + w log 3 for any targets."""
    z = np.zeros((5, 7))
    t = np.random.default_rng(1).dirichlet(np.ones(4), size=5)
    loss, dz, _ = cnn.loss_and_dlogits(z, t, np.array([0, 1, 2, 0, 1]), 0.5)
    assert loss == pytest.approx(np.log(4) + 0.5 * np.log(3), rel=1e-14)
    assert np.allclose(dz[:, :4].sum(axis=1), 0) and np.allclose(dz[:, 4:].sum(axis=1), 0)


def test_adam_first_step():
    """With bias correction the first step moves every weight by lr*sign(g)
    (up to eps)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 2.0])}
    z = {"w": np.zeros(3)}
    out, m, v = cnn.adam(p, g, z, z, 0.01, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(out["w"], p["w"] - 0.01 * np.sign(g["w"]), atol=1e-9)


# ---------------------------------------------------------------- training support
@pytest.mark.parametrize("L", [3, 13])
def test_he_init_statistics(L):
    """He-normal blocks: mean 0 and standard deviation sqrt(2 / fan-in) within
    sampling error (normal draws by Box-Muller from Philox); biases zero."""
    from oracle import cnn
    prm = cnn.he_init(L, 5).astype(np.float64)
    blocks = [(32 * 27, 27), (32, 0), (32 * 288, 288), (32, 0), (32 * 288, 288), (32, 0),
              (7 * 32 * L * L, 32 * L * L), (7, 0)]
    at = 0
    for size, fan in blocks:
        x = prm[at:at + size]
        at += size
        if fan == 0:
            assert (x == 0).all()
            continue
        sd = np.sqrt(2.0 / fan)
        assert abs(x.mean()) < 5 * sd / np.sqrt(size)
        assert abs(x.std() / sd - 1) < 5 * np.sqrt(0.5 / size) + 1e-3
    assert at == prm.size
    assert not np.array_equal(cnn.he_init(L, 5), cnn.he_init(L, 6))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 1000, 4097])
def test_epoch_permutation_is_a_bijection(n):
    from oracle import cnn
    p0 = cnn.epoch_permutation(n, 11, 0)
    assert sorted(p0.tolist()) == list(range(n))
    if n >= 64:
        assert not np.array_equal(p0, cnn.epoch_permutation(n, 11, 1))
        assert not np.array_equal(p0, cnn.epoch_permutation(n, 12, 0))
        assert not np.array_equal(p0, np.arange(n))


def test_budget_label_rule():
    from oracle import cnn
    full = np.array([0, 1, 2, 3, 1, 2])
    zero = np.array([0, 0, 2, 1, 3, 0])
    short = np.array([1, 1, 0, 3, 2, 2])
    assert cnn.budget_labels(zero, short, full).tolist() == [0, 1, 0, 1, 2, 1]


def test_relative_targets_by_enumeration():
    """Class probabilities read relative to the start decision, against a
    direct count at L = 3: every configuration F with the syndrome (a class
    start times every stabilizer product), grouped by the logical class of the
    Pauli product F x R, R the start of the decided class, each weighted by
    exp(-beta_bar n(F))."""
    from oracle import enumerate as en
    from oracle import geometry, matching, sampler, tables
    L, p = 3, 0.15
    lat = geometry.Lattice(L)
    beta = tables.beta_bar(p)
    syn, _, _ = sampler.sample(lat, p, 0x5E1, np.arange(40))
    stars = [lat.supports[s] for s in range(lat.n_stars)]
    plaqs = [lat.supports[s] for s in range(lat.n_stars, lat.n_stab)]

    def span(gens):
        out = [np.zeros(lat.n_qubits, dtype=np.uint8)]
        for g in gens:
            v = np.zeros(lat.n_qubits, dtype=np.uint8)
            v[list(g)] = 1
            out = out + [o ^ v for o in out]
        return np.array(out)

    xs, zs = span(stars), span(plaqs)
    seen = set()
    for i in range(syn.shape[0]):
        reps = matching.mwpm_representatives(lat, syn[i])
        start = int(np.argmin(geometry.weight(reps)))
        seen.add(start)
        prob = en.class_probabilities(en.class_histograms(lat, syn[i]), beta)
        rel = cnn.relative_targets(prob[None, :], np.array([start]))[0]
        direct = np.zeros(4)
        for e in range(4):
            xr, zr = reps[e] & 1, (reps[e] >> 1) & 1
            x = xs ^ xr[None, :]
            z = zs ^ zr[None, :]
            F = (x[:, None, :] | (z[None, :, :] << 1)).reshape(-1, lat.n_qubits)
            assert (geometry.syndrome(lat, F) == syn[i]).all()
            k = geometry.class_index(lat, F ^ reps[start][None, :])
            np.add.at(direct, k, np.exp(-beta * geometry.weight(F)))
        direct /= direct.sum()
        np.testing.assert_allclose(rel, direct, rtol=1e-12, atol=1e-15)
        assert rel[0] == prob[start]
    assert len(seen) >= 2      # some syndromes decide a class other than the identity


def test_start_weight_gap_hand_cases():
    w = np.array([[3, 5, 4, 9], [2, 2, 7, 7], [10, 3, 8, 8], [0, 0, 0, 0], [9, 8, 7, 6]])
    assert cnn.start_weight_gap(w).tolist() == [1, 0, 5, 0, 1]


def test_gap_bin_edges():
    """floor(p * 100) in fp32, capped: bin edges of decimal rates land where
    the fp32 product does."""
    p = np.array([0.0, 0.009, 0.01, 0.05, 0.0999, 0.1, 0.15, 0.289, 0.49, 0.5, 0.74])
    want = [int(np.floor(np.float32(x) * np.float32(100.0))) for x in p]
    want = [min(k, cnn.GAP_BINS - 1) for k in want]
    assert cnn.gap_bin(p).tolist() == want
    assert cnn.gap_bin(p).tolist() == [0, 0, 1, 5, 9, 10, 15, 28, 49, 49, 49]


def test_fit_gap_table_hand_case():
    """Bin 5: gaps 0..3 twice each, labels missing at gaps 0 and 1."""
    gaps = np.array([0, 0, 1, 1, 2, 2, 3, 3])
    w = np.stack([np.zeros(8, int), gaps, gaps + 5, gaps + 9], axis=1)
    p = np.full(8, 0.055)
    budget = np.array([1, 0, 2, 0, 0, 0, 0, 0])
    t = cnn.fit_gap_table(p, w, budget, 0.0, 2)
    assert t[5] == 2 and (np.delete(t, 5) == cnn.GAP_NEVER).all()
    assert cnn.fit_gap_table(p, w, budget, 0.25, 2)[5] == 0       # 2 of 8 at G = 0
    assert cnn.fit_gap_table(p, w, budget, 0.2, 2)[5] == 1        # 1 of 6 at G = 1
    assert cnn.fit_gap_table(p, w, budget, 0.0, 5)[5] == cnn.GAP_NEVER   # 4 < 5 left at G = 2
    route = cnn.gap_route(np.array([0.055, 0.055, 0.3]),
                          np.array([[0, 1, 5, 9], [0, 2, 5, 9], [0, 40, 50, 60]]), t)
    assert route.tolist() == [False, True, False]                # bin 30 is NEVER


def test_fit_gap_table_meets_its_definition():
    """On random labelled samples: every fitted threshold satisfies the
    miss bound with at least min_count samples, every smaller one does not,
    and a NEVER bin has no qualifying threshold with enough samples."""
    rng = np.random.default_rng(0x6A9)
    n = 4000
    p = rng.uniform(0.03, 0.2, n)
    w = np.sort(rng.integers(0, 30, size=(n, 4)), axis=1)[:, rng.permutation(4)]
    gap = cnn.start_weight_gap(w)
    # misses likelier at small gaps and high rates
    budget = (rng.random(n) < np.exp(-gap / 3.0) * p * 4).astype(np.int32)
    for max_miss, min_count in ((0.0, 1), (0.01, 20), (0.05, 40)):
        t = cnn.fit_gap_table(p, w, budget, max_miss, min_count)
        b = cnn.gap_bin(p)
        for k in range(cnn.GAP_BINS):
            gk, mk = gap[b == k], budget[b == k] != 0

            def ok(G):
                sel = gk >= G
                return sel.sum() >= min_count and mk[sel].sum() <= max_miss * sel.sum()

            if t[k] == cnn.GAP_NEVER:
                assert not any(ok(G) for G in range(cnn.GAP_NEVER))
            else:
                assert ok(int(t[k])) and not any(ok(G) for G in range(int(t[k])))
        assert (t != cnn.GAP_NEVER).sum() >= 5
