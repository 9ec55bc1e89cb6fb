"""Pins for the minimum-weight matching start (Sec. III, Sec. IV).

The blossom solver is checked against brute force over all perfect matchings,
against a subset dynamic program, against its own linear-programming
certificate and against an independent integer program (scipy's HiGHS);
the class starts against brute force over every configuration of one anyon
type (a representative times every product of the other type's stabilizers)
at L = 2 ... 5.
"""

import functools

import numpy as np
import pytest

from oracle import geometry, init, sampler
from oracle import matching as mm

from paper_1302_2669_amd.inputs import uniform_syndromes


def _random_weights(rng, n, hi):
    a = rng.integers(0, hi, size=(n, n)) * 2
    a = np.triu(a, 1)
    return a + a.T


def _brute(W):
    """Minimum total weight over every perfect matching, and the set of
    matchings reaching it (as sorted pair tuples)."""
    n = W.shape[0]
    best, arg = None, []

    def rec(free, pairs, tot):
        nonlocal best, arg
        if not free:
            if best is None or tot < best:
                best, arg = tot, [tuple(pairs)]
            elif tot == best:
                arg.append(tuple(pairs))
            return
        a = free[0]
        for k in range(1, len(free)):
            b = free[k]
            rec(free[1:k] + free[k + 1:], pairs + [(a, b)], tot + int(W[a, b]))

    rec(list(range(n)), [], 0)
    return best, arg


def _subset_dp(W):
    n = W.shape[0]

    @functools.lru_cache(maxsize=None)
    def f(mask):
        if mask == 0:
            return 0
        a = (mask & -mask).bit_length() - 1
        rest = mask & ~(1 << a)
        best = None
        m = rest
        while m:
            b = (m & -m).bit_length() - 1
            m &= m - 1
            v = int(W[a, b]) + f(rest & ~(1 << b))
            if best is None or v < best:
                best = v
        return best

    return f((1 << n) - 1)


def _total(W, mate):
    return sum(int(W[v, mate[v]]) for v in range(len(mate)) if mate[v] > v)


@pytest.mark.parametrize("n", [0, 2, 4, 6, 8, 10])
def test_blossom_against_brute_force(n):
    rng = np.random.default_rng(n)
    for trial in range(40):
        W = _random_weights(rng, n, 4 if trial % 2 else 1000)
        res = mm.min_weight_perfect_matching(W)
        best, arg = _brute(W)
        assert _total(W, res.mate) == best
        pairs = tuple(sorted((v, int(res.mate[v])) for v in range(n) if res.mate[v] > v))
        assert pairs in [tuple(sorted(a)) for a in arg]
        assert mm.certificate_holds(W, res)


@pytest.mark.parametrize("n", [12, 14, 16])
def test_blossom_against_subset_dp(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(4):
        W = _random_weights(rng, n, 3 if trial % 2 else 50)
        res = mm.min_weight_perfect_matching(W)
        assert _total(W, res.mate) == _subset_dp(W)


def test_certificate_rejects_a_worse_matching():
    """The certificate is not vacuous: swapping two matched pairs of an
    optimal matching with a unique optimum breaks it."""
    rng = np.random.default_rng(7)
    W = _random_weights(rng, 8, 10 ** 6)
    res = mm.min_weight_perfect_matching(W)
    mate = res.mate.copy()
    a = 0
    b = int(mate[a])
    c = next(v for v in range(8) if v not in (a, b))
    d = int(mate[c])
    mate[a], mate[c], mate[b], mate[d] = c, a, d, b
    assert not mm.certificate_holds(W, mm.Result(mate, res.u, res.blossoms))


@pytest.mark.parametrize("n", [30, 60])
def test_blossom_certificate_on_larger_graphs(n):
    rng = np.random.default_rng(n)
    for trial in range(3):
        W = _random_weights(rng, n, 5 if trial else 10 ** 6)
        assert mm.certificate_holds(W, mm.min_weight_perfect_matching(W))


def test_splitmix64_is_a_bijection_with_avalanche():
    """splitmix64's output function: distinct states give distinct outputs
    (it is a composition of invertible steps) and one flipped input bit flips
    about half of the output bits."""
    outs = {mm.splitmix64(s) for s in range(4096)}
    assert len(outs) == 4096
    flips = [bin(mm.splitmix64(s) ^ mm.splitmix64(s ^ (1 << b))).count("1")
             for s in range(64) for b in range(24)]
    assert 30 < np.mean(flips) < 34


# ---------------------------------------------------------------- class starts
def _span(gens):
    arr = np.zeros(1, dtype=np.uint64)
    for g in gens:
        arr = np.concatenate([arr, arr ^ np.uint64(g)])
    return arr


def _mask(bits):
    m = 0
    for q in bits:
        m |= 1 << int(q)
    return m


def _exact_type_minima(lat, syn):
    """[2 types][2 parities]: minimum number of x parts (plaquette anyons) and
    z parts (star anyons) over every part with the given anyons and line
    parity: a canonical part times every product of the stabilizers that
    act on that part (stars flip x parts, plaquettes flip z parts), and
    times the logical string."""
    reps = init.representatives(lat, syn)
    col0 = _mask(lat.column0)
    row0 = _mask(lat.row0)
    out = np.zeros((2, 2), dtype=np.int64)
    for t in (0, 1):
        if t == 0:
            gens = [_mask(lat.supports[s]) for s in range(lat.n_stars)]
            part0 = _mask(np.nonzero(reps[0] & 1)[0])
            logical, line = row0, col0
        else:
            gens = [_mask(lat.supports[s]) for s in range(lat.n_stars, lat.n_stab)]
            part0 = _mask(np.nonzero(reps[0] & 2)[0])
            logical, line = col0, row0
        span = _span(gens)
        parts = np.concatenate([span ^ np.uint64(part0), span ^ np.uint64(part0 ^ logical)])
        w = np.bitwise_count(parts).astype(np.int64)
        par = np.bitwise_count(parts & np.uint64(line)).astype(np.int64) & 1
        for b in (0, 1):
            out[t, b] = w[par == b].min()
    return out


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_starts_are_exact_per_type_minima(L):
    """Each class start's x part (z part) has the fewest x (z) parts of any
    configuration with the syndrome's plaquette (star) anyons and the class's
    bx (bz); the start has the syndrome and the class."""
    lat = geometry.Lattice(L)
    n = {2: 16, 3: 24, 4: 12, 5: 4}[L]
    syn = np.concatenate([uniform_syndromes(L, n, seed=L, density=0.5),
                          uniform_syndromes(L, n, seed=L + 9, density=0.15),
                          np.zeros((1, lat.n_stab), np.uint8), np.ones((1, lat.n_stab), np.uint8)])
    for s in syn:
        reps = mm.mwpm_representatives(lat, s)
        ex = _exact_type_minima(lat, s)
        tw = mm.type_weights(lat, s)
        assert np.array_equal(tw, ex)
        for c in range(4):
            assert np.array_equal(geometry.syndrome(lat, reps[c][None])[0], s)
            assert int(geometry.class_index(lat, reps[c][None])[0]) == c
            assert int((reps[c] & 1).sum()) == ex[0, c & 1]
            assert int(((reps[c] >> 1) & 1).sum()) == ex[1, c >> 1]


@pytest.mark.parametrize("L", [2, 3, 5])
def test_single_errors_are_recovered(L):
    """Sec. III (optimal as p -> 0): for every single-qubit error the start
    of the error's own class is the error itself."""
    lat = geometry.Lattice(L)
    for q in range(lat.n_qubits):
        for code in (1, 2, 3):
            e = np.zeros(lat.n_qubits, dtype=np.uint8)
            e[q] = code
            syn = geometry.syndrome(lat, e[None])[0]
            c = int(geometry.class_index(lat, e[None])[0])
            assert np.array_equal(mm.mwpm_representatives(lat, syn)[c], e), (q, code)


@pytest.mark.parametrize("L", [2, 3, 5, 13, 25])
def test_empty_syndrome(L):
    lat = geometry.Lattice(L)
    reps = mm.mwpm_representatives(lat, np.zeros(lat.n_stab, np.uint8))
    assert geometry.weight(reps).tolist() == [0, L, L, 2 * L - 1]


@pytest.mark.parametrize("L,p,n", [(7, 0.15, 3), (9, 0.12, 3), (13, 0.15, 2)])
def test_total_distance_against_integer_program(L, p, n):
    """The matching's total distance equals the optimum of an independent
    integer program (one binary per pair, degree one at every vertex),
    solved by scipy's HiGHS; the solver's certificate holds."""
    opt = pytest.importorskip("scipy.optimize")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, 0x77 + L, np.arange(n))
    for s in syn:
        for is_star in (False, True):
            for b in (0, 1):
                nodes, d, W = mm.problem(lat, s, is_star, b)
                m = len(nodes)
                res = mm.min_weight_perfect_matching(W)
                assert mm.certificate_holds(W, res)
                if m == 0:
                    continue
                iu = np.triu_indices(m, 1)
                A = np.zeros((m, iu[0].size))
                A[iu[0], np.arange(iu[0].size)] = 1
                A[iu[1], np.arange(iu[0].size)] = 1
                r = opt.milp(c=d[iu].astype(float),
                             constraints=opt.LinearConstraint(A, 1, 1),
                             integrality=np.ones(iu[0].size), bounds=opt.Bounds(0, 1))
                assert r.success
                tot = sum(int(d[v, res.mate[v]]) for v in range(m) if res.mate[v] > v)
                assert tot == round(r.fun)
                part, total = mm.type_part(lat, s, is_star, b)
                assert total == tot and int(part.sum()) == tot


def test_zero_sweep_decision_is_enhanced_matching():
    """Sec. III: the enhanced-matching decision is the class whose hypothesis
    has the fewest errors, an x and a z part on one qubit counting once."""
    lat = geometry.Lattice(5)
    syn, _, _ = sampler.sample(lat, 0.1, 5, np.arange(12))
    from oracle import decoder
    out = decoder.decode(5, syn, 0.1, 0, 1, chains_per_class=1, init_mode=decoder.INIT_MWPM)
    for i in range(12):
        w = geometry.weight(mm.mwpm_representatives(lat, syn[i]))
        assert out["chosen"][i] == int(np.argmin(w))
