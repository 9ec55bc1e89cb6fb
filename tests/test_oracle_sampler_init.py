"""Pins for the depolarizing sampler (Eq. pauliChannel with p/3 each) and the
class representatives."""

import numpy as np
import pytest

from oracle import geometry, init, sampler


def test_sampler_rates():
    lat = geometry.Lattice(9)
    p = 0.15
    e = sampler.sample_errors(lat, p, 0xABCDEF, np.arange(4000))
    n = e.size
    hit = (e != 0).mean()
    assert abs(hit - p) < 5 * np.sqrt(p * (1 - p) / n)
    for code in (1, 2, 3):
        frac = (e == code).mean()
        assert abs(frac - p / 3) < 5 * np.sqrt(p / 3 * (1 - p / 3) / n)
    # distinct ids give distinct errors; same id reproduces
    e2 = sampler.sample_errors(lat, p, 0xABCDEF, np.array([3, 0]))
    assert np.array_equal(e2[0], e[3]) and np.array_equal(e2[1], e[0])


def test_syndrome_is_linear():
    lat = geometry.Lattice(5)
    e = sampler.sample_errors(lat, 0.3, 7, np.arange(50))
    syn = geometry.syndrome(lat, e)
    acc = np.zeros_like(syn)
    for q in range(lat.n_qubits):
        single = np.zeros_like(e); single[:, q] = e[:, q]
        acc ^= geometry.syndrome(lat, single)
    assert np.array_equal(acc, syn)


@pytest.mark.parametrize("L", [2, 3, 4, 6, 9, 13])
def test_representatives(L):
    lat = geometry.Lattice(L)
    rng = np.random.default_rng(L)
    syns = rng.integers(0, 2, size=(30, lat.n_stab)).astype(np.uint8)
    for syn in syns:
        reps = init.representatives(lat, syn)
        assert np.array_equal(geometry.syndrome(lat, reps), np.broadcast_to(syn, (4, lat.n_stab)))
        assert geometry.class_index(lat, reps).tolist() == [0, 1, 2, 3]


@pytest.mark.parametrize("L", [2, 3, 5, 13, 25])
def test_empty_syndrome_representatives(L):
    """No anyons: the class representatives are I, Xbar, Zbar and Xbar*Zbar,
    of weights 0, L, L and 2L - 1 (Xbar and Zbar overlap in one qubit, which
    carries Y)."""
    lat = geometry.Lattice(L)
    reps = init.representatives(lat, np.zeros(lat.n_stab, dtype=np.uint8))
    assert geometry.weight(reps).tolist() == [0, L, L, 2 * L - 1]


def test_all_syndromes_small():
    lat = geometry.Lattice(3)
    for v in range(1 << lat.n_stab):
        syn = np.array([(v >> b) & 1 for b in range(lat.n_stab)], dtype=np.uint8)
        reps = init.representatives(lat, syn)
        assert np.array_equal(geometry.syndrome(lat, reps)[0], syn)


@pytest.mark.parametrize("L", [2, 3, 4, 5, 8, 13, 25])
def test_matching_representatives_valid(L):
    lat = geometry.Lattice(L)
    rng = np.random.default_rng(100 + L)
    for density in (0.05, 0.3, 0.7):
        syns = (rng.random((10, lat.n_stab)) < density).astype(np.uint8)
        for syn in syns:
            reps = init.matching_representatives(lat, syn)
            assert np.array_equal(geometry.syndrome(lat, reps), np.broadcast_to(syn, (4, lat.n_stab)))
            assert geometry.class_index(lat, reps).tolist() == [0, 1, 2, 3]


@pytest.mark.parametrize("L", [3, 5, 9])
def test_matching_recovers_single_errors(L):
    """Any single-qubit error is matched back exactly: its anyons are adjacent
    (or next to a boundary), so the start of the error's own class is the
    error itself, of weight 1."""
    lat = geometry.Lattice(L)
    for q in range(lat.n_qubits):
        for code in (1, 2, 3):
            e = np.zeros(lat.n_qubits, dtype=np.uint8)
            e[q] = code
            syn = geometry.syndrome(lat, e)
            reps = init.matching_representatives(lat, syn)
            c = int(geometry.class_index(lat, e))
            assert np.array_equal(reps[c], e), (q, code)


@pytest.mark.parametrize("L", [2, 3, 5, 13])
def test_matching_empty_syndrome(L):
    lat = geometry.Lattice(L)
    reps = init.matching_representatives(lat, np.zeros(lat.n_stab, dtype=np.uint8))
    assert geometry.weight(reps).tolist() == [0, L, L, 2 * L - 1]


def test_matching_start_against_exact_minimum_on_two_error_syndromes():
    """Every two-error syndrome at L = 3 (all qubit pairs, every Pauli on each):
    each class start is a member of its class, so it is never below that
    class's exact minimum weight (enumeration).  The greedy start reaches the
    exact minimum of the error's own class when the two errors are one X and
    one Z (at most one anyon of each type); with three or more anyons of one
    type (XX, YY, XY, ... pairs) the greedy pairing can miss it."""
    from oracle import enumerate as en
    lat = geometry.Lattice(3)
    xz_hits = xz_total = 0
    for q1 in range(lat.n_qubits):
        for q2 in range(q1 + 1, lat.n_qubits):
            for c1 in (1, 2, 3):
                for c2 in (1, 2, 3):
                    e = np.zeros(lat.n_qubits, dtype=np.uint8)
                    e[q1], e[q2] = c1, c2
                    syn = geometry.syndrome(lat, e)
                    h = en.class_histograms(lat, syn)
                    w = geometry.weight(init.matching_representatives(lat, syn))
                    exact_min = np.array([int(np.nonzero(h[k])[0][0]) for k in range(4)])
                    assert (w >= exact_min).all(), (q1, q2, c1, c2)
                    if (c1, c2) == (1, 2):
                        c = int(geometry.class_index(lat, e))
                        xz_hits += int(w[c] == exact_min[c])
                        xz_total += 1
    assert xz_hits == xz_total
