"""Pins for exact enumeration (Eq. partitionFunction, Eq. avgDefi, Eq. main)."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import enumerate as en
from oracle import geometry, tables


def syndrome_from_index(lat, v):
    return np.array([(v >> b) & 1 for b in range(lat.n_stab)], dtype=np.uint8)


@pytest.fixture(scope="module")
def brute3():
    return en.brute_force_histograms(geometry.Lattice(3))


def test_stabilizer_enumeration_equals_brute_force_L2():
    lat = geometry.Lattice(2)
    bf = en.brute_force_histograms(lat)
    assert bf.sum() == 4 ** lat.n_qubits
    for v in range(1 << lat.n_stab):
        assert np.array_equal(en.class_histograms(lat, syndrome_from_index(lat, v)), bf[v])


def test_stabilizer_enumeration_equals_brute_force_L3(brute3):
    lat = geometry.Lattice(3)
    assert brute3.sum() == 4 ** lat.n_qubits
    rng = np.random.default_rng(3)
    for v in list(range(8)) + rng.integers(0, 1 << lat.n_stab, 120).tolist():
        assert np.array_equal(en.class_histograms(lat, syndrome_from_index(lat, v)), brute3[v])


@pytest.mark.parametrize("L", [2, 3, 4])
def test_class_sizes_and_infinite_temperature(L):
    """Each class holds 2^n_stab configurations (so log Z_E(0) = n_stab log 2,
    Eq. main) and their mean weight is exactly (3/4) n_q (Sec. IV.A)."""
    lat = geometry.Lattice(L)
    rng = np.random.default_rng(L)
    for _ in range(2 if L == 4 else 6):
        syn = rng.integers(0, 2, lat.n_stab).astype(np.uint8)
        h = en.class_histograms(lat, syn)
        assert (h.sum(axis=1) == 2 ** lat.n_stab).all()
        w = np.arange(lat.n_qubits + 1)
        # exact rational comparison: sum w h = (3/4) n_q 2^n_stab
        assert ((h * w).sum(axis=1) * 4 == 3 * lat.n_qubits * 2 ** lat.n_stab).all()


@pytest.mark.parametrize("p", [0.05, 0.1, 0.15])
def test_thermodynamic_integration_identity(p):
    """Eq. main, checked on the exact enumeration with adaptive quadrature."""
    lat = geometry.Lattice(3)
    syn = syndrome_from_index(lat, 0b010011000101)
    h = en.class_histograms(lat, syn)
    bb = tables.beta_bar(p)
    lz = en.log_z(h, bb)
    for e in range(4):
        integral, _ = integrate.quad(lambda b: en.mean_n(h[e:e + 1], b)[0], 0.0, bb,
                                     epsabs=1e-12, epsrel=1e-12)
        assert -integral + lat.n_stab * math.log(2) == pytest.approx(lz[e], abs=1e-9)


def test_mean_decreasing_in_beta():
    """Sec. IV.A: <n>_{beta,E} decreases monotonically with beta."""
    lat = geometry.Lattice(3)
    h = en.class_histograms(lat, syndrome_from_index(lat, 0b100100100001))
    betas = np.linspace(0, 6, 61)
    m = np.array([en.mean_n(h, b) for b in betas])
    assert (np.diff(m, axis=0) < 0).all()


@pytest.mark.parametrize("L", [2, 3, 4])
def test_empty_syndrome(L):
    """Minimum weights 0, L, L, 2L-1 and the Xbar <-> Zbar transpose symmetry."""
    lat = geometry.Lattice(L)
    h = en.class_histograms(lat, np.zeros(lat.n_stab, dtype=np.uint8))
    minw = [int(np.nonzero(h[e])[0][0]) for e in range(4)]
    assert minw == [0, L, L, 2 * L - 1]
    assert np.array_equal(h[1], h[2])
    pr = en.class_probabilities(h, tables.beta_bar(0.1))
    assert pr[1] == pytest.approx(pr[2], rel=1e-13)


def test_total_probability_brute_force(brute3):
    """Summing (p/3)^w (1-p)^(n_q-w) over every error gives 1."""
    lat = geometry.Lattice(3)
    p = 0.1
    w = np.arange(lat.n_qubits + 1)
    pw = (p / 3) ** w * (1 - p) ** (lat.n_qubits - w)
    assert (brute3 * pw).sum() == pytest.approx(1.0, rel=1e-12)
