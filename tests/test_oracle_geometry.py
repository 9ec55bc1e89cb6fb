"""Pins for the oracle's lattice (Sec. II, Sec. IV.A, Sec. V).

Closed forms the paper prints, and the algebraic facts that make the layout a
distance-L planar code with one logical qubit.
"""

import json
import os

import numpy as np
import pytest

from oracle import geometry

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def gf2_rank(m):
    m = (np.array(m, dtype=np.uint8) % 2).copy()
    rank, rows, cols = 0, m.shape[0], m.shape[1]
    for c in range(cols):
        piv = None
        for r in range(rank, rows):
            if m[r, c]:
                piv = r
                break
        if piv is None:
            continue
        m[[rank, piv]] = m[[piv, rank]]
        for r in range(rows):
            if r != rank and m[r, c]:
                m[r] ^= m[rank]
        rank += 1
    return rank


@pytest.mark.parametrize("L", range(2, 26))
def test_counts_closed_form(L):
    lat = geometry.Lattice(L)
    assert lat.n_stab == 2 * L * (L - 1)             # Sec. II
    assert lat.n_qubits == lat.n_stab + 1            # Sec. IV.A
    assert lat.n_qubits == 2 * L * L - 2 * L + 1
    assert lat.sites_per_colour * 4 == lat.n_stab


def test_paper_printed_sizes():
    g = GOLDEN["n_stab_formula"]
    for L, ns in zip(g["L"], g["n_stab"]):
        assert geometry.Lattice(L).n_stab == ns
    g = GOLDEN["proof_of_principle"]
    for L, nq in zip(g["L"], g["n_qubits"]):
        assert geometry.Lattice(L).n_qubits == nq


@pytest.mark.parametrize("L", [2, 3, 4, 5, 7, 13])
def test_code_structure(L):
    lat = geometry.Lattice(L)
    Sx, Sz = lat.star_matrix(), lat.plaquette_matrix()
    w = [len(s) for s in lat.supports]
    assert set(w) <= {3, 4}
    assert sum(1 for v in w if v == 3) == 4 * (L - 1)          # boundary stabilizers
    # every star commutes with every plaquette: even overlaps
    assert not ((Sx.astype(int) @ Sz.T.astype(int)) % 2).any()
    # independent generators: one logical qubit
    assert gf2_rank(Sx) == L * (L - 1)
    assert gf2_rank(Sz) == L * (L - 1)
    assert lat.n_qubits - gf2_rank(Sx) - gf2_rank(Sz) == 1
    # every qubit is touched by at least one star and one plaquette
    assert Sx.sum(axis=0).min() >= 1 and Sz.sum(axis=0).min() >= 1
    # logical operators: Xbar (row 0) commutes with plaquettes, Zbar (column 0) with stars
    xbar = np.zeros(lat.n_qubits, dtype=int); xbar[lat.row0] = 1
    zbar = np.zeros(lat.n_qubits, dtype=int); zbar[lat.column0] = 1
    assert not ((Sz.astype(int) @ xbar) % 2).any()
    assert not ((Sx.astype(int) @ zbar) % 2).any()
    assert (xbar @ zbar) % 2 == 1                                 # anticommute
    assert len(lat.row0) == L and len(lat.column0) == L          # distance L
    # neither logical is a product of stabilizers
    assert gf2_rank(np.vstack([Sx, xbar])) == gf2_rank(Sx) + 1
    assert gf2_rank(np.vstack([Sz, zbar])) == gf2_rank(Sz) + 1


@pytest.mark.parametrize("L", range(2, 26))
def test_colours_disjoint(L):
    """Sec. V: sites of one group share no qubit, so they can be applied at once."""
    lat = geometry.Lattice(L)
    for ph in range(4):
        seen = set()
        for s in lat.phase_sites[ph]:
            for q in lat.supports[s]:
                assert q not in seen
                seen.add(q)
        assert len(lat.phase_sites[ph]) == L * (L - 1) // 2
    assert sorted(lat.draw_index.tolist()) == list(range(lat.n_stab))


@pytest.mark.parametrize("L", [3, 5, 8])
def test_class_bits(L):
    lat = geometry.Lattice(L)
    rng = np.random.default_rng(L)
    e = rng.integers(0, 4, size=(20, lat.n_qubits)).astype(np.uint8)
    c0 = geometry.class_index(lat, e)
    for s in range(lat.n_stab):       # stabilizers never change the class or the syndrome
        f = e.copy()
        f[:, lat.supports[s]] ^= (1 if lat.site_is_star[s] else 2)
        assert np.array_equal(geometry.class_index(lat, f), c0)
        assert np.array_equal(geometry.syndrome(lat, f), geometry.syndrome(lat, e))
    f = e.copy(); f[:, lat.row0] ^= 1
    assert np.array_equal(geometry.class_index(lat, f), c0 ^ 1)
    f = e.copy(); f[:, lat.column0] ^= 2
    assert np.array_equal(geometry.class_index(lat, f), c0 ^ 2)


def test_single_qubit_syndromes():
    """Sec. II: any single-qubit Pauli creates at least one anyon; in the bulk
    an X lights two plaquettes, a Z two stars and a Y all four."""
    L = 5
    lat = geometry.Lattice(L)
    q = lat.qubit_index[(4, 4)]
    for code, n_star, n_plaq in ((1, 0, 2), (2, 2, 0), (3, 2, 2)):
        e = np.zeros(lat.n_qubits, dtype=np.uint8); e[q] = code
        syn = geometry.syndrome(lat, e)
        assert syn[:lat.n_stars].sum() == n_star and syn[lat.n_stars:].sum() == n_plaq
    for q in range(lat.n_qubits):
        for code in (1, 2, 3):
            e = np.zeros(lat.n_qubits, dtype=np.uint8); e[q] = code
            assert geometry.syndrome(lat, e).sum() >= 1
