"""Exact class partition functions by enumeration (Eq. partitionFunction,
Eq. avgDefi) for small codes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Z_E(beta) sums exp(-beta n) over every configuration of class E with the given
syndrome: a class representative times every one of the 2^n_stab stabilizer
products (Sec. IV.A).  Star products only touch x parts and plaquette products
only z parts, so the class is the product set
    {x_rep ^ star span} x {z_rep ^ plaquette span}
and n = popcount(x | z).  The weight histogram h_E[n] gives Z_E(beta),
<n>_{beta,E} and P(E) = Z_E(beta_bar) / sum_E' Z_E'(beta_bar) exactly.
Feasible for L <= 4 (2^12 x 2^12 pairs per class at L = 4).

With noise = 1 (independent bit/phase flips) the energy is
popcount(x) + popcount(z) instead, histogrammed over 0..2 n_q.

`brute_force_histograms` is an independent route to the same numbers: it runs
over all 4^n_q Pauli errors, groups them by (syndrome, class) and histograms
their weights.  It uses neither the representatives nor the stabilizer span.
"""

import math

import numpy as np

from . import geometry, init


def _mask(bits):
    m = 0
    for q in bits:
        m |= 1 << int(q)
    return m


def _span(generators):
    """All 2^m XOR combinations of the given bitmasks, uint64."""
    arr = np.zeros(1, dtype=np.uint64)
    for g in generators:
        arr = np.concatenate([arr, arr ^ np.uint64(g)])
    return arr


def class_histograms(lat, syn, noise=0):
    """int64 [4, n_q + 1] (noise 0) or [4, 2 n_q + 1] (noise 1): number of
    class-E configurations of each energy."""
    if lat.n_qubits > 63:
        raise ValueError("enumeration limited to n_q <= 63")
    stars = [_mask(lat.supports[s]) for s in range(lat.n_stars)]
    plaqs = [_mask(lat.supports[s]) for s in range(lat.n_stars, lat.n_stab)]
    xs0, zs0 = _span(stars), _span(plaqs)
    reps = init.representatives(lat, np.asarray(syn, dtype=np.uint8))
    nb = (2 * lat.n_qubits if noise == 1 else lat.n_qubits) + 1
    hist = np.zeros((4, nb), dtype=np.int64)
    for e in range(4):
        xr = _mask(np.nonzero(reps[e] & 1)[0])
        zr = _mask(np.nonzero(reps[e] & 2)[0])
        zs = zs0 ^ np.uint64(zr)
        zc = np.bitwise_count(zs).astype(np.int64)
        for x in (xs0 ^ np.uint64(xr)):
            if noise == 1:
                w = zc + int(np.bitwise_count(x))
            else:
                w = np.bitwise_count(zs | x).astype(np.int64)
            hist[e] += np.bincount(w, minlength=nb)
    return hist


def brute_force_histograms(lat, noise=0):
    """int64 [2^n_stab, 4, n_q + 1] over all 4^n_q errors, indexed by the
    syndrome read as a little-endian bit string in site order; with noise = 1
    the last axis is x-part count + z-part count, 0..2 n_q."""
    nq = lat.n_qubits
    if nq > 13:
        raise ValueError("brute force limited to n_q <= 13")
    n_st = lat.n_stars
    allv = np.arange(1 << nq, dtype=np.uint64)

    def parity_bits(vals, site_range):
        out = np.zeros(vals.shape, dtype=np.int64)
        for bit, s in enumerate(site_range):
            m = np.uint64(_mask(lat.supports[s]))
            out |= ((np.bitwise_count(vals & m) & 1).astype(np.int64) << bit)
        return out

    # z parts light stars (sites 0..n_st-1), x parts light plaquettes.
    star_syn = parity_bits(allv, range(n_st))                   # from z
    plaq_syn = parity_bits(allv, range(n_st, lat.n_stab))       # from x
    bz = (np.bitwise_count(allv & np.uint64(_mask(lat.row0))) & 1).astype(np.int64)
    bx = (np.bitwise_count(allv & np.uint64(_mask(lat.column0))) & 1).astype(np.int64)
    n_syn = 1 << lat.n_stab
    nb = (2 * nq if noise == 1 else nq) + 1
    hist = np.zeros((n_syn, 4, nb), dtype=np.int64)
    zcount = np.bitwise_count(allv).astype(np.int64)
    for x in range(1 << nq):
        if noise == 1:
            w = zcount + bin(x).count("1")
        else:
            w = np.bitwise_count(allv | np.uint64(x)).astype(np.int64)
        syn_idx = star_syn | (int(plaq_syn[x]) << n_st)
        cls = int(bx[x]) + 2 * bz
        flat = (syn_idx * 4 + cls) * nb + w
        hist += np.bincount(flat, minlength=n_syn * 4 * nb).reshape(n_syn, 4, nb)
    return hist


def log_z(hist, beta):
    """log Z_E(beta) for each class from weight histograms [4, n_q+1]."""
    w = np.arange(hist.shape[-1], dtype=np.float64)
    out = []
    for h in hist:
        nz = h > 0
        a = np.log(h[nz].astype(np.float64)) - beta * w[nz]
        m = a.max()
        out.append(m + math.log(np.exp(a - m).sum()))
    return np.array(out)


def mean_n(hist, beta):
    """<n>_{beta,E} for each class (Eq. avgDefi with f(n) = n)."""
    w = np.arange(hist.shape[-1], dtype=np.float64)
    out = []
    for h in hist:
        nz = h > 0
        a = np.log(h[nz].astype(np.float64)) - beta * w[nz]
        p = np.exp(a - a.max())
        out.append(float((p * w[nz]).sum() / p.sum()))
    return np.array(out)


def class_probabilities(hist, beta):
    lz = log_z(hist, beta)
    e = np.exp(lz - lz.max())
    return e / e.sum()
