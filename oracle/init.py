"""One syndrome-consistent representative per logical class.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper starts each class's chain from a minimum-weight configuration found
by enhanced matching (Sec. III, Sec. IV); the decoder here starts from a
canonical configuration instead (the paper's conclusion leaves the effect of
other starting states open).  Construction:

* every lit plaquette at cell (r, c) is explained by X on (r, 0), (r, 2), ...,
  (r, c-1): a string to the left boundary;
* every lit star at cell (r, c) is explained by Z on (0, c), (2, c), ...,
  (r-1, c): a string to the top boundary;
* strings are multiplied together (x and z parts XOR).

That configuration E0 has the measured syndrome.  The representative of class
k is E0 * Xbar^a * Zbar^b with a = bx(E0) xor (k & 1), b = bz(E0) xor (k >> 1),
where Xbar = X on row 0 and Zbar = Z on column 0; it has the same syndrome
(both logicals commute with every stabilizer) and class k.
"""

import numpy as np

from . import geometry


def canonical(lat, syn):
    """uint8 [n_q] configuration E0 with syndrome `syn` (uint8 [n_stab])."""
    x = np.zeros(lat.n_qubits, dtype=np.uint8)
    z = np.zeros(lat.n_qubits, dtype=np.uint8)
    for s in range(lat.n_stab):
        if not syn[s]:
            continue
        r, c = (int(v) for v in lat.site_rc[s])
        if lat.site_is_star[s]:
            for rr in range(0, r, 2):
                z[lat.qubit_index[(rr, c)]] ^= 1
        else:
            for cc in range(0, c, 2):
                x[lat.qubit_index[(r, cc)]] ^= 1
    return (x | (z << 1)).astype(np.uint8)


def representatives(lat, syn):
    """uint8 [4, n_q]: row k is a configuration of class k with syndrome `syn`."""
    e0 = canonical(lat, syn)
    cls0 = int(geometry.class_index(lat, e0))
    bx0, bz0 = cls0 & 1, cls0 >> 1
    out = np.zeros((4, lat.n_qubits), dtype=np.uint8)
    for k in range(4):
        e = e0.copy()
        if bx0 ^ (k & 1):
            e[lat.row0] ^= 1          # X-bar
        if bz0 ^ (k >> 1):
            e[lat.column0] ^= 2       # Z-bar
        out[k] = e
    return out


# ---------------------------------------------------------------------------
# Matching start (Sec. III, Sec. IV): the paper starts every class's chain
# from a minimum-weight configuration of that class, found by matching each
# anyon type separately and then forcing the other parity ("enhanced"
# matching).  The decoder approximates the matching greedily:
#
# * anyons of one type are the lit sites of that type, in ascending index;
#   the distance of two anyons is their Manhattan distance |di| + |dj| (the
#   number of qubits on the path below); an anyon's boundary distance is
#   j+1 / L-1-j (plaquettes: left / right) or i+1 / L-1-i (stars: top /
#   bottom), the nearer side winning ties towards left / top;
# * for d = 1, 2, ...: every still-free anyon a in ascending order takes the
#   first free partner b > a at distance d, else its boundary if that is at
#   distance d;
# * the class parity of a type equals the number of its anyons matched to the
#   left (plaquettes) or top (stars) boundary, mod 2.  The other parity is
#   reached by the cheapest single change: move one boundary-matched anyon to
#   the other side, or split one pair into one left/top and one right/bottom
#   match; with no anyon at all, the logical string itself;
# * paths: plaquette pair (i1,j1) < (i2,j2): X on (2i1, 2j+2) for j between
#   j1 and j2, then on (2i+1, 2j2+1) for i1 <= i < i2; left: X on (2i, 0..2j);
#   right: X on (2i, 2j+2..2L-2).  Star pair: Z on (2i+2, 2j1) for
#   i1 <= i < i2, then on (2i2+1, 2j+1) for j between j1 and j2; top:
#   Z on (0..2i, 2j); bottom: Z on (2i+2..2L-2, 2j).
# ---------------------------------------------------------------------------

def _greedy_type(L, anyons, is_star):
    """anyons: list of (i, j).  Returns (pairs, bmatch) with bmatch a list of
    (a, side) for boundary matches, side 0 = left/top, 1 = right/bottom."""
    k = len(anyons)

    def bd(a):
        i, j = anyons[a]
        near, far = (j + 1, L - 1 - j) if not is_star else (i + 1, L - 1 - i)
        return (near, 0) if near <= far else (far, 1)

    def dist(a, b):
        return abs(anyons[a][0] - anyons[b][0]) + abs(anyons[a][1] - anyons[b][1])

    free = [True] * k
    pairs, bmatch = [], []
    d = 1
    while any(free):
        for a in range(k):
            if not free[a]:
                continue
            for b in range(a + 1, k):
                if free[b] and dist(a, b) == d:
                    free[a] = free[b] = False
                    pairs.append((a, b))
                    break
            if free[a]:
                dd, side = bd(a)
                if dd == d:
                    free[a] = False
                    bmatch.append((a, side))
        d += 1
    return pairs, bmatch


def _flip_parity(L, anyons, is_star, pairs, bmatch):
    """Cheapest single change that flips the type's class parity, returned as
    (pairs, bmatch, add_logical)."""
    def side_dist(a, side):
        i, j = anyons[a]
        if is_star:
            return i + 1 if side == 0 else L - 1 - i
        return j + 1 if side == 0 else L - 1 - j

    def dist(a, b):
        return abs(anyons[a][0] - anyons[b][0]) + abs(anyons[a][1] - anyons[b][1])

    best = None  # (delta, kind, index, option)
    for idx, (a, side) in enumerate(bmatch):
        delta = side_dist(a, 1 - side) - side_dist(a, side)
        if best is None or delta < best[0]:
            best = (delta, "b", idx, 0)
    for idx, (a, b) in enumerate(pairs):
        for opt, (sa, sb) in enumerate(((0, 1), (1, 0))):
            delta = side_dist(a, sa) + side_dist(b, sb) - dist(a, b)
            if best is None or delta < best[0]:
                best = (delta, "p", idx, opt)
    if best is None:
        return list(pairs), list(bmatch), True
    _, kind, idx, opt = best
    pairs2, bm2 = list(pairs), list(bmatch)
    if kind == "b":
        a, side = bm2[idx]
        bm2[idx] = (a, 1 - side)
    else:
        a, b = pairs2.pop(idx)
        sa, sb = ((0, 1), (1, 0))[opt]
        bm2 = bm2 + [(a, sa), (b, sb)]
    return pairs2, bm2, False


def _paint(lat, part, anyons, is_star, pairs, bmatch, logical):
    """XOR the matching's paths into `part` (x parts for plaquettes, z parts
    for stars)."""
    L = lat.L
    qi = lat.qubit_index

    def flip(r, c):
        part[qi[(r, c)]] ^= 1

    for (a, b) in pairs:
        (i1, j1), (i2, j2) = anyons[a], anyons[b]
        if not is_star:
            for j in range(min(j1, j2), max(j1, j2)):
                flip(2 * i1, 2 * j + 2)
            for i in range(min(i1, i2), max(i1, i2)):
                flip(2 * i + 1, 2 * j2 + 1)
        else:
            for i in range(min(i1, i2), max(i1, i2)):
                flip(2 * i + 2, 2 * j1)
            for j in range(min(j1, j2), max(j1, j2)):
                flip(2 * i2 + 1, 2 * j + 1)
    for (a, side) in bmatch:
        i, j = anyons[a]
        if not is_star:
            cols = range(0, 2 * j + 1, 2) if side == 0 else range(2 * j + 2, 2 * L - 1, 2)
            for c in cols:
                flip(2 * i, c)
        else:
            rows = range(0, 2 * i + 1, 2) if side == 0 else range(2 * i + 2, 2 * L - 1, 2)
            for r in rows:
                flip(r, 2 * j)
    if logical:
        for q in (lat.row0 if not is_star else lat.column0):
            part[q] ^= 1


def matching_representatives(lat, syn):
    """uint8 [4, n_q]: greedy-matching start of every class (see above)."""
    L = lat.L
    syn = np.asarray(syn)
    parts = {}
    for is_star in (False, True):
        rng = range(0, lat.n_stars) if is_star else range(lat.n_stars, lat.n_stab)
        anyons = [tuple(int(v) for v in lat.site_ij[s]) for s in rng if syn[s]]
        pairs, bmatch = _greedy_type(L, anyons, is_star)
        base_par = sum(1 for (_, side) in bmatch if side == 0) % 2
        fp, fb, flog = _flip_parity(L, anyons, is_star, pairs, bmatch)
        for par, (pp, bb, lg) in ((base_par, (pairs, bmatch, False)),
                                  (1 - base_par, (fp, fb, flog))):
            part = np.zeros(lat.n_qubits, dtype=np.uint8)
            _paint(lat, part, anyons, is_star, pp, bb, lg)
            parts[(is_star, par)] = part
    out = np.zeros((4, lat.n_qubits), dtype=np.uint8)
    for k in range(4):
        out[k] = parts[(False, k & 1)] | (parts[(True, k >> 1)] << 1)
    return out
