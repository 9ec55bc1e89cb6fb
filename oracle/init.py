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
