"""Planar surface code of distance L (Sec. II, Fig. code; Sec. V for the colouring).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (the figure of the code is not available, so the orientation is a
reading of Sec. II: sigma^x stabilizers absorb their anyons at the top/bottom
boundaries, sigma^z stabilizers at the left/right ones):

* A (2L-1) x (2L-1) grid of cells (r, c).  Data qubits sit on the cells with
  r + c even; there are n_q = 2L^2 - 2L + 1 of them, numbered row-major.
* Stars (sigma^x stabilizers) sit on cells (r odd, c even): an (L-1) x L array
  indexed (i, j) = ((r-1)/2, c/2).  Plaquettes (sigma^z stabilizers) sit on
  cells (r even, c odd): an L x (L-1) array indexed (i, j) = (r/2, (c-1)/2).
  A stabilizer's support is its in-grid 4-neighbourhood (3 or 4 qubits), so
  there are n_stab = 2L(L-1) stabilizers (Sec. II) and n_q = n_stab + 1
  (Sec. IV.A).
* Site numbering: stars row-major (0 .. L(L-1)-1), then plaquettes row-major.
* Colours: phase 0 = stars with i+j even, 1 = stars with i+j odd,
  2 = plaquettes with i+j even, 3 = plaquettes with i+j odd.  Sites of one
  colour never share a qubit; these are the paper's four groups of
  non-overlapping regions (Sec. V) with one stabilizer per region.
* Pauli code per qubit: bit 0 = x part, bit 1 = z part (I=0, X=1, Z=2, Y=3).
* Logical lines (Sec. III: a class is fixed by error parities along lines that
  join opposite boundaries): bx = parity of the x parts on column 0, bz =
  parity of the z parts on row 0.  Class index = bx + 2*bz
  (0 = I, 1 = X-bar, 2 = Z-bar, 3 = Y-bar).  X-bar is X on every qubit of
  row 0, Z-bar is Z on every qubit of column 0.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Lattice:
    L: int
    side: int = field(init=False)
    n_qubits: int = field(init=False)
    n_stab: int = field(init=False)
    n_stars: int = field(init=False)
    sites_per_colour: int = field(init=False)
    qubit_rc: np.ndarray = field(init=False)        # [n_q, 2] grid cell of each qubit
    qubit_index: dict = field(init=False)           # (r, c) -> qubit
    site_rc: np.ndarray = field(init=False)         # [n_stab, 2] grid cell of each site
    site_is_star: np.ndarray = field(init=False)    # [n_stab] bool
    site_ij: np.ndarray = field(init=False)         # [n_stab, 2] (i, j) within its type
    site_colour: np.ndarray = field(init=False)     # [n_stab] 0..3
    supports: list = field(init=False)              # per site: list of qubit indices
    phase_sites: list = field(init=False)           # per colour: ascending site list
    draw_index: np.ndarray = field(init=False)      # [n_stab] phase*S + rank in phase
    column0: np.ndarray = field(init=False)         # qubits on column 0
    row0: np.ndarray = field(init=False)            # qubits on row 0

    def __post_init__(self):
        L = self.L
        if L < 2:
            raise ValueError("distance L must be at least 2")
        self.side = 2 * L - 1
        cells = [(r, c) for r in range(self.side) for c in range(self.side)
                 if (r + c) % 2 == 0]
        self.qubit_rc = np.array(cells, dtype=np.int64)
        self.qubit_index = {rc: q for q, rc in enumerate(cells)}
        self.n_qubits = len(cells)

        rcs, is_star, ijs, colours = [], [], [], []
        for i in range(L - 1):                 # stars
            for j in range(L):
                rcs.append((2 * i + 1, 2 * j))
                is_star.append(True)
                ijs.append((i, j))
                colours.append((i + j) % 2)
        for i in range(L):                     # plaquettes
            for j in range(L - 1):
                rcs.append((2 * i, 2 * j + 1))
                is_star.append(False)
                ijs.append((i, j))
                colours.append(2 + (i + j) % 2)
        self.site_rc = np.array(rcs, dtype=np.int64)
        self.site_is_star = np.array(is_star, dtype=bool)
        self.site_ij = np.array(ijs, dtype=np.int64)
        self.site_colour = np.array(colours, dtype=np.int64)
        self.n_stab = len(rcs)
        self.n_stars = L * (L - 1)
        self.sites_per_colour = L * (L - 1) // 2

        self.supports = []
        for (r, c) in rcs:
            sup = []
            for (dr, dc) in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                rr, cc = r + dr, c + dc
                if 0 <= rr < self.side and 0 <= cc < self.side:
                    sup.append(self.qubit_index[(rr, cc)])
            self.supports.append(sup)

        self.phase_sites = [[s for s in range(self.n_stab) if self.site_colour[s] == ph]
                            for ph in range(4)]
        self.draw_index = np.zeros(self.n_stab, dtype=np.int64)
        for ph in range(4):
            for rank, s in enumerate(self.phase_sites[ph]):
                self.draw_index[s] = ph * self.sites_per_colour + rank

        self.column0 = np.array([self.qubit_index[(r, 0)] for r in range(0, self.side, 2)])
        self.row0 = np.array([self.qubit_index[(0, c)] for c in range(0, self.side, 2)])

    # --- check matrices -------------------------------------------------
    def star_matrix(self):
        """[n_stars, n_q] 0/1: which qubits each star acts on."""
        m = np.zeros((self.n_stars, self.n_qubits), dtype=np.uint8)
        for s in range(self.n_stars):
            m[s, self.supports[s]] = 1
        return m

    def plaquette_matrix(self):
        """[n_plaquettes, n_q] 0/1: which qubits each plaquette acts on."""
        m = np.zeros((self.n_stab - self.n_stars, self.n_qubits), dtype=np.uint8)
        for s in range(self.n_stars, self.n_stab):
            m[s - self.n_stars, self.supports[s]] = 1
        return m


def pauli_x(codes):
    return np.asarray(codes) & 1


def pauli_z(codes):
    return (np.asarray(codes) >> 1) & 1


def weight(codes):
    """Number of non-identity single-qubit factors (Y counts once, Sec. III)."""
    return (np.asarray(codes) != 0).sum(axis=-1)


def flip_count(codes):
    """Number of bit flips plus phase flips (x parts + z parts; Y counts
    twice): the energy of the independent bit/phase-flip model."""
    codes = np.asarray(codes).astype(np.int64)
    return pauli_x(codes).sum(axis=-1) + pauli_z(codes).sum(axis=-1)


def energy(codes, noise):
    """The chain energy of a noise model: weight (0, depolarizing) or
    flip_count (1, independent bit/phase flips)."""
    return flip_count(codes) if noise == 1 else weight(codes)


def syndrome(lat, codes):
    """Anyon configuration of an error (Sec. II).

    A star (sigma^x) is lit iff an odd number of its qubits carry a z part
    (Z or Y); a plaquette (sigma^z) is lit iff an odd number carry an x part.
    `codes` is [..., n_q]; returns uint8 [..., n_stab] in site order.
    """
    codes = np.asarray(codes)
    x = pauli_x(codes).astype(np.int64)
    z = pauli_z(codes).astype(np.int64)
    out = np.zeros(codes.shape[:-1] + (lat.n_stab,), dtype=np.uint8)
    for s in range(lat.n_stab):
        part = z if lat.site_is_star[s] else x
        out[..., s] = part[..., lat.supports[s]].sum(axis=-1) % 2
    return out


def class_index(lat, codes):
    """Logical class of an error or correction: bx + 2*bz (see module doc)."""
    codes = np.asarray(codes)
    bx = pauli_x(codes)[..., lat.column0].sum(axis=-1) % 2
    bz = pauli_z(codes)[..., lat.row0].sum(axis=-1) % 2
    return (bx + 2 * bz).astype(np.int64)
