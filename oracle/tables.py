"""Inverse temperatures and the integer acceptance table.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Eq. (betaBar): for depolarizing noise a chain with n single-qubit errors has
  relative weight ((p/3)/(1-p))^n = exp(-beta_bar n), so
  beta_bar = -log((p/3)/(1-p)); it is positive for 0 < p < 3/4.
* Sec. IV.A sets the single sampling temperature to beta* = beta_bar.
* The integration variant (Sec. IV.A, 21 equidistant temperatures between 0
  and beta_bar) uses beta_k = k*beta_bar/K for k = 1..K; beta_0 = 0 is never
  sampled because <n> there is known in closed form (3/4 of the qubits).
* Metropolis acceptance (Sec. IV): a move with Delta n > 0 is taken with
  probability exp(-beta Delta n).  It is realised with a uniform 32-bit word u
  as  u < A[Delta],  A[Delta] = floor(2^32 exp(-beta Delta)), Delta = 1..4.
  Moves with Delta <= 0 are always taken.

Scalars are computed with Python's math module (the C library's exp/log) in
exactly this operation order.
"""

import math

import numpy as np


def beta_bar(p):
    p = float(p)
    if not (0.0 < p < 0.75):
        raise ValueError("depolarizing rate must satisfy 0 < p < 0.75")
    return -math.log((p / 3.0) / (1.0 - p))


def ladder(p, n_temps):
    """beta_k for k = 1..K (K = n_temps); K = 1 gives [beta_bar]."""
    b = beta_bar(p)
    return [(k * b) / n_temps for k in range(1, n_temps + 1)]


def acceptance_table(beta):
    """uint32 A[Delta] for Delta = 1..4 at inverse temperature beta."""
    out = []
    for d in range(1, 5):
        w = math.exp(-(beta * d))
        out.append(int(math.floor(math.ldexp(w, 32))))
    return np.array(out, dtype=np.uint64).astype(np.uint32)


def tables(p, n_temps):
    """[K, 4] uint32 acceptance tables, row k-1 for beta_k."""
    return np.stack([acceptance_table(b) for b in ladder(p, n_temps)])


def error_threshold(p):
    """floor(p * 2^32): a qubit is hit iff its uniform word is below this."""
    return int(math.floor(math.ldexp(float(p), 32)))
