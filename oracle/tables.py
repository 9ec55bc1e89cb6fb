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

Independent bit- and phase-flip noise (Eq. pauliChannel with
p_x = p_b(1-p_p), p_z = p_p(1-p_b), p_y = p_b p_p), here with one flip
probability q = p_b = p_p (the case Sec. IV.A's last paragraph studies): a
qubit's x part and z part are each set with probability q, independently, so a
configuration with m = (number of x parts) + (number of z parts) has relative
weight (q/(1-q))^m = exp(-beta_bar m), beta_bar = log((1-q)/q), positive for
0 < q < 1/2.  Y counts twice in m.  The paper finds the single sampling
temperature beta* = 0.85 beta_bar best for this model; with the ladder
(K > 1) the temperatures run to beta_bar as above.

Scalars are computed with Python's math module (the C library's exp/log) in
exactly this operation order.
"""

import math

import numpy as np

DEPOLARIZING = 0
BITPHASE = 1


def beta_bar(p, noise=DEPOLARIZING):
    p = float(p)
    if noise == DEPOLARIZING:
        if not (0.0 < p < 0.75):
            raise ValueError("depolarizing rate must satisfy 0 < p < 0.75")
        return -math.log((p / 3.0) / (1.0 - p))
    if noise == BITPHASE:
        if not (0.0 < p < 0.5):
            raise ValueError("bit/phase-flip rate must satisfy 0 < q < 0.5")
        return math.log((1.0 - p) / p)
    raise ValueError("unknown noise model")


def default_beta_scale(noise):
    """beta* / beta_bar of the single-temperature decoder for each model."""
    return 0.85 if noise == BITPHASE else 1.0


def beta_star(p, noise=DEPOLARIZING, beta_scale=None):
    """The single sampling temperature beta* = beta_scale * beta_bar."""
    s = default_beta_scale(noise) if beta_scale is None else float(beta_scale)
    if not (s > 0.0):
        raise ValueError("beta_scale must be positive")
    return s * beta_bar(p, noise)


def ladder(p, n_temps, noise=DEPOLARIZING, beta_scale=None):
    """beta_k for k = 1..K (K = n_temps); K = 1 gives [beta*]."""
    if n_temps == 1:
        return [beta_star(p, noise, beta_scale)]
    if beta_scale is not None and float(beta_scale) != 1.0:
        raise ValueError("the temperature ladder runs to beta_bar (beta_scale 1)")
    b = beta_bar(p, noise)
    return [(k * b) / n_temps for k in range(1, n_temps + 1)]


def acceptance_table(beta):
    """uint32 A[Delta] for Delta = 1..4 at inverse temperature beta."""
    out = []
    for d in range(1, 5):
        w = math.exp(-(beta * d))
        out.append(int(math.floor(math.ldexp(w, 32))))
    return np.array(out, dtype=np.uint64).astype(np.uint32)


def tables(p, n_temps, noise=DEPOLARIZING, beta_scale=None):
    """[K, 4] uint32 acceptance tables, row k-1 for beta_k."""
    return np.stack([acceptance_table(b) for b in ladder(p, n_temps, noise, beta_scale)])


def error_threshold(p):
    """floor(p * 2^32): a qubit is hit iff its uniform word is below this."""
    return int(math.floor(math.ldexp(float(p), 32)))
