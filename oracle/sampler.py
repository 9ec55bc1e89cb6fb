"""Depolarizing error sampling, syndrome and true class (Eq. pauliChannel,
Sec. IV: X, Y and Z each with probability p/3, nothing with 1 - p, i.i.d.).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Draw rule for qubit q of sample s (seed split into the Philox key):
  (w0, w1, w2, w3) = Philox4x32-10(ctr = (q >> 1, 0, s, 1 << 30), key)
  u0, u1 = w[2(q & 1)], w[2(q & 1) + 1]
  the qubit is hit iff u0 < floor(p 2^32); the Pauli is then
  t = (u1 * 3) >> 32 in {0, 1, 2} -> X, Y, Z.

Independent bit/phase flips with rate q (noise = 1; Eq. pauliChannel with
p_b = p_p = q): the same two words, x part iff u0 < floor(q 2^32), z part iff
u1 < floor(q 2^32).
"""

import numpy as np

from . import geometry, philox, tables

# t = 0, 1, 2 -> X (code 1), Y (code 3), Z (code 2)
_TYPE_TO_CODE = np.array([1, 3, 2], dtype=np.uint8)


def sample_errors(lat, p, seed, sample_ids, noise=0):
    """uint8 [n, n_q] Pauli codes for the given sample ids."""
    sample_ids = np.asarray(sample_ids, dtype=np.uint64)
    k0, k1 = philox.seed_key(seed)
    q = np.arange(lat.n_qubits, dtype=np.uint64)
    w = philox.philox4x32_10(q[None, :] >> np.uint64(1), 0, sample_ids[:, None],
                             philox.sampler_ctr3(), k0, k1)
    w = np.stack(w, axis=-1).astype(np.uint64)            # [n, n_q, 4]
    half = (q & np.uint64(1)).astype(np.int64) * 2
    u0 = np.take_along_axis(w, half[None, :, None], axis=-1)[..., 0]
    u1 = np.take_along_axis(w, half[None, :, None] + 1, axis=-1)[..., 0]
    thr = np.uint64(tables.error_threshold(p))
    if noise == 1:
        return ((u0 < thr).astype(np.uint8) | ((u1 < thr).astype(np.uint8) << 1))
    hit = u0 < thr
    t = ((u1 * np.uint64(3)) >> np.uint64(32)).astype(np.int64)
    return np.where(hit, _TYPE_TO_CODE[t], 0).astype(np.uint8)


def sample(lat, p, seed, sample_ids, noise=0):
    """(syndromes uint8 [n, n_stab], true_class int64 [n], errors uint8 [n, n_q])."""
    e = sample_errors(lat, p, seed, sample_ids, noise)
    return geometry.syndrome(lat, e), geometry.class_index(lat, e), e
