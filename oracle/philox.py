"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
as 1, 2, 3", SC'11), written from that paper's definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One call maps a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1) to
four 32-bit words.  Each of the ten rounds multiplies c0 and c2 by the two
round multipliers, keeps both halves of each 64-bit product, and mixes the
high halves with the other two words and the round key; between rounds the key
is advanced by the two Weyl constants.  The decoder takes k0/k1 from the low
and high halves of its 64-bit seed.

Counter layout used by the decoder (the paper prescribes no generator; this
keying makes every draw a function of logical coordinates only):

  chain move    : (d >> 2, sweep, syndrome_id, 0<<30 | cls<<28 | temp<<20 | chain),
                  draw d of the sweep uses word d & 3
  error sampler : (q >> 1, 0, sample_id, 1<<30), qubit q uses words 2(q&1), 2(q&1)+1
  random scan   : (t >> 1, sweep, syndrome_id, 2<<30 | cls<<28 | temp<<20 | chain),
                  step t of the sweep uses words 2(t&1) (site) and 2(t&1)+1 (accept)

Arithmetic is done on uint64 numpy arrays and masked to 32 bits, vectorised
over any number of counters.
"""

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF

DOMAIN_CHAIN = 0
DOMAIN_SAMPLER = 1
DOMAIN_RANDOM_SCAN = 2


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Inputs broadcast; returns four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = (v.copy() for v in (c0, c1, c2, c3))
    for rnd in range(10):
        p0 = c0 * np.uint64(M0)            # < 2^64: exact in uint64
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def seed_key(seed):
    seed = int(seed) & ((1 << 64) - 1)
    return seed & MASK, seed >> 32


def chain_ctr3(cls, temp, chain, domain=DOMAIN_CHAIN):
    """Fourth counter word of a chain-move draw; arguments broadcast."""
    cls = np.asarray(cls, dtype=np.uint64)
    temp = np.asarray(temp, dtype=np.uint64)
    chain = np.asarray(chain, dtype=np.uint64)
    return ((np.uint64(domain) << np.uint64(30)) | (cls << np.uint64(28))
            | (temp << np.uint64(20)) | chain)


def sampler_ctr3():
    return DOMAIN_SAMPLER << 30
