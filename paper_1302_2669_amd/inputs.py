"""Seeded synthetic inputs shared by the tests (oracle and HIP path alike)
and the benchmark.

Holds none of the decoder's arithmetic: only numpy's own generator (PCG64)
for uniformly random syndrome bits (every bit string is a valid planar-code
syndrome), the fixed seeds of the workloads, and the mixed-size workload
descriptor.  Depolarizing samples themselves come from each side's own
sampler, keyed by (seed, sample id).
"""

import numpy as np

# 64-bit Philox keys of the workloads (decode and sampling use the same seed)
SEED_SMALL = 0x1302266900000001      # L = 3, p = 0.10, 1000 samples, 4 x 1 chains, 2000 sweeps
SEED_L9 = 0x1302266900000002         # L = 9, p in {0.05, 0.10, 0.15}, 4 x 4 chains, 81 sweeps
SEED_METRIC = 0x1302266900000013     # L = 13, p = 0.15, 4 x 4 chains, 169 sweeps
SEED_L25 = 0x1302266900000004        # L = 25, p in {0.16, 0.17, 0.18}, 4 x 8 chains, up to 4 L^2


def n_stab(L):
    return 2 * L * (L - 1)


def uniform_syndromes(L, n, seed, density=0.5):
    rng = np.random.default_rng(seed)
    return (rng.random((n, n_stab(L))) < density).astype(np.uint8)


def mixed_workload(n, seed, Ls=(5, 7, 9, 11, 13, 15, 17, 19, 21, 23, 25), p_lo=0.05, p_hi=0.18):
    """(L [n], p [n], sweeps [n] = L^2) for the mixed-size batch."""
    rng = np.random.default_rng(seed)
    L = rng.choice(np.asarray(Ls), size=n)
    p = p_lo + (p_hi - p_lo) * rng.random(n)
    return L.astype(np.int32), p, (L * L).astype(np.int32)


def cnn_init(L, seed, channels=32):
    """Initial gate-network parameters as one float32 vector, in the order
    W1 [32][9][3], b1 [32], W2 [32][9][32], b2, W3 [32][9][32], b3,
    Wh [7][L*L*32], bh [7]: He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    shapes = [(channels, 9, 3), (channels,), (channels, 9, channels), (channels,),
              (channels, 9, channels), (channels,), (7, L * L * channels), (7,)]
    parts = []
    for k, shape in enumerate(shapes):
        if k % 2 == 1:
            parts.append(np.zeros(shape, dtype=np.float32).reshape(-1))
        else:
            fan_in = int(np.prod(shape[1:]))
            parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), size=shape).astype(np.float32).reshape(-1))
    return np.concatenate(parts)


def uniform_rates(n, seed, lo=0.05, hi=0.18):
    """n depolarizing rates uniform in [lo, hi), float32 (the network's input
    precision; the same values, widened, serve the float64 decoder)."""
    rng = np.random.default_rng(seed)
    return (lo + (hi - lo) * rng.random(n)).astype(np.float32)


def cnn_targets(n, seed):
    """Synthetic training targets: class distributions [n][4] (Dirichlet(1))
    and budget labels [n] in 0..2."""
    rng = np.random.default_rng(seed)
    t = rng.dirichlet(np.ones(4), size=n).astype(np.float32)
    b = rng.integers(0, 3, size=n).astype(np.int32)
    return t, b
