"""Pins for the oracle's Philox4x32-10 against rocRAND's engine.

rocRAND is an independent implementation (ROCm's own, compiled here from its
header for the host), so agreement on random counters and keys pins the
oracle's rounds, multipliers, key schedule and word order.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    out = tmp_path_factory.mktemp("rr") / "rocrand_philox"
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", str(out),
                    os.path.join(HERE, "rocrand_philox.cpp")], check=True,
                   capture_output=True)
    return str(out)


def _rocrand(exe, rows):
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    return np.array([[int(v) for v in line.split()] for line in res.stdout.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(rocrand_exe):
    rng = np.random.default_rng(20130212)
    n = 400
    c0 = rng.integers(0, 2**32, n, dtype=np.uint64)
    c1 = rng.integers(0, 2**29, n, dtype=np.uint64)      # keeps 4*(c1:c0) < 2^64
    c2 = rng.integers(0, 2**32, n, dtype=np.uint64)
    c3 = rng.integers(0, 2**32, n, dtype=np.uint64)
    k0 = rng.integers(0, 2**32, n, dtype=np.uint64)
    k1 = rng.integers(0, 2**32, n, dtype=np.uint64)
    # include the all-zero and small counters explicitly
    c0[:4] = [0, 1, 2, 0xFFFFFFFF]; c1[:4] = 0; c2[:4] = 0; c3[:4] = 0; k0[:4] = 0; k1[:4] = 0
    ref = _rocrand(rocrand_exe, np.stack([c0, c1, c2, c3, k0, k1], axis=1))
    got = np.stack(philox.philox4x32_10(c0, c1, c2, c3, k0, k1), axis=1).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_decoder_counter_layout(rocrand_exe):
    """The exact counters the chain and sampler use, for a 64-bit seed."""
    seed = 0x1302266900000002
    k0, k1 = philox.seed_key(seed)
    assert (k0, k1) == (0x00000002, 0x13022669)
    rows = []
    for d in range(0, 24, 4):
        rows.append([d >> 2, 7, 12345, int(philox.chain_ctr3(3, 1, 5)), k0, k1])
    rows.append([5, 0, 99, philox.sampler_ctr3(), k0, k1])
    ref = _rocrand(rocrand_exe, rows)
    r = np.array(rows, dtype=np.uint64)
    got = np.stack(philox.philox4x32_10(*[r[:, i] for i in range(6)]), axis=1).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_uniformity_sanity():
    """Coarse statistical check: bit balance of a million words."""
    c0 = np.arange(250000, dtype=np.uint64)
    w = np.stack(philox.philox4x32_10(c0, 1, 2, 3, 4, 5)).reshape(-1)
    bits = np.unpackbits(w.view(np.uint8)).mean()
    assert abs(bits - 0.5) < 5e-4
