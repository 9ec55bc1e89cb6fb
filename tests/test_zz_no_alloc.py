"""mcmc_decode_batch_noalloc (the decode with its scratch in a static device
buffer, for callers that cannot allocate) called through the C-ABI: two calls
in a row, the second smaller, each equal to mcmc_decode_batch with a
caller-allocated workspace on the same inputs; a decode needing more scratch
than the buffer holds is rejected before anything runs."""

import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from paper_1302_2669_amd import _lib  # noqa: E402

DEV = "cuda"
SCRATCH_BYTES = 64 << 20


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def noalloc_decode(syn, ids, L, p, sweeps, seed, chains, n_temps, burn, init):
    n = int(syn.shape[0])
    nq, _ = mc.geometry(L)
    prm = mc.make_params(L, p, sweeps, seed, chains, n_temps, burn, init=init)
    out = {
        "class_prob": torch.full((n, 4), -1.0, dtype=torch.float64, device=DEV),
        "mean_n": torch.full((n, 4), -1.0, dtype=torch.float64, device=DEV),
        "chosen": torch.full((n,), 9, dtype=torch.uint8, device=DEV),
        "correction": torch.full((n, nq), 9, dtype=torch.uint8, device=DEV),
        "sum_n": torch.full((n, 4, n_temps, chains), -1, dtype=torch.int64, device=DEV),
        "accepts": torch.full((n, 4, n_temps, chains), -1, dtype=torch.int64, device=DEV),
    }
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = _lib._lib().mcmc_decode_batch_noalloc(
        ptr(syn), ptr(ids), n, ctypes.byref(prm), ptr(out["class_prob"]), ptr(out["mean_n"]),
        ptr(out["sum_n"]), ptr(out["accepts"]), ptr(out["chosen"]), ptr(out["correction"]),
        None, None, stream)
    return st, out


def reference(syn, ids, L, p, sweeps, seed, chains, n_temps, burn, init):
    return mc.decode_batch(syn, L, p, sweeps, seed, chains=chains, n_temps=n_temps, burn=burn,
                           syndrome_ids=ids, want_sums=True, init=init)


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def test_noalloc_decode_equals_workspace_decode_twice():
    calls = [
        # L, p, sweeps, seed, chains, K, burn, n, init
        (13, 0.15, 12, 0x1301, 4, 1, 2, 4096, mc.MCMC_INIT_MWPM),
        (9, 0.10, 8, 0x0902, 2, 2, 1, 700, mc.MCMC_INIT_MATCHING),
    ]
    for L, p, sweeps, seed, chains, K, burn, n, init in calls:
        say(f"noalloc decode L={L} n={n} chains={chains} K={K} init={init}")
        syn, _, _ = mc.sample_errors(L, p, seed, n, device=DEV)
        ids = torch.arange(3, 3 + 5 * n, 5, dtype=torch.int32, device=DEV)
        st, got = noalloc_decode(syn, ids, L, p, sweeps, seed, chains, K, burn, init)
        assert st == 0, _lib.STATUS.get(st, st)
        want = reference(syn, ids, L, p, sweeps, seed, chains, K, burn, init)
        torch.cuda.synchronize()
        for k in ("chosen", "correction", "sum_n", "accepts", "class_prob", "mean_n"):
            assert torch.equal(got[k], want[k]), k


def test_noalloc_rejects_a_decode_larger_than_its_scratch():
    L, chains, n = 13, 4, 70000
    prm = mc.make_params(L, 0.15, 10, 1, chains)
    assert mc.workspace_size(prm, n) > SCRATCH_BYTES
    syn = torch.zeros((n, 2 * L * (L - 1)), dtype=torch.uint8, device=DEV)
    chosen = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
    prob = torch.empty((n, 4), dtype=torch.float64, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = _lib._lib().mcmc_decode_batch_noalloc(ptr(syn), None, n, ctypes.byref(prm), ptr(prob),
                                               None, None, None, ptr(chosen), None, None, None,
                                               stream)
    assert st == -5  # MCMC_EWORKSPACE, before anything is enqueued
    torch.cuda.synchronize()
    assert bool((chosen == 9).all())
