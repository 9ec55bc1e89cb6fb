"""Parity over randomly drawn configurations (fixed seed): L, noise model,
rate, temperatures, chains, burn-in, sweeps, start mode, scan, beta*/beta_bar,
batch size and syndrome ids drawn together, so that combinations the
hand-written cases do not list are exercised too.  Every output is compared
with the oracle: integers bit-exact, FP64 within 1e-12 relative."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from oracle import decoder, geometry, sampler  # noqa: E402
from oracle import spacetime as stm  # noqa: E402

DEV = "cuda"
RTOL = 1e-12


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def draw_configs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        L = int(rng.integers(2, 26))
        noise = int(rng.integers(0, 2))
        p = float(rng.uniform(0.02, 0.3))
        K = int(rng.choice([1, 1, 2, 4]))
        chains = int(rng.integers(1, 4))
        burn = int(rng.integers(0, 3))
        sweeps = int(rng.integers(0, 4 if L <= 13 else 3))
        init = int(rng.integers(0, 2))
        random_scan = bool(rng.random() < 0.25)
        scale = float(rng.choice([0.0, 0.6, 1.0, 1.4])) if K == 1 else 0.0
        n = int(rng.integers(1, 6))
        ids = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.int64)
        out.append((L, noise, p, K, chains, burn, sweeps, init, random_scan, scale, n, ids,
                    int(rng.integers(0, 1 << 63))))
    return out


CONFIGS = draw_configs(120, 0x13022669)


@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_random_configuration(cfg):
    L, noise, p, K, chains, burn, sweeps, init, random_scan, scale, n, ids, seed = CONFIGS[cfg]
    say(f"fuzz {cfg}: L={L} noise={noise} p={p:.3f} K={K} chains={chains} burn={burn} "
        f"sweeps={sweeps} init={init} random_scan={random_scan} scale={scale} n={n}")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, seed, ids.astype(np.uint64), noise=noise)
    trace = not random_scan
    tid = torch.from_numpy(ids.astype(np.uint32).view(np.int32))
    out = mc.decode_batch(torch.from_numpy(syn).to(DEV), L, p, sweeps, seed, chains=chains,
                          n_temps=K, burn=burn, syndrome_ids=tid, want_sums=True, trace=trace,
                          init=init, noise=noise, beta_scale=scale, random_scan=random_scan)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    o = decoder.decode(L, syn, p, sweeps, seed, chains_per_class=chains, n_temps=K, burn=burn,
                       syndrome_ids=ids.astype(np.uint64), trace=trace, init_mode=init,
                       noise=noise, beta_scale=None if scale == 0.0 else scale,
                       scan=decoder.SCAN_RANDOM if random_scan else decoder.SCAN_COLOUR)
    for k in ("sum_n", "accepts", "chosen", "correction"):
        assert np.array_equal(g[k], o[k]), k
    if trace:
        assert np.array_equal(g["trace"], o["trace"]), "trace"
    np.testing.assert_allclose(g["class_prob"], o["class_prob"], rtol=RTOL, atol=0)
    np.testing.assert_allclose(g["mean_n"], o["mean_n"], rtol=RTOL, atol=0)


def draw_st_configs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        L = int(rng.integers(2, 10))
        T = int(rng.integers(1, 6))
        p = float(rng.uniform(0.01, 0.15))
        pm = float(rng.uniform(0.01, 0.2))
        chains = int(rng.integers(1, 3))
        burn = int(rng.integers(0, 2))
        sweeps = int(rng.integers(0, 3))
        n = int(rng.integers(1, 4))
        ids = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.int64)
        out.append((L, T, p, pm, chains, burn, sweeps, n, ids, int(rng.integers(0, 1 << 63))))
    return out


ST_CONFIGS = draw_st_configs(40, 0x2669)


@pytest.mark.parametrize("cfg", range(len(ST_CONFIGS)))
def test_random_spacetime_configuration(cfg):
    L, T, p, pm, chains, burn, sweeps, n, ids, seed = ST_CONFIGS[cfg]
    say(f"space-time fuzz {cfg}: L={L} T={T} p={p:.3f} pm={pm:.3f} chains={chains} "
        f"burn={burn} sweeps={sweeps} n={n}")
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, p, pm, T, seed, ids.astype(np.uint64))
    tid = torch.from_numpy(ids.astype(np.uint32).view(np.int32))
    g = mc.decode_spacetime(torch.from_numpy(obs).to(DEV), L, p, pm, sweeps, seed, chains=chains,
                            burn=burn, syndrome_ids=tid, want_sums=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = stm.decode(L, obs, p, pm, sweeps, seed, chains_per_class=chains, burn=burn,
                   syndrome_ids=ids.astype(np.uint64))
    for k in ("sum_n", "sum_m", "accepts", "chosen", "correction"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("class_prob", "mean_n", "mean_m"):
        np.testing.assert_allclose(g[k], o[k], rtol=RTOL, atol=0)
