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
        L = int(rng.integers(2, 16))
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


@pytest.mark.parametrize("plan_seed", [1, 2, 3])
def test_random_mixed_plan(plan_seed):
    """A plan of 60 randomly drawn items (every kernel range, both noise
    models, several beta*/beta_bar, temperature counts, chains, burn-in and
    sweeps, random ids): each item's results equal its uniform decode, and a
    sampled third of them equal the oracle."""
    rng = np.random.default_rng(plan_seed)
    items, syns = [], []
    for i in range(60):
        L = int(rng.integers(2, 26))
        noise = int(rng.integers(0, 2))
        p = float(rng.uniform(0.03, 0.25))
        K = int(rng.choice([1, 1, 2]))
        it = dict(L=L, p=p, noise=noise, n_temps=K, chains=int(rng.integers(1, 4)),
                  burn=int(rng.integers(0, 3)), sweeps=int(rng.integers(0, 6 if L <= 13 else 3)),
                  syndrome_id=int(rng.integers(0, 1 << 31)),
                  beta_scale=float(rng.choice([0.0, 0.8, 1.2])) if K == 1 else 0.0)
        syn, _, _ = sampler.sample(geometry.Lattice(L), p, 1000 + plan_seed, [it["syndrome_id"]],
                                   noise=noise)
        items.append(it)
        syns.append(syn[0])
    say(f"random plan {plan_seed}: {len(items)} items")
    flat = torch.from_numpy(np.concatenate(syns)).to(DEV)
    seed = 0xC0FFEE + plan_seed
    plan = mc.MixedPlan(items, seed=seed)
    out = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    for i, it in enumerate(items):
        a, b = plan.chain_offsets[i], plan.chain_offsets[i + 1]
        c0, c1 = plan.corr_offsets[i], plan.corr_offsets[i + 1]
        u = mc.decode_batch(torch.from_numpy(syns[i][None]).to(DEV), it["L"], it["p"], it["sweeps"],
                            seed, chains=it["chains"], n_temps=it["n_temps"], burn=it["burn"],
                            syndrome_ids=torch.tensor([it["syndrome_id"]]), want_sums=True,
                            noise=it["noise"], beta_scale=it["beta_scale"])
        torch.cuda.synchronize()
        assert np.array_equal(got["sum_n"][a:b], u["sum_n"].reshape(-1).cpu().numpy()), i
        assert np.array_equal(got["accepts"][a:b], u["accepts"].reshape(-1).cpu().numpy()), i
        assert got["chosen"][i] == int(u["chosen"][0]), i
        assert np.array_equal(got["correction"][c0:c1], u["correction"][0].cpu().numpy()), i
        assert np.array_equal(got["class_prob"][i], u["class_prob"][0].cpu().numpy()), i
        if i % 3 == 0:
            o = decoder.decode(it["L"], syns[i][None], it["p"], it["sweeps"], seed,
                               chains_per_class=it["chains"], n_temps=it["n_temps"],
                               burn=it["burn"], syndrome_ids=[it["syndrome_id"]],
                               noise=it["noise"],
                               beta_scale=None if it["beta_scale"] == 0.0 else it["beta_scale"])
            assert np.array_equal(got["sum_n"][a:b], o["sum_n"].reshape(-1)), i
            assert got["chosen"][i] == int(o["chosen"][0]), i
            np.testing.assert_allclose(got["class_prob"][i], o["class_prob"][0], rtol=RTOL, atol=0)
    plan.close()
