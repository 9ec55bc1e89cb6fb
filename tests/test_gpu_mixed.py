"""Mixed batches through the plan API: every syndrome's results equal the
uniform decode of that syndrome alone (same id and parameters), bit for bit,
whatever the batch composition, launch shape or graph replay; sampled
syndromes are also replayed on the oracle."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from oracle import decoder, geometry, sampler  # noqa: E402

from paper_1302_2669_amd.inputs import mixed_workload  # noqa: E402

DEV = "cuda"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_batch(Ls, ps, sweeps, seed, chains=None, n_temps=None, burns=None, noise=None,
               scales=None):
    items, syns = [], []
    for i, (L, p, sw) in enumerate(zip(Ls, ps, sweeps)):
        lat = geometry.Lattice(int(L))
        nz = int(noise[i]) if noise is not None else 0
        syn, _, _ = sampler.sample(lat, float(p), seed, [1000 + i], noise=nz)
        syns.append(syn[0])
        items.append(dict(L=int(L), p=float(p), sweeps=int(sw),
                          burn=int(burns[i]) if burns is not None else 0,
                          chains=int(chains[i]) if chains is not None else 2,
                          n_temps=int(n_temps[i]) if n_temps is not None else 1,
                          syndrome_id=7 * i + 1, noise=nz,
                          beta_scale=float(scales[i]) if scales is not None else 0.0))
    flat = torch.from_numpy(np.concatenate(syns)).to(DEV)
    return items, syns, flat


def per_item(plan, out, i):
    a, b = plan.chain_offsets[i], plan.chain_offsets[i + 1]
    c0, c1 = plan.corr_offsets[i], plan.corr_offsets[i + 1]
    return dict(sum_n=out["sum_n"][a:b].cpu().numpy(), accepts=out["accepts"][a:b].cpu().numpy(),
                chosen=int(out["chosen"][i]), correction=out["correction"][c0:c1].cpu().numpy(),
                class_prob=out["class_prob"][i].cpu().numpy(), mean_n=out["mean_n"][i].cpu().numpy())


def uniform(item, syn, seed):
    s = torch.from_numpy(syn[None]).to(DEV)
    o = mc.decode_batch(s, item["L"], item["p"], item["sweeps"], seed, chains=item["chains"],
                        n_temps=item["n_temps"], burn=item["burn"],
                        syndrome_ids=torch.tensor([item["syndrome_id"]]), want_sums=True,
                        noise=item.get("noise", 0), beta_scale=item.get("beta_scale", 0.0))
    torch.cuda.synchronize()
    return dict(sum_n=o["sum_n"].reshape(-1).cpu().numpy(),
                accepts=o["accepts"].reshape(-1).cpu().numpy(), chosen=int(o["chosen"][0]),
                correction=o["correction"][0].cpu().numpy(),
                class_prob=o["class_prob"][0].cpu().numpy(), mean_n=o["mean_n"][0].cpu().numpy())


def same(a, b):
    for k in ("sum_n", "accepts", "correction", "class_prob", "mean_n"):
        assert np.array_equal(a[k], b[k]), k
    assert a["chosen"] == b["chosen"]


def test_mixed_plan_equals_uniform_decodes():
    say("mixed plan vs uniform decodes")
    rng = np.random.default_rng(3)
    Ls = [3, 25, 5, 17, 9, 13, 2, 20, 16, 23, 7, 11, 19, 22, 24, 21, 18, 4]
    ps = rng.uniform(0.05, 0.18, len(Ls))
    sweeps = [min(L * L, 40) for L in Ls]
    chains = rng.integers(1, 4, len(Ls))
    n_temps = [1 if i % 3 else 2 for i in range(len(Ls))]
    burns = [i % 3 for i in range(len(Ls))]
    items, syns, flat = make_batch(Ls, ps, sweeps, 11, chains, n_temps, burns)
    plan = mc.MixedPlan(items, seed=0xABCD)
    out = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        same(per_item(plan, out, i), uniform(it, syns[i], 0xABCD))
    # every launch shape gives the same bits
    base = {k: v.clone() for k, v in out.items()}
    for tun in (dict(wg_narrow=64, occ_narrow=-4, wg_wide=128, occ_wide=-2, concurrent=0),
                dict(wg_narrow=128, occ_narrow=3, wg_wide=64, occ_wide=2, concurrent=1),
                dict(wg_narrow=256, occ_narrow=0, wg_wide=256, occ_wide=1, concurrent=2)):
        plan.tuning = tun
        o2 = plan.execute(flat, want_sums=True)
        torch.cuda.synchronize()
        for k in base:
            assert torch.equal(base[k], o2[k]), (tun, k)
    plan.close()


def test_mixed_plan_against_oracle():
    say("mixed plan vs oracle")
    Ls, ps, sweeps = [5, 9, 13, 17], [0.07, 0.12, 0.15, 0.17], [6, 5, 4, 2]
    items, syns, flat = make_batch(Ls, ps, sweeps, 5)
    plan = mc.MixedPlan(items, seed=99)
    out = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        g = per_item(plan, out, i)
        o = decoder.decode(it["L"], syns[i][None], it["p"], it["sweeps"], 99,
                           chains_per_class=it["chains"], syndrome_ids=[it["syndrome_id"]])
        assert np.array_equal(g["sum_n"], o["sum_n"].reshape(-1))
        assert np.array_equal(g["accepts"], o["accepts"].reshape(-1))
        assert g["chosen"] == int(o["chosen"][0])
        assert np.array_equal(g["correction"], o["correction"][0])
        np.testing.assert_allclose(g["class_prob"], o["class_prob"][0], rtol=1e-12, atol=0)
    plan.close()


def test_graph_replays_match_eager():
    """The captured graph is replayed several times with eager work and
    synchronisations in between; every replay equals the eager execution."""
    say("graph replays")
    L, p, sw = mixed_workload(200, seed=21)
    sw = np.minimum(sw, 30)
    items, syns, flat = make_batch(L, p, sw, 8)
    plan = mc.MixedPlan(items, seed=5)
    eager = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in eager.items()}
    out = plan._outputs(flat.device, True, True)
    for rep in range(4):
        for v in out.values():
            v.fill_(0)
        plan.execute(flat, want_sums=True, graph=True, out=out)
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(eager[k], out[k]), (rep, k)
        junk = torch.randn(1 << 20, device=DEV).sum()   # eager work between replays
        torch.cuda.synchronize()
        del junk
    plan.close()


def test_autotune_keeps_results(tmp_path):
    say("autotune")
    L, p, sw = mixed_workload(300, seed=4)
    sw = np.minimum(sw, 12)
    items, syns, flat = make_batch(L, p, sw, 9)
    plan = mc.MixedPlan(items, seed=77)
    ref = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    cache = tmp_path / "tune.txt"
    t1 = plan.autotune(flat, cache_path=cache)
    assert cache.exists() and cache.read_text().strip()
    t2 = plan.autotune(flat, cache_path=cache)      # served from the cache
    assert t1 == t2 == plan.tuning
    o = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], o[k]), k
    plan.close()


def test_plan_sampler_parity():
    """Per-item depolarizing samples of a plan equal the oracle sampler's."""
    say("plan sampler")
    L, p, sw = mixed_workload(40, seed=12)
    items = [dict(L=int(l), p=float(q), sweeps=1, syndrome_id=1000 + 3 * i)
             for i, (l, q) in enumerate(zip(L, p))]
    plan = mc.MixedPlan(items, seed=1)
    syn, cls = plan.sample(0xFEED)
    torch.cuda.synchronize()
    syn, cls = syn.cpu().numpy(), cls.cpu().numpy()
    for i, it in enumerate(items):
        lat = geometry.Lattice(it["L"])
        o_syn, o_cls, _ = sampler.sample(lat, it["p"], 0xFEED, [it["syndrome_id"]])
        a, b = plan.syn_offsets[i], plan.syn_offsets[i + 1]
        assert np.array_equal(syn[a:b], o_syn[0])
        assert cls[i] == o_cls[0]
    plan.close()


def test_mixed_noise_models_equal_uniform_decodes():
    """Items of both noise models, with default and explicit beta*, in every
    kernel range of one plan: each equals its uniform decode bit for bit, in
    every launch shape."""
    say("mixed plan with both noise models")
    rng = np.random.default_rng(17)
    Ls = [3, 25, 5, 17, 9, 13, 2, 20, 16, 23, 7, 14, 19, 22, 3, 21, 18, 4, 13, 25]
    noise = [i % 2 for i in range(len(Ls))]
    ps = [float(rng.uniform(0.05, 0.15)) for _ in Ls]
    scales = [(0.0, 0.7, 1.0, 0.0, 1.3)[i % 5] for i in range(len(Ls))]
    n_temps = [2 if i % 7 == 3 else 1 for i in range(len(Ls))]
    scales = [0.0 if k == 2 else s for k, s in zip(n_temps, scales)]
    sweeps = [min(L * L, 30) for L in Ls]
    chains = rng.integers(1, 4, len(Ls))
    burns = [i % 2 for i in range(len(Ls))]
    items, syns, flat = make_batch(Ls, ps, sweeps, 23, chains, n_temps, burns, noise, scales)
    plan = mc.MixedPlan(items, seed=0x5EED)
    out = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        same(per_item(plan, out, i), uniform(it, syns[i], 0x5EED))
    base = {k: v.clone() for k, v in out.items()}
    for tun in (dict(wg_narrow=64, occ_narrow=-4, wg_wide=128, occ_wide=-2, concurrent=0),
                dict(wg_narrow=128, occ_narrow=3, wg_wide=64, occ_wide=2, concurrent=1),
                dict(wg_narrow=256, occ_narrow=0, wg_wide=256, occ_wide=1, concurrent=2)):
        plan.tuning = tun
        o2 = plan.execute(flat, want_sums=True)
        torch.cuda.synchronize()
        for k in base:
            assert torch.equal(base[k], o2[k]), (tun, k)
    plan.close()


def test_mixed_bitphase_items_against_oracle():
    say("mixed plan bit/phase items vs oracle")
    Ls, ps, sweeps = [5, 9, 14, 18, 22], [0.07, 0.1, 0.12, 0.09, 0.1], [6, 5, 3, 2, 2]
    noise, scales = [1, 1, 0, 1, 1], [0.0, 0.9, 0.0, 1.0, 0.0]
    items, syns, flat = make_batch(Ls, ps, sweeps, 6, noise=noise, scales=scales)
    plan = mc.MixedPlan(items, seed=31)
    out = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        g = per_item(plan, out, i)
        o = decoder.decode(it["L"], syns[i][None], it["p"], it["sweeps"], 31,
                           chains_per_class=it["chains"], syndrome_ids=[it["syndrome_id"]],
                           noise=it["noise"],
                           beta_scale=None if it["beta_scale"] == 0.0 else it["beta_scale"])
        assert np.array_equal(g["sum_n"], o["sum_n"].reshape(-1))
        assert np.array_equal(g["accepts"], o["accepts"].reshape(-1))
        assert g["chosen"] == int(o["chosen"][0])
        assert np.array_equal(g["correction"], o["correction"][0])
        np.testing.assert_allclose(g["class_prob"], o["class_prob"][0], rtol=1e-12, atol=0)
        np.testing.assert_allclose(g["mean_n"], o["mean_n"][0], rtol=1e-12, atol=0)
    plan.close()


def test_plan_sampler_noise_models():
    """A plan's sampler follows each item's noise model (oracle sampler)."""
    say("plan sampler, both noise models")
    L, p, _ = mixed_workload(40, seed=13)
    items = [dict(L=int(l), p=float(q), sweeps=1, syndrome_id=2000 + 5 * i, noise=i % 2)
             for i, (l, q) in enumerate(zip(L, p))]
    plan = mc.MixedPlan(items, seed=1)
    syn, cls = plan.sample(0xBEEF)
    torch.cuda.synchronize()
    syn, cls = syn.cpu().numpy(), cls.cpu().numpy()
    for i, it in enumerate(items):
        lat = geometry.Lattice(it["L"])
        o_syn, o_cls, _ = sampler.sample(lat, it["p"], 0xBEEF, [it["syndrome_id"]],
                                         noise=it["noise"])
        a, b = plan.syn_offsets[i], plan.syn_offsets[i + 1]
        assert np.array_equal(syn[a:b], o_syn[0]), i
        assert cls[i] == o_cls[0], i
    plan.close()


@pytest.mark.parametrize("noise", [0, 1])
def test_pair_mapping_equals_one_chain_mapping(noise):
    """Two chains per lane for the small codes (mcmc_tuning.pair_small):
    every output equal to the one-chain mapping's and to the uniform decodes,
    at every small L, with chain counts that make a lane's two chains belong
    to different items, classes and temperatures, and groups whose task
    count is not a multiple of a pair tile."""
    say(f"pair mapping noise={noise}")
    rng = np.random.default_rng(31 + noise)
    n = 90
    Ls = np.concatenate([np.arange(2, 9), rng.integers(2, 9, n - 10), [9, 13, 17]])
    ps = rng.uniform(0.03, 0.15, Ls.size)
    sweeps = rng.integers(0, 9, Ls.size)
    chains = rng.choice([1, 2, 3, 5], Ls.size)
    temps = rng.choice([1, 2, 4], Ls.size)
    burns = rng.integers(0, 3, Ls.size)
    items, syns, flat = make_batch(Ls, ps, sweeps, 12, chains=chains, n_temps=temps,
                                   burns=burns, noise=np.full(Ls.size, noise))
    plan = mc.MixedPlan(items, seed=0xBEEF)
    t = plan.tuning
    assert t["pair_small"] == 1           # the default
    t["pair_small"] = 0
    plan.tuning = t
    ref = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    for wg, occ in ((256, 0), (64, -2), (128, 2)):
        t.update(pair_small=1, wg_narrow=wg, occ_narrow=occ)
        plan.tuning = t
        out = plan.execute(flat, want_sums=True)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], out[k]), (wg, occ, k)
    for i in (0, 3, 6, Ls.size - 5):
        same(per_item(plan, out, i), uniform(items[i], syns[i], 0xBEEF))
    with pytest.raises(mc.McmcError):
        plan.tuning = dict(t, pair_small=2)
    # a graph recorded under the pair mapping replays it
    g = plan._outputs(flat.device, True, True)
    for _ in range(2):
        plan.execute(flat, want_sums=True, graph=True, out=g)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], g[k]), k
    plan.close()
