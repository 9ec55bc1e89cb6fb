"""Parity of the exact minimum-weight matching start (MCMC_INIT_MWPM, Sec. III)
with the oracle, through the C-ABI: class starts bit-exact at every size,
chains started from them bit-exact, the zero-sweep decision equal to the
enhanced-matching decoder, plans equal to uniform decodes."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from oracle import decoder, geometry, sampler  # noqa: E402
from oracle import matching as mm  # noqa: E402

from paper_1302_2669_amd.inputs import uniform_syndromes, SEED_METRIC  # noqa: E402

DEV = "cuda"
MWPM = mc.MCMC_INIT_MWPM


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_starts(syn, L):
    reps = mc.init_representatives(torch.from_numpy(np.ascontiguousarray(syn)).to(DEV), L,
                                   init=MWPM)
    torch.cuda.synchronize()
    return reps.cpu().numpy()


@pytest.mark.parametrize("L", [2, 3, 4, 5, 8, 9, 12, 13, 16, 17])
def test_starts_parity(L):
    """Random syndromes at three densities, empty and fully lit."""
    say(f"mwpm starts L={L}")
    lat = geometry.Lattice(L)
    syn = np.concatenate([uniform_syndromes(L, 8, seed=700 + L, density=0.3),
                          uniform_syndromes(L, 8, seed=800 + L, density=0.1),
                          uniform_syndromes(L, 4, seed=900 + L, density=0.6),
                          np.zeros((1, lat.n_stab), np.uint8),
                          np.ones((1, lat.n_stab), np.uint8)])
    reps = gpu_starts(syn, L)
    for i in range(syn.shape[0]):
        assert np.array_equal(reps[i], mm.mwpm_representatives(lat, syn[i])), i


@pytest.mark.parametrize("L,p", [(21, 0.16), (24, 0.12), (25, 0.18)])
def test_starts_parity_large_codes(L, p):
    """Codes whose problems no longer fit four to a workgroup."""
    say(f"mwpm starts L={L} p={p}")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, 0x2525 + L, np.arange(2))
    reps = gpu_starts(syn, L)
    for i in range(syn.shape[0]):
        assert np.array_equal(reps[i], mm.mwpm_representatives(lat, syn[i])), i


def test_starts_at_the_metric_point():
    """L = 13, p = 0.15: 16384 sampled syndromes in one launch; sampled ones
    replayed on the oracle, every start checked for its syndrome and class,
    and each type's weight never above the greedy start's."""
    L, p, n = 13, 0.15, 16384
    say("mwpm starts at L=13 p=0.15, 16384 syndromes")
    lat = geometry.Lattice(L)
    syn_d, _, _ = mc.sample_errors(L, p, SEED_METRIC, n, device=DEV)
    reps = mc.init_representatives(syn_d, L, init=MWPM)
    greedy = mc.init_representatives(syn_d, L, init=mc.MCMC_INIT_MATCHING)
    torch.cuda.synchronize()
    reps, greedy, syn = reps.cpu().numpy(), greedy.cpu().numpy(), syn_d.cpu().numpy()
    for i in (0, 1, 4097, 9000, n - 1):
        assert np.array_equal(reps[i], mm.mwpm_representatives(lat, syn[i])), i
    chk = np.arange(0, n, 61)
    for c in range(4):
        sub = reps[chk, c]
        assert np.array_equal(geometry.syndrome(lat, sub), syn[chk])
        assert (geometry.class_index(lat, sub) == c).all()
        for bit in (1, 2):
            ours = ((reps[chk, c] & bit) != 0).sum(axis=1)
            theirs = ((greedy[chk, c] & bit) != 0).sum(axis=1)
            assert (ours <= theirs).all()


CASES = [
    # L, p, sweeps, burn, chains, K, n, noise
    (3, 0.10, 40, 5, 2, 1, 6, 0),
    (5, 0.15, 10, 0, 2, 2, 4, 0),
    (9, 0.12, 6, 1, 3, 1, 4, 0),
    (13, 0.15, 4, 0, 2, 1, 3, 0),
    (13, 0.10, 3, 0, 1, 1, 3, 1),
    (17, 0.16, 2, 0, 1, 1, 2, 0),
    (25, 0.17, 1, 0, 1, 1, 1, 0),
]


@pytest.mark.parametrize("L,p,sweeps,burn,chains,K,n,noise", CASES)
def test_chain_parity_from_mwpm_starts(L, p, sweeps, burn, chains, K, n, noise):
    say(f"mwpm chains L={L} p={p} sweeps={sweeps} K={K} noise={noise}")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, 0x5151 + L, np.arange(n), noise=noise)
    ids = np.arange(n) * 3 + 2
    s = torch.from_numpy(syn).to(DEV)
    out = mc.decode_batch(s, L, p, sweeps, 0x77, chains=chains, n_temps=K, burn=burn,
                          syndrome_ids=torch.from_numpy(ids), want_sums=True, trace=True,
                          init=MWPM, noise=noise)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if k != "chain_state"}
    o = decoder.decode(L, syn, p, sweeps, 0x77, chains_per_class=chains, n_temps=K, burn=burn,
                       syndrome_ids=ids, trace=True, init_mode=decoder.INIT_MWPM, noise=noise)
    for k in ("sum_n", "accepts", "trace", "chosen", "correction"):
        assert np.array_equal(g[k], o[k]), k
    np.testing.assert_allclose(g["class_prob"], o["class_prob"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(g["mean_n"], o["mean_n"], rtol=1e-12, atol=0)


def test_zero_sweeps_is_the_enhanced_matching_decoder():
    """With no sweep the decision is Sec. III's: the class whose start has the
    fewest errors (an x and a z part on one qubit counting once)."""
    L, p, n = 9, 0.10, 512
    say("mwpm zero sweeps")
    lat = geometry.Lattice(L)
    syn_d, _, _ = mc.sample_errors(L, p, 0x99, n, device=DEV)
    out = mc.decode_batch(syn_d, L, p, 0, 0x99, chains=1, init=MWPM)
    reps = mc.init_representatives(syn_d, L, init=MWPM)
    torch.cuda.synchronize()
    w = geometry.weight(reps.cpu().numpy().reshape(-1, lat.n_qubits)).reshape(n, 4)
    assert np.array_equal(out["chosen"].cpu().numpy(), np.argmin(w, axis=1))
    syn = syn_d.cpu().numpy()
    for i in (0, 17, n - 1):
        ow = geometry.weight(mm.mwpm_representatives(lat, syn[i]))
        assert int(np.argmin(ow)) == int(out["chosen"][i])


def test_plan_with_mwpm_starts_equals_uniform_decodes():
    """A mixed plan sizes the start kernel's LDS for its largest code."""
    say("mwpm plan vs uniform decodes")
    Ls = [3, 25, 9, 13, 17, 5]
    items, syns = [], []
    for i, L in enumerate(Ls):
        lat = geometry.Lattice(L)
        syn, _, _ = sampler.sample(lat, 0.12, 31, [i])
        syns.append(syn[0])
        items.append(dict(L=L, p=0.12, sweeps=3, chains=2, syndrome_id=5 * i + 1))
    flat = torch.from_numpy(np.concatenate(syns)).to(DEV)
    plan = mc.MixedPlan(items, seed=0xAB, init=MWPM)
    out = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        a, b = plan.chain_offsets[i], plan.chain_offsets[i + 1]
        c0, c1 = plan.corr_offsets[i], plan.corr_offsets[i + 1]
        u = mc.decode_batch(torch.from_numpy(syns[i][None]).to(DEV), it["L"], it["p"],
                            it["sweeps"], 0xAB, chains=2,
                            syndrome_ids=torch.tensor([it["syndrome_id"]]), want_sums=True,
                            init=MWPM)
        torch.cuda.synchronize()
        assert np.array_equal(out["sum_n"][a:b].cpu().numpy(), u["sum_n"].reshape(-1).cpu().numpy())
        assert np.array_equal(out["correction"][c0:c1].cpu().numpy(),
                              u["correction"][0].cpu().numpy())
        assert int(out["chosen"][i]) == int(u["chosen"][0])
    plan.close()


def boundary_syndromes(L, counts, seed):
    """Syndromes whose busier anyon type has exactly k lit sites, for each k
    in `counts`, both ways round (the other type: a random count up to k)."""
    lat = geometry.Lattice(L)
    ns = L * (L - 1)
    rng = np.random.default_rng(seed)
    out = []
    for k in counts:
        for busy_first in (True, False):
            s = np.zeros(lat.n_stab, np.uint8)
            other = int(rng.integers(0, k + 1))
            kb, ko = (k, other) if busy_first else (other, k)
            s[rng.choice(ns, kb, replace=False)] = 1
            s[ns + rng.choice(ns, ko, replace=False)] = 1
            out.append(s)
    return np.stack(out)


# lit counts k whose larger problem (k + 2 vertices for even k, k + 3 for
# odd) falls on either side of the launch capacities 64 and 88 at L = 13
TIER_COUNTS = [20, 60, 61, 62, 63, 64, 84, 85, 86, 87, 88, 120]


def test_starts_parity_at_capacity_tiers():
    """One batch spanning the three capacity tiers (the larger two on the
    library's side stream), every start bit-exact with the oracle."""
    L = 13
    say(f"mwpm starts at the capacity tiers, L={L}")
    lat = geometry.Lattice(L)
    syn = boundary_syndromes(L, TIER_COUNTS, 0x7135)
    reps = gpu_starts(syn, L)
    for i in range(syn.shape[0]):
        assert np.array_equal(reps[i], mm.mwpm_representatives(lat, syn[i])), i


def test_plan_graph_with_mwpm_starts_replays():
    """A plan's graph holds the side-stream fork and join of the starts:
    three replays, with eager decodes and synchronisations between them, all
    equal to the eager execution."""
    L = 13
    say("mwpm plan graph replays")
    syn = boundary_syndromes(L, TIER_COUNTS, 0x7136)
    items = [dict(L=L, p=0.15, sweeps=2, chains=2, syndrome_id=100 + i)
             for i in range(syn.shape[0])]
    flat = torch.from_numpy(syn.reshape(-1)).to(DEV)
    plan = mc.MixedPlan(items, seed=0x5EED, init=MWPM)
    ref = plan.execute(flat, want_sums=True)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    out = None
    for r in range(3):
        out = plan.execute(flat, want_sums=True, graph=True, out=out)
        torch.cuda.synchronize()
        for k in ("sum_n", "chosen", "correction"):
            assert torch.equal(out[k], ref[k]), (r, k)
        # eager work of the program's own between replays
        mc.init_representatives(flat.view(len(items), -1), L, init=MWPM)
        torch.cuda.synchronize()
    plan.close()


def test_concurrent_decodes_on_two_streams():
    """Two host threads decoding with the exact starts on streams of their
    own share the library's side stream (and its lock): every output equals
    the same decode run alone."""
    import threading
    L, p, n = 13, 0.18, 4096          # at p = 0.18 about 8% of syndromes take the later tiers
    say("concurrent mwpm decodes")
    batches = [mc.sample_errors(L, p, 0x51DE + k, n, device=DEV)[0] for k in range(2)]
    ids = [torch.arange(k * n, (k + 1) * n, dtype=torch.int32, device=DEV) for k in range(2)]

    def run(k):
        return mc.decode_batch(batches[k], L, p, 4, 0xC0DE, chains=2, syndrome_ids=ids[k],
                               want_correction=True, want_sums=True, init=MWPM)

    alone = []
    for k in range(2):
        o = run(k)
        torch.cuda.synchronize()
        alone.append({key: v.clone() for key, v in o.items() if torch.is_tensor(v)})
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got, errors = [None, None], []

    def worker(k):
        try:
            with torch.cuda.stream(streams[k]):
                for _ in range(3):
                    o = run(k)
                streams[k].synchronize()
                got[k] = o
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for k in range(2):
        for key in ("chosen", "correction", "sum_n"):
            assert torch.equal(got[k][key], alone[k][key]), (k, key)
