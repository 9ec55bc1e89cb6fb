"""Parity of the HIP path with the CPU oracle, through the C-ABI.

Integer work (errors, syndromes, class starts, chain trajectories, energy sums,
accept counts, final states, decisions, corrections) must be bit-exact; FP64
class probabilities and means must agree to 1e-12 relative.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from oracle import decoder, geometry, init, sampler  # noqa: E402

from paper_1302_2669_amd.inputs import (uniform_syndromes, SEED_SMALL, SEED_L9,  # noqa: E402
                                        SEED_METRIC, SEED_L25)

DEV = "cuda"
RTOL = 1e-12


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_np(d):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in d.items()}


def gpu_decode(L, syn, p, sweeps, seed, chains=1, K=1, burn=0, ids=None, trace=True,
               chain_state=True, init=mc.MCMC_INIT_MATCHING):
    s = torch.from_numpy(np.ascontiguousarray(syn, dtype=np.uint8)).to(DEV)
    tid = None if ids is None else torch.from_numpy(np.asarray(ids, dtype=np.int64))
    out = mc.decode_batch(s, L, p, sweeps, seed, chains=chains, n_temps=K, burn=burn,
                          syndrome_ids=tid, want_sums=True, trace=trace, chain_state=chain_state,
                          init=init)
    res = to_np({k: v for k, v in out.items() if k != "chain_state"})
    if chain_state:
        st, w = mc.unpack_chain_state(out["chain_state"], syn.shape[0], L, p, sweeps, seed, chains,
                                      K, burn)
        res["states"], res["n_final"] = st.cpu().numpy(), w.cpu().numpy()
    return res


def assert_parity(g, o, check_trace=True):
    assert np.array_equal(g["sum_n"], o["sum_n"]), "energy sums differ"
    assert np.array_equal(g["accepts"], o["accepts"]), "accept counts differ"
    if check_trace:
        assert np.array_equal(g["trace"], o["trace"]), "trajectories differ"
    if "states" in g:
        assert np.array_equal(g["states"], o["states"]), "final states differ"
        assert np.array_equal(g["n_final"], o["n_final"]), "final weights differ"
    assert np.array_equal(g["chosen"], o["chosen"]), "decisions differ"
    assert np.array_equal(g["correction"], o["correction"]), "corrections differ"
    np.testing.assert_allclose(g["class_prob"], o["class_prob"], rtol=RTOL, atol=0)
    np.testing.assert_allclose(g["mean_n"], o["mean_n"], rtol=RTOL, atol=0)


# ---------------------------------------------------------------- sampler
@pytest.mark.parametrize("L,p", [(2, 0.3), (3, 0.1), (9, 0.15), (13, 0.15), (16, 0.05),
                                 (17, 0.18), (25, 0.17)])
def test_sampler_parity(L, p):
    say(f"sampler L={L} p={p}")
    n = 257
    syn, cls, err = mc.sample_errors(L, p, SEED_L9, n, device=DEV, id_base=1000,
                                     want_errors=True)
    torch.cuda.synchronize()
    lat = geometry.Lattice(L)
    o_syn, o_cls, o_err = sampler.sample(lat, p, SEED_L9, np.arange(1000, 1000 + n))
    assert np.array_equal(err.cpu().numpy(), o_err)
    assert np.array_equal(syn.cpu().numpy(), o_syn)
    assert np.array_equal(cls.cpu().numpy(), o_cls)


# ---------------------------------------------------------------- class starts
@pytest.mark.parametrize("mode", [mc.MCMC_INIT_CANONICAL, mc.MCMC_INIT_MATCHING])
@pytest.mark.parametrize("L", [2, 3, 4, 5, 9, 13, 15, 16, 17, 24, 25])
def test_init_parity(L, mode):
    say(f"init L={L} mode={mode}")
    lat = geometry.Lattice(L)
    start = init.matching_representatives if mode == mc.MCMC_INIT_MATCHING else init.representatives
    syn = np.concatenate([uniform_syndromes(L, 30, seed=L),
                          uniform_syndromes(L, 30, seed=L + 100, density=0.08)])
    syn[0] = 0
    syn[1] = 1
    reps = mc.init_representatives(torch.from_numpy(syn).to(DEV), L, init=mode).cpu().numpy()
    for i in range(syn.shape[0]):
        assert np.array_equal(reps[i], start(lat, syn[i])), i


# ---------------------------------------------------------------- chains
CASES = [
    # L, p, sweeps, burn, chains, K, n
    (2, 0.15, 40, 5, 3, 1, 6),
    (3, 0.10, 50, 10, 2, 1, 8),
    (3, 0.10, 20, 0, 1, 4, 5),
    (4, 0.05, 15, 3, 2, 2, 5),
    (5, 0.18, 12, 2, 2, 1, 6),
    (6, 0.30, 8, 0, 1, 1, 5),
    (9, 0.15, 6, 1, 4, 1, 4),
    (13, 0.15, 4, 1, 2, 1, 3),
    (16, 0.12, 2, 0, 1, 2, 2),
    (17, 0.16, 2, 1, 1, 1, 2),
    (21, 0.10, 2, 0, 1, 1, 2),
    (25, 0.17, 2, 0, 1, 1, 2),
]


@pytest.mark.parametrize("L,p,sweeps,burn,chains,K,n", CASES)
@pytest.mark.parametrize("mode", [mc.MCMC_INIT_MATCHING, mc.MCMC_INIT_CANONICAL])
def test_chain_parity(L, p, sweeps, burn, chains, K, n, mode):
    say(f"chains L={L} p={p} sweeps={sweeps} burn={burn} chains={chains} K={K} n={n} init={mode}")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, SEED_L9 + L, np.arange(n))
    ids = np.arange(n) * 7 + 3
    g = gpu_decode(L, syn, p, sweeps, SEED_L9, chains, K, burn, ids=ids, init=mode)
    o = decoder.decode(L, syn, p, sweeps, SEED_L9, chains_per_class=chains, n_temps=K, burn=burn,
                       syndrome_ids=ids, trace=True, init_mode=mode)
    o["n_final"] = o["n_final"].astype(np.int32)
    assert_parity(g, o)


TI_CASES = [
    # L, p, sweeps, burn, chains, K, n: the paper's 21 temperatures (K = 20, Sec. IV.A)
    # at the small workload's size and budget, at larger L for a few sweeps, and the
    # largest ladder the library takes (K = 64)
    (3, 0.10, 2000, 0, 1, 20, 4),
    (9, 0.12, 6, 1, 2, 20, 3),
    (13, 0.15, 3, 0, 1, 20, 2),
    (5, 0.08, 3, 1, 1, 64, 2),
]


@pytest.mark.parametrize("L,p,sweeps,burn,chains,K,n", TI_CASES)
def test_thermodynamic_integration_parity(L, p, sweeps, burn, chains, K, n):
    """Every temperature's trajectory, sums and accept counts bit-exact; the
    Simpson class probabilities within 1e-12 relative."""
    say(f"TI chains L={L} p={p} sweeps={sweeps} burn={burn} chains={chains} K={K} n={n}")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, SEED_SMALL + L, np.arange(n))
    ids = np.arange(n) * 5 + 1
    g = gpu_decode(L, syn, p, sweeps, SEED_SMALL, chains, K, burn, ids=ids)
    o = decoder.decode(L, syn, p, sweeps, SEED_SMALL, chains_per_class=chains, n_temps=K,
                       burn=burn, syndrome_ids=ids, trace=True)
    o["n_final"] = o["n_final"].astype(np.int32)
    assert_parity(g, o)


def test_edge_syndromes():
    """Empty and fully lit syndromes, zero counted sweeps, burn-in only."""
    say("edge syndromes")
    for L, p in ((3, 0.1), (13, 0.15)):
        lat = geometry.Lattice(L)
        syn = np.stack([np.zeros(lat.n_stab, np.uint8), np.ones(lat.n_stab, np.uint8)])
        for sweeps, burn in ((0, 0), (0, 3), (3, 0)):
            g = gpu_decode(L, syn, p, sweeps, 99, 2, 1, burn)
            o = decoder.decode(L, syn, p, sweeps, 99, chains_per_class=2, burn=burn, trace=True)
            o["n_final"] = o["n_final"].astype(np.int32)
            assert_parity(g, o)


def test_batch_composition_invariance():
    """Outputs of a syndrome depend only on (bytes, id, params)."""
    say("batch composition")
    L, p = 9, 0.1
    syn = uniform_syndromes(L, 300, seed=5, density=0.2)
    ids = np.arange(300)
    full = gpu_decode(L, syn, p, 5, 11, 2, 1, 0, ids=ids, trace=False, chain_state=False)
    sel = np.array([299, 0, 150, 7])
    part = gpu_decode(L, syn[sel], p, 5, 11, 2, 1, 0, ids=ids[sel], trace=False, chain_state=False)
    for k in ("sum_n", "accepts", "chosen", "correction", "class_prob", "mean_n"):
        assert np.array_equal(full[k][sel], part[k])


def test_resume_is_bit_exact():
    say("resume")
    L, p, chains, sweeps, burn, n = 9, 0.15, 2, 30, 5, 16
    syn = uniform_syndromes(L, n, seed=7, density=0.25)
    s = torch.from_numpy(syn).to(DEV)
    whole = mc.decode_batch(s, L, p, sweeps, 5, chains=chains, burn=burn, want_sums=True,
                            chain_state=True)
    # first 12 absolute sweeps, then the rest from the saved state
    first = mc.decode_batch(s, L, p, 12 - burn, 5, chains=chains, burn=burn, want_sums=True,
                            chain_state=True)
    second = mc.decode_batch(s, L, p, sweeps, 5, chains=chains, burn=burn, want_sums=True,
                             resume_from=(first["chain_state"], 12))
    a = to_np({k: v for k, v in whole.items() if k != "chain_state"})
    b = to_np({k: v for k, v in second.items() if k != "chain_state"})
    for k in ("sum_n", "accepts", "chosen", "correction", "class_prob", "mean_n"):
        assert np.array_equal(a[k], b[k]), k
    sa = mc.unpack_chain_state(whole["chain_state"], n, L, p, sweeps, 5, chains, 1, burn)
    sb = mc.unpack_chain_state(second["chain_state"], n, L, p, sweeps, 5, chains, 1, burn)
    assert torch.equal(sa[0], sb[0]) and torch.equal(sa[1], sb[1])


# ---------------------------------------------------------------- workloads
def test_small_workload_against_oracle():
    """L = 3, p = 0.10, 1000 samples, 4 classes x 1 chain, 2000 sweeps: every
    output equals the oracle's on the same samples."""
    L, p, n, sweeps = 3, 0.10, 1000, 2000
    say("small workload L=3 p=0.10 n=1000 sweeps=2000")
    lat = geometry.Lattice(L)
    syn, _, _ = sampler.sample(lat, p, SEED_SMALL, np.arange(n))
    g = gpu_decode(L, syn, p, sweeps, SEED_SMALL, 1, 1, 0, trace=False)
    o = decoder.decode(L, syn, p, sweeps, SEED_SMALL, chains_per_class=1)
    o["n_final"] = o["n_final"].astype(np.int32)
    assert_parity(g, o, check_trace=False)


@pytest.mark.parametrize("p", [0.05, 0.10, 0.15])
def test_l9_workload_sampled(p):
    """L = 9, 4 x 4 chains, 81 sweeps: the GPU decodes 10^4 samples at once;
    an evenly spaced subset is replayed on the oracle with full trajectories."""
    L, n, sweeps, chains = 9, 10000, 81, 4
    say(f"L9 workload p={p}")
    syn_d, cls_d, _ = mc.sample_errors(L, p, SEED_L9, n, device=DEV)
    out = mc.decode_batch(syn_d, L, p, sweeps, SEED_L9, chains=chains, want_sums=True)
    g = to_np(out)
    syn = syn_d.cpu().numpy()
    pick = np.linspace(0, n - 1, 12).astype(np.int64)
    lat = geometry.Lattice(L)
    o_syn, _, _ = sampler.sample(lat, p, SEED_L9, pick)
    assert np.array_equal(syn[pick], o_syn)
    o = decoder.decode(L, o_syn, p, sweeps, SEED_L9, chains_per_class=chains, syndrome_ids=pick)
    for k in ("sum_n", "accepts", "chosen", "correction"):
        assert np.array_equal(g[k][pick], o[k]), k
    np.testing.assert_allclose(g["class_prob"][pick], o["class_prob"], rtol=RTOL, atol=0)
    fail = (g["chosen"] != cls_d.cpu().numpy()).mean()
    say(f"  logical error rate L=9 p={p}: {fail:.4f}")


def test_metric_workload_sampled():
    """L = 13, p = 0.15, 4 x 4 chains, 169 sweeps, launched exactly as the
    benchmark launches it; sampled syndromes replayed on the oracle."""
    L, p, sweeps, chains, n = 13, 0.15, 169, 4, 16384
    say("metric workload L=13 p=0.15")
    syn_d, cls_d, _ = mc.sample_errors(L, p, SEED_METRIC, n, device=DEV)
    out = mc.decode_batch(syn_d, L, p, sweeps, SEED_METRIC, chains=chains, want_sums=True)
    g = to_np(out)
    pick = np.array([0, 4097, n - 1])
    lat = geometry.Lattice(L)
    o_syn, _, _ = sampler.sample(lat, p, SEED_METRIC, pick)
    o = decoder.decode(L, o_syn, p, sweeps, SEED_METRIC, chains_per_class=chains,
                       syndrome_ids=pick)
    for k in ("sum_n", "accepts", "chosen", "correction"):
        assert np.array_equal(g[k][pick], o[k]), k
    np.testing.assert_allclose(g["class_prob"][pick], o["class_prob"], rtol=RTOL, atol=0)
    # properties that hold at any size: probabilities normalised, decision is
    # the integer-key argmin, every correction has the input syndrome and the
    # chosen class
    assert np.allclose(g["class_prob"].sum(axis=1), 1.0, rtol=1e-13)
    key = g["sum_n"].sum(axis=(2, 3))
    assert np.array_equal(np.argmin(key, axis=1), g["chosen"])
    syn = syn_d.cpu().numpy()
    chk = np.arange(0, n, 997)
    assert np.array_equal(geometry.syndrome(lat, g["correction"][chk]), syn[chk])
    assert np.array_equal(geometry.class_index(lat, g["correction"][chk]), g["chosen"][chk])
    say(f"  logical error rate L=13 p=0.15: {(g['chosen'] != cls_d.cpu().numpy()).mean():.4f}")


@pytest.mark.parametrize("p", [0.16, 0.17, 0.18])
def test_near_threshold_workload_checkpointed(p):
    """L = 25, 2 x 10^4 samples, 4 classes x 8 chains, up to 4 L^2 sweeps,
    run as one batch in checkpointed segments (resume): 25, L^2, 2 L^2, 3 L^2,
    4 L^2.  The first segment is replayed on the oracle for sampled syndromes
    (every chain: S, A, final states); the full length is checked against a
    one-shot decode of a sub-batch and by properties that hold at any size.
    The logical error at each checkpoint is the error vs sweep-count curve."""
    L, n, chains = 25, 20000, 8
    say(f"near-threshold workload L=25 p={p}")
    syn_d, cls_d, _ = mc.sample_errors(L, p, SEED_L25, n, device=DEV)
    first = mc.decode_batch(syn_d, L, p, 25, SEED_L25, chains=chains, want_sums=True,
                            chain_state=True)
    cs = first["chain_state"]
    if p == 0.17:
        g = to_np({k: v for k, v in first.items() if k != "chain_state"})
        st, nf = mc.unpack_chain_state(cs, n, L, p, 25, SEED_L25, chains)
        st, nf = st.cpu().numpy(), nf.cpu().numpy()
        pick = np.array([0, n - 1])
        lat = geometry.Lattice(L)
        o_syn, _, _ = sampler.sample(lat, p, SEED_L25, pick)
        assert np.array_equal(syn_d.cpu().numpy()[pick], o_syn)
        o = decoder.decode(L, o_syn, p, 25, SEED_L25, chains_per_class=chains, syndrome_ids=pick)
        for k in ("sum_n", "accepts", "chosen", "correction"):
            assert np.array_equal(g[k][pick], o[k]), k
        assert np.array_equal(st[pick], o["states"])
        assert np.array_equal(nf[pick], o["n_final"])
    prev, curve = 25, []
    for m in (1, 2, 3, 4):
        total = m * L * L
        out = mc.decode_batch(syn_d, L, p, total, SEED_L25, chains=chains, want_sums=True,
                              resume_from=(cs, prev))
        prev = total
        err = float((out["chosen"] != cls_d).float().mean())
        curve.append((total, err))
    say(f"  logical error vs sweeps at L=25 p={p}: {curve}")
    g = to_np({k: v for k, v in out.items() if k != "chain_state"})
    sub = 96
    one = to_np(mc.decode_batch(syn_d[:sub], L, p, 4 * L * L, SEED_L25, chains=chains,
                                want_sums=True))
    for k in ("sum_n", "accepts", "chosen", "correction", "class_prob", "mean_n"):
        assert np.array_equal(g[k][:sub], one[k]), k
    assert np.allclose(g["class_prob"].sum(axis=1), 1.0, rtol=1e-13)
    key = g["sum_n"].sum(axis=(2, 3))
    assert np.array_equal(np.argmin(key, axis=1), g["chosen"])
    lat = geometry.Lattice(L)
    chk = np.arange(0, n, 1999)
    syn = syn_d.cpu().numpy()
    assert np.array_equal(geometry.syndrome(lat, g["correction"][chk]), syn[chk])
    assert np.array_equal(geometry.class_index(lat, g["correction"][chk]), g["chosen"][chk])
