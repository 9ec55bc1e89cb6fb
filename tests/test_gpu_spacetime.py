"""Imperfect measurements (Sec. VI) on the GPU, through the C-ABI: sampler
and space-time chains bit-exact with the oracle (energy sums, wrong-outcome
sums, accept counts, decisions, corrections), FP64 outputs within 1e-12."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from oracle import geometry, spacetime as stm  # noqa: E402

DEV = "cuda"
RTOL = 1e-12
SEED = 0x1302266900000031


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,T,p,pm", [(2, 1, 0.2, 0.1), (3, 3, 0.1, 0.05), (5, 4, 0.05, 0.1),
                                      (13, 5, 0.03, 0.03), (25, 2, 0.05, 0.2)])
def test_sampler_parity(L, T, p, pm):
    say(f"space-time sampler L={L} T={T}")
    n = 129
    obs, cls = mc.sample_spacetime(L, T, p, pm, SEED, n, device=DEV, id_base=77)
    torch.cuda.synchronize()
    o_obs, o_cls, _, _ = stm.sample(geometry.Lattice(L), p, pm, T, SEED, np.arange(77, 77 + n))
    assert np.array_equal(obs.cpu().numpy(), o_obs)
    assert np.array_equal(cls.cpu().numpy(), o_cls)


CASES = [
    # L, T, p, pm, sweeps, burn, chains, n
    (2, 1, 0.15, 0.1, 30, 3, 2, 5),
    (2, 2, 0.15, 0.1, 30, 3, 3, 5),
    (3, 3, 0.10, 0.05, 10, 2, 2, 4),
    (4, 2, 0.12, 0.2, 8, 0, 1, 4),
    (5, 4, 0.05, 0.08, 4, 1, 2, 3),
    (9, 3, 0.06, 0.04, 2, 0, 1, 2),
    (10, 2, 0.05, 0.05, 2, 1, 1, 2),
    (11, 3, 0.04, 0.06, 1, 0, 2, 2),
    (12, 2, 0.05, 0.05, 1, 0, 1, 1),
    (13, 2, 0.04, 0.04, 1, 1, 1, 2),
    (14, 2, 0.05, 0.05, 1, 0, 1, 1),     # L >= 13: streaming-window kernel
    (15, 3, 0.04, 0.04, 2, 1, 2, 2),
    (16, 2, 0.05, 0.05, 2, 0, 1, 1),
    (17, 2, 0.05, 0.05, 1, 0, 1, 1),
    (17, 4, 0.03, 0.03, 2, 1, 1, 1),
    (18, 2, 0.04, 0.04, 1, 0, 1, 1),
    (25, 2, 0.03, 0.03, 1, 0, 1, 1),
    (3, 64, 0.05, 0.05, 1, 0, 1, 2),     # the most rounds, register kernel
    (14, 24, 0.02, 0.02, 1, 0, 1, 1),    # many rounds, streaming-window kernel
    (21, 12, 0.02, 0.02, 1, 0, 1, 1),    # many rounds, a large code
]


@pytest.mark.parametrize("L,T,p,pm,sweeps,burn,chains,n", CASES)
def test_chain_parity(L, T, p, pm, sweeps, burn, chains, n):
    say(f"space-time chains L={L} T={T} p={p} pm={pm} sweeps={sweeps} burn={burn} "
        f"chains={chains} n={n}")
    lat = geometry.Lattice(L)
    obs, _, _, _ = stm.sample(lat, p, pm, T, SEED + L, np.arange(n))
    ids = np.arange(n) * 11 + 4
    g = mc.decode_spacetime(torch.from_numpy(obs).to(DEV), L, p, pm, sweeps, SEED, chains=chains,
                            burn=burn, syndrome_ids=torch.from_numpy(ids), want_sums=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = stm.decode(L, obs, p, pm, sweeps, SEED, chains_per_class=chains, burn=burn,
                   syndrome_ids=ids)
    assert np.array_equal(g["sum_n"], o["sum_n"]), "data-error sums differ"
    assert np.array_equal(g["sum_m"], o["sum_m"]), "wrong-outcome sums differ"
    assert np.array_equal(g["accepts"], o["accepts"]), "accept counts differ"
    assert np.array_equal(g["chosen"], o["chosen"])
    assert np.array_equal(g["correction"], o["correction"])
    np.testing.assert_allclose(g["class_prob"], o["class_prob"], rtol=RTOL, atol=0)
    np.testing.assert_allclose(g["mean_n"], o["mean_n"], rtol=RTOL, atol=0)
    np.testing.assert_allclose(g["mean_m"], o["mean_m"], rtol=RTOL, atol=0)


def test_edge_histories():
    """All-quiet and all-lit histories, no counted sweep, burn-in only."""
    say("space-time edge histories")
    L, T = 3, 3
    lat = geometry.Lattice(L)
    obs = np.stack([np.zeros((T, lat.n_stab), np.uint8), np.ones((T, lat.n_stab), np.uint8)])
    for sweeps, burn in ((0, 0), (0, 2), (3, 0)):
        g = mc.decode_spacetime(torch.from_numpy(obs).to(DEV), L, 0.1, 0.1, sweeps, 3, chains=2,
                                burn=burn, want_sums=True)
        torch.cuda.synchronize()
        o = stm.decode(L, obs, 0.1, 0.1, sweeps, 3, chains_per_class=2, burn=burn)
        assert np.array_equal(g["chosen"].cpu().numpy(), o["chosen"])
        assert np.array_equal(g["sum_n"].cpu().numpy(), o["sum_n"])
        assert np.array_equal(g["correction"].cpu().numpy(), o["correction"])
        np.testing.assert_allclose(g["class_prob"].cpu().numpy(), o["class_prob"], rtol=RTOL)


def test_decoder_beats_ignoring_outcome_errors():
    """L = 5, T = 5, p = p_M = 0.03 on 2048 GPU-sampled histories: the
    space-time decoder's logical error is below that of decoding the final
    perfect round alone with the single-round decoder, and below 10%."""
    L, T, p, pm, n = 5, 5, 0.03, 0.03, 2048
    say("space-time decoder vs last round only")
    obs, cls = mc.sample_spacetime(L, T, p, pm, SEED, n, device=DEV)
    st = mc.decode_spacetime(obs, L, p, pm, 50, SEED, chains=2, burn=10, want_correction=False)
    # the accumulated error's syndrome is the last (perfect) round; its rate
    # over T intervals is about 1 - (1-p)^T
    p_eff = 1 - (1 - p) ** T
    last = mc.decode_batch(obs[:, T - 1].contiguous(), L, p_eff, 50, SEED, chains=2, burn=10,
                           want_correction=False)
    torch.cuda.synchronize()
    e_st = float((st["chosen"] != cls).float().mean())
    e_last = float((last["chosen"] != cls).float().mean())
    say(f"  logical error: space-time {e_st:.4f}, final round only {e_last:.4f}")
    assert e_st < 0.10
    assert e_st <= e_last + 0.01


def test_workload_sampled():
    """The benchmarked launch: L = 7, T = 7, p = p_M = 0.02, 4 x 4 chains,
    784 sweeps, 32768 histories sampled on the GPU and decoded in one call
    (the register-resident kernel at full residency).  The last history is
    replayed on the oracle with the same id (about a minute of CPU) and must
    match bit for bit."""
    L, T, p, pm, n, sweeps, chains = 7, 7, 0.02, 0.02, 32768, 784, 4
    say(f"space-time workload L={L} T={T} n={n} sweeps={sweeps}")
    obs, cls = mc.sample_spacetime(L, T, p, pm, SEED, n, device=DEV, id_base=7)
    ids = torch.arange(7, 7 + n, dtype=torch.int32, device=DEV)
    g = mc.decode_spacetime(obs, L, p, pm, sweeps, SEED, chains=chains, syndrome_ids=ids,
                            want_sums=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    sel = np.array([n - 1])
    o_obs = obs.cpu().numpy()[sel]
    lat = geometry.Lattice(L)
    r_obs, r_cls, _, _ = stm.sample(lat, p, pm, T, SEED, 7 + sel)
    assert np.array_equal(o_obs, r_obs) and np.array_equal(cls.cpu().numpy()[sel], r_cls)
    say("  replaying history n-1 on the oracle")
    o = stm.decode(L, o_obs, p, pm, sweeps, SEED, chains_per_class=chains, syndrome_ids=7 + sel)
    for k in ("sum_n", "sum_m", "accepts", "chosen", "correction"):
        assert np.array_equal(g[k][sel], o[k]), k
    for k in ("class_prob", "mean_n", "mean_m"):
        np.testing.assert_allclose(g[k][sel], o[k], rtol=RTOL, atol=0)
    err = float((g["chosen"] != cls.cpu().numpy()).mean())
    say(f"  logical error {err:.4f}")
    assert err < 0.08
