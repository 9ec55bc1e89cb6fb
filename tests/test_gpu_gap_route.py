"""The start-weight gap route through the C-ABI: class start weights equal
to the weights of the oracle's starts, the fitted threshold table equal to
the oracle's fit on the same seeded labelled samples, and the gated
decoder's routes equal to the network's route combined with the oracle's
gap rule, every output against the plain entry point at its route's budget.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from paper_1302_2669_amd import gate  # noqa: E402
from paper_1302_2669_amd.inputs import uniform_syndromes  # noqa: E402
from oracle import cnn, geometry, init  # noqa: E402
from oracle import matching as mm  # noqa: E402
from test_gpu_gated import check_routes, spread_params  # noqa: E402

DEV = "cuda"
SEED = 0x1302266900000A90
ORACLE_STARTS = {mc.MCMC_INIT_CANONICAL: init.representatives,
                 mc.MCMC_INIT_MATCHING: init.matching_representatives,
                 mc.MCMC_INIT_MWPM: mm.mwpm_representatives}


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_weights(L, syn, mode):
    """[n][4] non-identity qubits of each class start of the oracle."""
    lat = geometry.Lattice(L)
    return np.stack([(ORACLE_STARTS[mode](lat, s) != 0).sum(axis=1) for s in syn])


@pytest.mark.parametrize("mode", sorted(ORACLE_STARTS))
@pytest.mark.parametrize("L", [3, 5, 8])
def test_start_weights_match_oracle(L, mode):
    say(f"start weights L={L} mode={mode}")
    n_stab = 2 * L * (L - 1)
    syn = np.concatenate([uniform_syndromes(L, 40, SEED + L, density=0.15),
                          uniform_syndromes(L, 10, SEED + 2 * L, density=0.5),
                          np.zeros((1, n_stab), np.uint8), np.ones((1, n_stab), np.uint8)])
    w = mc.start_weights(torch.from_numpy(syn).to(DEV), L, init=mode)
    torch.cuda.synchronize()
    assert np.array_equal(w.cpu().numpy(), oracle_weights(L, syn, mode))


def labelled_samples(n, seed):
    """Seeded rates (some on bin edges), class start weights and budget
    labels whose misses grow at small gaps and high rates."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.03, 0.2, n)
    p[:40] = np.repeat([0.07, 0.1, 0.15, 0.19], 10)
    w = np.sort(rng.integers(0, 30, size=(n, 4)), axis=1)[:, rng.permutation(4)]
    gap = cnn.start_weight_gap(w)
    budget = np.where(rng.random(n) < np.exp(-gap / 3.0) * p * 4,
                      rng.integers(1, 3, n), 0).astype(np.int32)
    return p, w.astype(np.int32), budget


@pytest.mark.parametrize("max_miss,min_count", [(0.0, 1), (0.01, 20), (0.05, 40), (1.0, 1)])
def test_fit_gap_table_matches_oracle(max_miss, min_count):
    p, w, budget = labelled_samples(6000, SEED + 1)
    got = gate.fit_gap_table(p, torch.from_numpy(w).to(DEV), torch.from_numpy(budget).to(DEV),
                             max_miss, min_count)
    want = cnn.fit_gap_table(p, w, budget, max_miss, min_count)
    say(f"table {got.tolist()}")
    assert np.array_equal(got, want)


def network_routes(logits, thr):
    """The budget head's route (q0 >= thr: 0, q0 + q1 >= thr: 1, else 2) and
    whether both confidences are clear of the threshold."""
    z = logits[:, 4:7].astype(np.float64)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    q = e / e.sum(axis=1, keepdims=True)
    c0, c01 = q[:, 0], q[:, 0] + q[:, 1]
    route = np.where(c0 >= thr, 0, np.where(c01 >= thr, 1, 2))
    clear = (np.abs(c0 - thr) > 1e-5) & (np.abs(c01 - thr) > 1e-5)
    return route, clear


@pytest.mark.parametrize("escalate", [0.0, 2.5])
def test_gated_gap_route(escalate):
    """Routes: the network's, with route 0 added where the oracle's gap rule
    takes the syndrome; outputs against the plain entry point per route."""
    L, n, chains, seed, thr = 5, 300, 3, SEED + 5, 0.5
    say(f"gated gap route L={L} escalate={escalate}")
    syn_h = uniform_syndromes(L, n, seed, density=0.12)
    syn = torch.from_numpy(syn_h).to(DEV)
    rng = np.random.default_rng(seed + 2)
    p = rng.choice([0.06, 0.1, 0.14], size=n)
    ids = (np.arange(n, dtype=np.int64) * 3 + 1).astype(np.uint32)
    table = np.full(cnn.GAP_BINS, cnn.GAP_NEVER, np.uint8)
    table[6], table[10] = 1, 2          # rate 0.14: never by gap
    prm = torch.from_numpy(spread_params(L, seed + 1)).to(DEV)
    # the default starts (greedy matching), as the plain entry point that
    # check_routes compares with
    g = gate.GatedDecoder(L, 0.1, seed, max_batch=n, sweeps_short=3, sweeps_full=9,
                          chains=chains, threshold=thr, escalate=escalate, gap_table=table)
    out = g.decode(prm, syn, p=p, ids=ids, want_correction=True)
    torch.cuda.synchronize()
    net, clear = network_routes(out["logits"].cpu().numpy(), thr)
    by_gap = cnn.gap_route(p, oracle_weights(L, syn_h, mc.MCMC_INIT_MATCHING), table)
    route = out["route"].cpu().numpy()
    want0 = (net == 0) | by_gap
    assert np.array_equal(route[clear] == 0, want0[clear])
    assert (by_gap & (net != 0)).sum() > 20 and (net == 0).sum() > 0, "both ways to route 0"
    keep = clear & ~want0
    if escalate == 0.0:
        assert np.array_equal(route[keep], net[keep])
    else:
        assert np.array_equal(np.where(route[keep] == 3, 1, route[keep]), net[keep])
    counts, _ = check_routes(L, syn, p, ids.astype(np.int64), out, chains, 3, 9, seed)
    say(f"routes {counts}")
    # switched off: the network's routes alone
    g.set_gap_table(None)
    out2 = g.decode(prm, syn, p=p, ids=ids, want_correction=True)
    torch.cuda.synchronize()
    r2 = out2["route"].cpu().numpy()
    assert np.array_equal(r2[clear] == 0, (net == 0)[clear])
    g.close()
