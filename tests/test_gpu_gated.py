"""The gated decoder through the C-ABI: every syndrome's output against
mcmc_decode_batch with the same rate, id and the sweep budget of its route
(0: none, 1: short, 2 and 3: full), bit for bit (class and correction).
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from paper_1302_2669_amd import gate  # noqa: E402
from paper_1302_2669_amd.inputs import cnn_init, uniform_rates, uniform_syndromes  # noqa: E402

DEV = "cuda"
SEED = 0x1302266900000A20


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def spread_params(L, seed):
    """Initial parameters with a wide budget head, so that every route is
    taken by some syndrome."""
    prm = cnn_init(L, seed)
    n = prm.size
    kh = L * L * 32
    wh0 = n - 7 - 7 * kh
    prm[wh0 + 4 * kh:wh0 + 7 * kh] *= 8.0
    return prm


def margin(sum_n, K):
    """Replica margin z of each syndrome's decision from its per-chain sums
    [m][4][K][C] (the escalation statistic of mcmc_gated_decode)."""
    w = np.array([1 if k + 1 == K else (4 if (k + 1) % 2 == 1 else 2) for k in range(K)])
    key = (sum_n * w[None, None, :, None]).sum(axis=2).astype(np.float64)   # [m][4][C]
    mean = key.mean(axis=2)
    var = key.var(axis=2, ddof=1)
    b = np.argmin(mean, axis=1)
    masked = mean.copy()
    masked[np.arange(len(b)), b] = np.inf
    s = np.argmin(masked, axis=1)
    rows = np.arange(len(b))
    gap = mean[rows, s] - mean[rows, b]
    se = np.sqrt((var[rows, b] + var[rows, s]) / key.shape[2])
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(se > 0, gap / se, np.where(gap > 0, np.inf, 0.0))
    return z


def check_routes(L, syn, p_host, ids, out, chains, sweeps_short, sweeps_full, seed,
                 class_route=False, threshold=None):
    """Every syndrome's class and correction against the plain entry point at
    its route's budget; returns the route counts and, per route 1 and 3, the
    short run's replica margins.  Under class_route a route-0 syndrome whose
    class head is confident answers the no-sweep decision composed with the
    head's class, its correction the start of that class."""
    chosen = out["chosen"].cpu().numpy()
    route = out["route"].cpu().numpy()
    corr = out["correction"].cpu().numpy()
    counts = [int((route == r).sum()) for r in range(4)]
    assert counts == list(out["counts"])
    flip = np.zeros(len(route), dtype=np.int64)
    if class_route:
        z = out["logits"][:, :4].cpu().numpy().astype(np.float64)
        e = np.exp(z - z.max(axis=1, keepdims=True))
        c = (e / e.sum(axis=1, keepdims=True)).max(axis=1)
        assert (np.abs(c - threshold) > 1e-5).all(), "a class confidence at the threshold"
        flip = np.where((route == 0) & (c >= threshold), np.argmax(z, axis=1), 0)
    budget = {0: 0, 1: sweeps_short, 2: sweeps_full, 3: sweeps_full}
    margins = {}
    for r, sweeps in budget.items():
        sel = np.nonzero(route == r)[0]
        if sel.size == 0:
            continue
        # the uniform-rate entry point: one decode per distinct rate
        for pv in np.unique(p_host[sel]):
            sub = sel[p_host[sel] == pv]
            ref = mc.decode_batch(syn[torch.from_numpy(sub).to(DEV)], L, float(pv), sweeps, seed,
                                  chains=chains, syndrome_ids=torch.from_numpy(ids[sub]))
            torch.cuda.synchronize()
            want = ref["chosen"].cpu().numpy() ^ flip[sub]
            assert np.array_equal(chosen[sub], want), f"route {r}"
            want_corr = ref["correction"].cpu().numpy()
            moved = np.nonzero(flip[sub])[0]
            if moved.size:
                reps = mc.init_representatives(syn[torch.from_numpy(sub[moved]).to(DEV)], L,
                                               init=mc.MCMC_INIT_MATCHING).cpu().numpy()
                want_corr[moved] = reps[np.arange(moved.size), want[moved]]
            assert np.array_equal(corr[sub], want_corr), f"route {r}"
            if r in (1, 3):
                short = mc.decode_batch(syn[torch.from_numpy(sub).to(DEV)], L, float(pv),
                                        sweeps_short, seed, chains=chains,
                                        syndrome_ids=torch.from_numpy(ids[sub]), want_sums=True)
                torch.cuda.synchronize()
                margins.setdefault(r, []).append(margin(short["sum_n"].cpu().numpy(), 1))
    return counts, {r: np.concatenate(v) for r, v in margins.items()}


@pytest.mark.parametrize("L", [5, 13])
def test_gated_routes_match_plain_entry_points(L):
    say(f"gated L={L}")
    n, chains, seed = 300, 2, SEED + L
    syn = torch.from_numpy(uniform_syndromes(L, n, seed, density=0.08)).to(DEV)
    prm = torch.from_numpy(spread_params(L, seed + 1)).to(DEV)
    g = gate.GatedDecoder(L, 0.1, seed, max_batch=n, sweeps_short=3, sweeps_full=9,
                          chains=chains, threshold=0.5)
    ids = (np.arange(n, dtype=np.int64) * 7 + 11).astype(np.uint32)
    out = g.decode(prm, syn, ids=ids, want_correction=True)
    counts, _ = check_routes(L, syn, np.full(n, 0.1), ids.astype(np.int64), out, chains, 3, 9,
                             seed)
    say(f"routes {counts}")
    assert all(c > 0 for c in counts[:3]) and counts[3] == 0, counts
    # a second, smaller call on the same decoder (plan storage reused)
    m = 97
    syn2 = torch.from_numpy(uniform_syndromes(L, m, seed + 5, density=0.12)).to(DEV)
    out2 = g.decode(prm, syn2, want_correction=True)
    check_routes(L, syn2, np.full(m, 0.1), np.arange(m, dtype=np.int64), out2, chains, 3, 9, seed)
    g.close()


def test_gated_per_syndrome_rates():
    L, n, chains, seed = 7, 200, 2, SEED + 77
    syn = torch.from_numpy(uniform_syndromes(L, n, seed, density=0.1)).to(DEV)
    # a few distinct rates so that the reference can run per rate
    p = np.asarray([0.05, 0.09, 0.13, 0.17], dtype=np.float32)[np.arange(n) % 4].astype(np.float64)
    prm = torch.from_numpy(spread_params(L, seed + 1)).to(DEV)
    g = gate.GatedDecoder(L, 0.1, seed, max_batch=256, sweeps_short=4, sweeps_full=12,
                          chains=chains, threshold=0.5)
    out = g.decode(prm, syn, p=p, want_correction=True)
    check_routes(L, syn, p, np.arange(n, dtype=np.int64), out, chains, 4, 12, seed)
    # the network saw the per-syndrome rates: same logits as a direct pass
    logits, _ = gate.forward(L, prm, syn, torch.from_numpy(p.astype(np.float32)).to(DEV))
    torch.cuda.synchronize()
    assert torch.equal(logits[:, :7], out["logits"][:, :7])
    # a following call without rates uses the configured rate, not the tables
    # the previous call uploaded
    out2 = g.decode(prm, syn, want_correction=True)
    check_routes(L, syn, np.full(n, 0.1), np.arange(n, dtype=np.int64), out2, chains, 4, 12, seed)
    g.close()


def test_gated_threshold_one_is_plain_decoder():
    """With threshold 1 only a class softmax that rounds to exactly 1 passes;
    an untrained network's logits are far from that, so every syndrome takes
    the full budget and the output is the plain decoder's."""
    L, n, seed = 5, 128, SEED + 5
    syn = torch.from_numpy(uniform_syndromes(L, n, seed, density=0.1)).to(DEV)
    prm = torch.from_numpy(cnn_init(L, seed + 1)).to(DEV)
    g = gate.GatedDecoder(L, 0.12, seed, max_batch=n, sweeps_full=25, chains=2, threshold=1.0)
    out = g.decode(prm, syn, want_correction=True)
    ref = mc.decode_batch(syn, L, 0.12, 25, seed, chains=2)
    torch.cuda.synchronize()
    assert out["counts"] == [0, 0, n, 0]
    assert torch.equal(out["chosen"], ref["chosen"])
    assert torch.equal(out["correction"], ref["correction"])
    g.close()


def test_gated_escalation():
    """Short-budget syndromes whose decision margin across the replicas is
    below the escalation level take the full budget; the others keep the
    short one."""
    L, n, chains, seed = 9, 400, 3, SEED + 9
    syn = torch.from_numpy(uniform_syndromes(L, n, seed, density=0.06)).to(DEV)
    prm = torch.from_numpy(spread_params(L, seed + 1)).to(DEV)
    esc = 2.5
    g = gate.GatedDecoder(L, 0.08, seed, max_batch=n, sweeps_short=9, sweeps_full=30,
                          chains=chains, threshold=0.5, escalate=esc)
    out = g.decode(prm, syn, want_correction=True)
    counts, z = check_routes(L, syn, np.full(n, 0.08), np.arange(n, dtype=np.int64), out,
                             chains, 9, 30, seed)
    say(f"routes {counts}")
    assert counts[1] > 0 and counts[3] > 0, counts
    clear1 = np.abs(z[1] - esc) > 1e-9 * max(1.0, esc)
    clear3 = np.abs(z[3] - esc) > 1e-9 * max(1.0, esc)
    assert (z[1][clear1] >= esc).all() and (z[3][clear3] < esc).all()
    g.close()


def test_gated_class_route():
    """A class head read relative to the start decision: confident syndromes
    answer without sweeps, some of them with a class other than the start
    decision; everything else as the plain entry points."""
    L, n, chains, seed = 7, 300, 2, SEED + 21
    syn = torch.from_numpy(uniform_syndromes(L, n, seed, density=0.08)).to(DEV)
    prm = torch.from_numpy(spread_params(L, seed + 1)).to(DEV)
    # a wide class head as well, so that it is confident on some syndromes
    kh = L * L * 32
    wh0 = prm.numel() - 7 - 7 * kh
    prm[wh0:wh0 + 4 * kh] *= 8.0
    thr = 0.8
    g = gate.GatedDecoder(L, 0.1, seed, max_batch=n, sweeps_short=3, sweeps_full=9,
                          chains=chains, threshold=thr, init=mc.MCMC_INIT_MATCHING,
                          class_route=True)
    ids = (np.arange(n, dtype=np.int64) * 5 + 3).astype(np.uint32)
    out = g.decode(prm, syn, ids=ids, want_correction=True)
    counts, _ = check_routes(L, syn, np.full(n, 0.1), ids.astype(np.int64), out, chains, 3, 9,
                             seed, class_route=True, threshold=thr)
    z = out["logits"][:, :4].cpu().numpy().astype(np.float64)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    conf = (e / e.sum(axis=1, keepdims=True)).max(axis=1)
    moved = int(((conf >= thr) & (np.argmax(z, axis=1) != 0)).sum())
    say(f"routes {counts}, {moved} answered with another class")
    assert counts[0] > 0 and counts[2] > 0 and moved > 0
    g.close()


def test_gated_rejects_oversized_batch():
    L = 5
    g = gate.GatedDecoder(L, 0.1, 1, max_batch=16)
    syn = torch.zeros((17, mc.geometry(L)[1]), dtype=torch.uint8, device=DEV)
    prm = torch.from_numpy(cnn_init(L, 3)).to(DEV)
    with pytest.raises(mc.McmcError):
        g.decode(prm, syn)
    g.close()
