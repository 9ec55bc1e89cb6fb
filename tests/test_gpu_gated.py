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


def check_routes(L, syn, p_host, ids, out, chains, sweeps_short, sweeps_full, seed):
    chosen = out["chosen"].cpu().numpy()
    route = out["route"].cpu().numpy()
    corr = out["correction"].cpu().numpy()
    counts = [int((route == r).sum()) for r in range(4)]
    assert counts == list(out["counts"])
    budget = {0: 0, 1: sweeps_short, 2: sweeps_full, 3: sweeps_full}
    probs = {}
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
            assert np.array_equal(chosen[sub], ref["chosen"].cpu().numpy()), f"route {r}"
            assert np.array_equal(corr[sub], ref["correction"].cpu().numpy()), f"route {r}"
            if r in (1, 3):
                short = ref if r == 1 else mc.decode_batch(
                    syn[torch.from_numpy(sub).to(DEV)], L, float(pv), sweeps_short, seed,
                    chains=chains, syndrome_ids=torch.from_numpy(ids[sub]))
                probs.setdefault(r, []).append(short["class_prob"].max(dim=1).values.cpu().numpy())
    return counts, {r: np.concatenate(v) for r, v in probs.items()}


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
    """Short-budget syndromes whose own class estimate is below the
    escalation level take the full budget; the others keep the short one."""
    L, n, chains, seed = 9, 400, 2, SEED + 9
    syn = torch.from_numpy(uniform_syndromes(L, n, seed, density=0.06)).to(DEV)
    prm = torch.from_numpy(spread_params(L, seed + 1)).to(DEV)
    esc = 0.9
    g = gate.GatedDecoder(L, 0.08, seed, max_batch=n, sweeps_short=9, sweeps_full=30,
                          chains=chains, threshold=0.5, escalate=esc)
    out = g.decode(prm, syn, want_correction=True)
    counts, probs = check_routes(L, syn, np.full(n, 0.08), np.arange(n, dtype=np.int64), out,
                                 chains, 9, 30, seed)
    say(f"routes {counts}")
    assert counts[1] > 0 and counts[3] > 0, counts
    assert (probs[1] >= esc).all() and (probs[3] < esc).all()
    g.close()


def test_gated_rejects_oversized_batch():
    L = 5
    g = gate.GatedDecoder(L, 0.1, 1, max_batch=16)
    syn = torch.zeros((17, mc.geometry(L)[1]), dtype=torch.uint8, device=DEV)
    prm = torch.from_numpy(cnn_init(L, 3)).to(DEV)
    with pytest.raises(mc.McmcError):
        g.decode(prm, syn)
    g.close()
