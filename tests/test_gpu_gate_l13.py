"""The gate at distance 13 with the exact enhanced-matching starts.

* Escalation margin: the replica margin z of a short run's decision
  (mcmc_gated_decode's escalation statistic) is checked against the
  21-temperature thermodynamic-integration labels: the short decision
  disagrees with the label's most likely class less often as z grows, and
  rarely above the margin the bench uses.
* Gain: a network trained on relative class targets and budget labels (both
  made by the decoder itself) against the plain decoder on the same fresh
  syndromes and chains, at p uniform in [0.05, 0.18] (the training
  distribution) and at p = 0.15: Metropolis work saved, and the pairwise
  logical-error price (plain right and gated wrong, and the reverse).
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from paper_1302_2669_amd import gate  # noqa: E402
from paper_1302_2669_amd.inputs import uniform_rates  # noqa: E402

DEV = "cuda"
SEED = 0x1302266900000B13
L = 13
MWPM = mc.MCMC_INIT_MWPM


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def replica_margin(sum_n):
    """z per syndrome from per-chain sums [m][4][1][C] (one temperature)."""
    key = sum_n[:, :, 0, :].astype(np.float64)
    mean, var = key.mean(axis=2), key.var(axis=2, ddof=1)
    rows = np.arange(key.shape[0])
    b = np.argmin(mean, axis=1)
    masked = mean.copy()
    masked[rows, b] = np.inf
    s = np.argmin(masked, axis=1)
    gap = mean[rows, s] - mean[rows, b]
    se = np.sqrt((var[rows, b] + var[rows, s]) / key.shape[2])
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(se > 0, gap / se, np.where(gap > 0, np.inf, 0.0)), b


def test_escalation_margin_is_calibrated_against_ti_labels():
    n, C = 20000, 4
    p = uniform_rates(n, SEED).astype(np.float64)
    syn, _, ids = gate.sample_dataset(L, p, SEED, id_base=0)
    flat = syn.reshape(-1)
    short = mc.MixedPlan.from_arrays(L, p, L, SEED, chains=C, syndrome_ids=ids, init=MWPM)
    out = short.execute(flat, want_sums=True)
    short.close()
    ti = mc.MixedPlan.from_arrays(L, p, L * L, SEED, chains=1, n_temps=20, syndrome_ids=ids,
                                  init=MWPM)
    label = ti.execute(flat)["class_prob"].cpu().numpy().argmax(axis=1)
    ti.close()
    z, b = replica_margin(out["sum_n"].cpu().numpy().reshape(n, 4, 1, C))
    assert np.array_equal(b, out["chosen"].cpu().numpy())
    wrong = b != label
    edges = [0.0, 1.0, 2.0, 4.0, np.inf]
    rates = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (z >= lo) & (z < hi) if np.isfinite(hi) else (z >= lo)
        rates.append((int(sel.sum()), float(wrong[sel].mean()) if sel.any() else 0.0))
    say("margin bins [0,1) [1,2) [2,4) [4,inf]: (count, disagreement with the TI label) "
        + str(rates))
    r = [q for _, q in rates]
    assert all(cnt > 100 for cnt, _ in rates)
    assert r[0] > r[1] > r[2] > r[3]
    assert r[3] < 0.01
    assert r[0] > 5 * r[3]


def work(counts):
    return counts[1] * L + (counts[2] + counts[3]) * L * L + counts[3] * L


def test_trained_gate_at_l13():
    n_train, n_eval = 200_000, 30_000
    p_tr = uniform_rates(n_train, SEED + 1).astype(np.float64)
    syn, _, ids = gate.sample_dataset(L, p_tr, SEED + 1, id_base=0)
    soft, bud, _ = gate.mcmc_labels(L, syn, p_tr, ids, SEED, init=MWPM, relative=True)
    say(f"labels: budget histogram {np.bincount(bud.cpu().numpy(), minlength=3).tolist()}, "
        f"mean P(start decision right) {float(soft[:, 0].mean()):.3f}")
    net = gate.GateNet(L, gate.init_params(L, SEED + 2, device=DEV), device=DEV)
    hist = gate.train(net, syn, torch.from_numpy(p_tr.astype(np.float32)).to(DEV), soft, bud,
                      epochs=3, batch=512, lr=3e-3, seed=SEED, log=say)
    assert hist[-1] < hist[0]
    # the start-weight gap route's table from the same labels
    table = gate.fit_gap_table(p_tr, mc.start_weights(syn, L, init=MWPM), bud, 0.003, 50)
    say(f"gap table {table.tolist()}")

    def evaluate(p_ev, tag):
        syn_e, cls_e, ids_e = gate.sample_dataset(L, p_ev, SEED + 3, id_base=1 << 30)
        plan = mc.MixedPlan.from_arrays(L, p_ev, L * L, SEED, chains=4, syndrome_ids=ids_e,
                                        init=MWPM)
        plain = plan.execute(syn_e.reshape(-1), want_correction=False)["chosen"]
        plan.close()
        pr = (plain == cls_e).cpu().numpy()
        res = {}
        # (class route, gap route): the network alone, with its class head,
        # and the gap route alone (threshold 1 leaves the network no route
        # 0 or 1)
        for class_route, gap in ((False, False), (True, False), (False, True)):
            g = gate.GatedDecoder(L, 0.15, SEED, max_batch=n_eval, chains=4,
                                  threshold=1.0 if gap else 0.99, init=MWPM,
                                  class_route=class_route, gap_table=table if gap else None)
            out = g.decode(net.params, syn_e, p=p_ev, ids=ids_e)
            g.close()
            gr = (out["chosen"] == cls_e).cpu().numpy()
            worse, better = int((pr & ~gr).sum()), int((~pr & gr).sum())
            gain = n_eval * L * L / max(1, work(out["counts"]))
            say(f"{tag} class_route={class_route} gap={gap}: routes {out['counts']} work gain "
                f"{gain:.3f}; logical error plain {1 - pr.mean():.4f} gated "
                f"{1 - gr.mean():.4f}; plain-right/gated-wrong {worse}, reverse {better}")
            res[(class_route, gap)] = (gain, worse, better, 1 - pr.mean(), 1 - gr.mean())
        return res

    uni = evaluate(uniform_rates(n_eval, SEED + 4).astype(np.float64), "p uniform")
    for gain, worse, better, e_plain, e_gated in uni.values():
        assert gain >= 1.5
        assert worse - better <= 0.003 * n_eval
        assert e_gated <= 1.02 * e_plain
    # the gap route alone: more work saved than the network, at a smaller
    # error cost
    gain, worse, better, e_plain, e_gated = uni[(False, True)]
    assert gain >= 1.8 and gain > uni[(False, False)][0]
    assert worse - better <= 0.002 * n_eval
    fixed = evaluate(np.full(n_eval, 0.15), "p 0.15")
    for gain, worse, better, e_plain, e_gated in fixed.values():
        assert gain >= 1.0
        assert e_gated <= 1.02 * e_plain
