"""What the trained gate network gains over the decoder without it.

A distance-7 network is trained on the GPU (the library's forward, backward
and Adam kernels) on labels the decoder makes itself, then the gated decoder
and the plain decoder (full budget for every syndrome) decode the same fresh
syndromes with the same chains.  The gain is measured in Metropolis work
(stabilizer updates, which is what the gate saves; wall time at this small
size is dominated by fixed costs), and the price in logical errors is
measured pairwise on the same syndromes:

* the trained gate saves at least a fifth of the work (it routes easy
  syndromes to no or few sweeps);
* the untrained network at the same confidence level saves almost nothing,
  so the saving comes from training;
* syndromes the plain decoder gets right and the gated one gets wrong
  outnumber the reverse by at most 0.3% of the batch.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from paper_1302_2669_amd import gate  # noqa: E402
from paper_1302_2669_amd.inputs import cnn_init, uniform_rates  # noqa: E402

DEV = "cuda"
SEED = 0x1302266900000A60
L = 7


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def work(counts):
    """Counted sweeps per class chain, summed over the batch (a short run that
    escalated pays for both)."""
    return counts[1] * L + (counts[2] + counts[3]) * L * L + counts[3] * L


def test_trained_gate_saves_work_at_matched_error():
    n_train, n_eval = 200_000, 40_000
    p_tr = uniform_rates(n_train, SEED).astype(np.float64)
    syn, _, ids = gate.sample_dataset(L, p_tr, SEED, id_base=0)
    soft, bud, _ = gate.mcmc_labels(L, syn, p_tr, ids, SEED)
    say(f"labels: budget histogram {np.bincount(bud.cpu().numpy(), minlength=3).tolist()}")
    net = gate.GateNet(L, cnn_init(L, SEED + 1), device=DEV)
    untrained = net.params.clone()
    hist = gate.train(net, syn, torch.from_numpy(p_tr.astype(np.float32)).to(DEV), soft, bud,
                      epochs=3, batch=512, lr=3e-3, seed=SEED, log=say)
    assert hist[-1] < hist[0]

    p_ev = uniform_rates(n_eval, SEED + 2).astype(np.float64)
    syn_e, cls_e, ids_e = gate.sample_dataset(L, p_ev, SEED + 3, id_base=1 << 30)
    plan = mc.MixedPlan.from_arrays(L, p_ev, L * L, SEED, chains=4, syndrome_ids=ids_e)
    plain = plan.execute(syn_e.reshape(-1), want_correction=False)["chosen"]
    plan.close()

    g = gate.GatedDecoder(L, 0.1, SEED, max_batch=n_eval, chains=4, threshold=0.99,
                          escalate=2.0)
    res = g.decode(net.params, syn_e, p=p_ev, ids=ids_e)
    base = g.decode(untrained, syn_e, p=p_ev, ids=ids_e)
    g.close()
    full = n_eval * L * L
    gain = full / work(res["counts"])
    gain0 = full / work(base["counts"])
    pr = (plain == cls_e).cpu().numpy()
    gr = (res["chosen"] == cls_e).cpu().numpy()
    worse, better = int((pr & ~gr).sum()), int((~pr & gr).sum())
    say(f"routes {res['counts']} work gain {gain:.3f} (untrained {gain0:.3f}); "
        f"logical error plain {1 - pr.mean():.4f} gated {1 - gr.mean():.4f}; "
        f"plain-right/gated-wrong {worse}, reverse {better}")
    assert gain >= 1.2
    assert gain0 < 1.05
    assert worse - better <= 0.003 * n_eval
