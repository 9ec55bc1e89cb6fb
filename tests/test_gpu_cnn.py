"""Parity of the gate network's HIP kernels with the float64 oracle, through
the C-ABI, layer by layer.

Every matrix product on the GPU takes bfloat16 operands (exact in fp32
products) and accumulates in fp32; the oracle takes the same bf16 operands
and accumulates exactly.  Each layer is checked on the GPU's own input to
that layer (the previous layer's GPU output), so the bound is per layer:

* fp32 outputs (logits, gradients): |gpu - ref| <= (K + 2) 2^-24 sum|terms|,
  K the number of terms summed (any summation order satisfies this);
* bf16 outputs (ReLU activations, back-propagated pre-activation
  gradients): the same plus one bf16 unit in the last place,
  2^-7 max(|gpu|, |ref|) (both sides round to nearest even, so a rounding
  can fall on different sides of a tie only if the fp32 sum moved across it);
* terms that depend on dL/dlogits add its fp32 error: each entry is
  (softmax - target) / B (times the budget weight), with softmax from expf
  and a division a few ulp off, so its absolute error stays below
  DZ_ABS (1 + w_b) / B.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402
from paper_1302_2669_amd import gate  # noqa: E402
from paper_1302_2669_amd.inputs import (cnn_init, cnn_targets, uniform_rates,  # noqa: E402
                                        uniform_syndromes)
from oracle import cnn  # noqa: E402

DEV = "cuda"
U32 = 2.0 ** -24
BF_ULP = 2.0 ** -7
DZ_ABS = 4e-6
SEED = 0x1302266900000A10


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16_tensor(ws, off, rows, cols):
    t = ws[off:off + rows * cols * 2].view(torch.bfloat16).reshape(rows, cols)
    return t.float().cpu().numpy().astype(np.float64)


def within(gpu, ref, bound, what, frac_equal=None):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(gpu - ref)
    bad = err > bound
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside the bound; worst "
                           f"excess {np.max(err - bound):.3e} at {np.argmax(err - bound)}")
    if frac_equal is not None:
        eq = np.mean(gpu == ref)
        assert eq >= frac_equal, f"{what}: only {eq:.4f} of the entries identical"


def conv_ref(x, W, b):
    """fp64 conv + bias and the matching sum of |terms| (same tap order)."""
    y = cnn.conv(x, W, b)
    s = cnn.conv(np.abs(x), np.abs(W), np.abs(b))
    return y, s


def run_layers(L, B, seed):
    """Forward + backward on the GPU and every teacher-forced comparison."""
    nq, ns = mc.geometry(L)
    syn = uniform_syndromes(L, B, seed, density=0.15)
    p = uniform_rates(B, seed + 1)
    prm = cnn_init(L, seed + 2)
    # non-zero biases so that the bias path is exercised
    rng = np.random.default_rng(seed + 3)
    off = cnn.unflatten(L, np.arange(prm.size))
    for k in ("b1", "b2", "b3", "bh"):
        idx = off[k].reshape(-1).astype(np.int64)
        prm[idx] = rng.normal(0.0, 0.1, size=idx.size).astype(np.float32)
    tgt, bud = cnn_targets(B, seed + 4)
    wb = 0.5

    d_syn = torch.from_numpy(syn).to(DEV)
    d_p = torch.from_numpy(p).to(DEV)
    d_prm = torch.from_numpy(prm).to(DEV)
    logits, ws = gate.forward(L, d_prm, d_syn, d_p)
    grads, loss = gate.backward(L, d_prm, logits, torch.from_numpy(tgt).to(DEV),
                                torch.from_numpy(bud).to(DEV), ws, wb)
    torch.cuda.synchronize()
    o = gate.workspace_offsets(L, B)
    P = B * L * L
    g = dict(x0=bf16_tensor(ws, o["x0"], P, 8), a1=bf16_tensor(ws, o["a1"], P, 32),
             a2=bf16_tensor(ws, o["a2"], P, 32), a3=bf16_tensor(ws, o["a3"], P, 32),
             dp3=bf16_tensor(ws, o["dp3"], P, 32), dp2=bf16_tensor(ws, o["dp2"], P, 32),
             dp1=bf16_tensor(ws, o["dp1"], P, 32))
    g["logits"] = logits.cpu().numpy().astype(np.float64)[:, :7]
    g["grads"] = grads.cpu().numpy().astype(np.float64)
    g["loss"] = loss.cpu().numpy().astype(np.float64)
    params = cnn.unflatten(L, prm.astype(np.float64))
    return dict(L=L, B=B, syn=syn, p=p, params=params, tgt=tgt, bud=bud, wb=wb, gpu=g)


CASES = [(3, 37), (5, 64), (13, 23)]


@pytest.fixture(scope="module", params=CASES, ids=[f"L{L}_B{B}" for L, B in CASES])
def layers(request):
    L, B = request.param
    say(f"cnn layers L={L} B={B}")
    return run_layers(L, B, SEED + 100 * L + B)


def test_input_planes_exact(layers):
    L, B, g = layers["L"], layers["B"], layers["gpu"]
    x = cnn.to_bf16(cnn.encode(L, layers["syn"], layers["p"].astype(np.float64)))
    x0 = g["x0"].reshape(B, L, L, 8)
    assert np.array_equal(x0[..., :3], x)
    assert not x0[..., 3:].any()


def test_forward_layers(layers):
    L, B, g = layers["L"], layers["B"], layers["gpu"]
    P = layers["params"]
    W = {k: cnn.to_bf16(P[k]) for k in ("W1", "W2", "W3", "Wh")}
    prev = g["x0"].reshape(B, L, L, 8)[..., :3]
    for i, (w, b, name, K) in enumerate([("W1", "b1", "a1", 27), ("W2", "b2", "a2", 288),
                                         ("W3", "b3", "a3", 288)]):
        y, s = conv_ref(prev, W[w], P[b])
        ref = cnn.to_bf16(np.maximum(y, 0.0)).reshape(-1, 32)
        got = g[name]
        bound = (K + 2) * U32 * s.reshape(-1, 32) + BF_ULP * np.maximum(np.abs(got), np.abs(ref))
        within(got, ref, bound, name, frac_equal=0.9)
        prev = got.reshape(B, L, L, 32)
    flat = g["a3"].reshape(B, -1)
    ref = flat @ W["Wh"].T + P["bh"]
    s = np.abs(flat) @ np.abs(W["Wh"]).T + np.abs(P["bh"])
    K = flat.shape[1]
    within(g["logits"], ref, (K + 2) * U32 * s, "logits")


def test_backward_layers(layers):
    L, B, g = layers["L"], layers["B"], layers["gpu"]
    P = layers["params"]
    W = {k: cnn.to_bf16(P[k]) for k in ("W1", "W2", "W3", "Wh")}
    off = cnn.unflatten(L, np.arange(sum(np.prod(s) for _, s in cnn.param_shapes(L))))
    grads = {k: g["grads"][off[k].reshape(-1).astype(np.int64)].reshape(off[k].shape)
             for k in off}
    logits = g["logits"]
    loss, dz, per = cnn.loss_and_dlogits(logits, layers["tgt"].astype(np.float64), layers["bud"],
                                         layers["wb"])
    within(g["loss"], per, 1e-5 * (1.0 + np.abs(per)), "per-sample loss")

    a = {k: g[k].reshape(B, L, L, -1) for k in ("a1", "a2", "a3")}
    x0 = g["x0"].reshape(B, L, L, 8)[..., :3]
    a3f = a["a3"].reshape(B, -1)
    # head
    e_dz = DZ_ABS * (1.0 + layers["wb"]) / B
    ref = dz.T @ a3f
    s = np.abs(dz).T @ np.abs(a3f)
    within(grads["Wh"], ref, (B + 2) * U32 * s + e_dz * np.abs(a3f).sum(axis=0)[None, :],
           "grad Wh")
    within(grads["bh"], dz.sum(axis=0), (B + 2) * U32 * np.abs(dz).sum(axis=0) + B * e_dz,
           "grad bh")
    da3 = dz @ W["Wh"]
    s3 = np.abs(dz) @ np.abs(W["Wh"])                      # [B][features]
    e3 = np.broadcast_to(e_dz * np.abs(W["Wh"]).sum(axis=0)[None, :], s3.shape)
    ref = cnn.to_bf16(da3 * (a["a3"].reshape(B, -1) > 0)).reshape(-1, 32)
    got = g["dp3"]
    bound = (9 * U32 * s3 + e3).reshape(-1, 32) + BF_ULP * np.maximum(np.abs(got), np.abs(ref))
    within(got, ref, bound, "dpre3", frac_equal=0.9)

    # convolutions, each from the GPU's own gradient and activations
    chain = [("W3", "b3", g["dp3"], a["a2"], "dp2", 32),
             ("W2", "b2", g["dp2"], a["a1"], "dp1", 32),
             ("W1", "b1", g["dp1"], x0, None, 3)]
    n_pix = B * L * L
    for w, b, dpre, inp, nxt, cin in chain:
        dpre = dpre.reshape(B, L, L, 32)
        dW, db, dx = cnn._conv_backward(inp, dpre, W[w])
        sW, sb, sx = cnn._conv_backward(np.abs(inp), np.abs(dpre), np.abs(W[w]))
        within(grads[w], dW, (n_pix + 2) * U32 * sW, f"grad {w}")
        within(grads[b], db, (n_pix + 2) * U32 * sb, f"grad {b}")
        if nxt is not None:
            ref = cnn.to_bf16(dx * (inp > 0)).reshape(-1, 32)
            got = g[nxt]
            bound = (288 + 2) * U32 * sx.reshape(-1, 32) + \
                BF_ULP * np.maximum(np.abs(got), np.abs(ref))
            within(got, ref, bound, nxt, frac_equal=0.9)


def test_end_to_end_close_to_oracle(layers):
    """The whole pass against the oracle run from the same inputs: rounding
    flips compound, so this is a closeness check (1% of the logit scale,
    gradient direction), the per-layer tests above are the parity bar."""
    L, B, g = layers["L"], layers["B"], layers["gpu"]
    loss, per, grads, logits = cnn.backward(L, layers["params"], layers["syn"],
                                            layers["p"].astype(np.float64),
                                            layers["tgt"].astype(np.float64), layers["bud"],
                                            layers["wb"], bf16=True)
    scale = np.abs(logits).max() + 1.0
    assert np.abs(g["logits"] - logits).max() <= 0.01 * scale
    ref = cnn.flatten(L, grads)
    cos = float(g["grads"] @ ref / (np.linalg.norm(g["grads"]) * np.linalg.norm(ref)))
    assert cos > 0.999, cos


def test_adam_step_matches_oracle():
    n = 1000
    rng = np.random.default_rng(SEED + 7)
    prm = rng.normal(size=n).astype(np.float32)
    gr = rng.normal(size=n).astype(np.float32)
    m = rng.normal(scale=0.1, size=n).astype(np.float32)
    v = rng.random(n).astype(np.float32) * 0.01
    d = [torch.from_numpy(x.copy()).to(DEV) for x in (prm, gr, m, v)]
    step, lr = 5, 3e-3
    gate.adam_step(d[0], d[1], d[2], d[3], step, lr)
    torch.cuda.synchronize()
    # the entry point takes its hyper-parameters as fp32: give the oracle the
    # same values (1 - fp32(0.999) is 1.3e-5 away from 0.001)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    op, om, ov = cnn.adam({"w": prm.astype(np.float64)}, {"w": gr.astype(np.float64)},
                          {"w": m.astype(np.float64)}, {"w": v.astype(np.float64)},
                          f32(lr), f32(0.9), f32(0.999), f32(1e-8), step)
    np.testing.assert_allclose(d[2].cpu().numpy(), om["w"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(d[3].cpu().numpy(), ov["w"], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(d[0].cpu().numpy(), op["w"], rtol=1e-5, atol=lr * 1e-4)


@pytest.mark.parametrize("class_route", [False, True])
def test_gate_decisions(class_route):
    B = 5000
    rng = np.random.default_rng(SEED + 8)
    z = rng.normal(scale=3.0, size=(B, 8)).astype(np.float32)
    z[:10, :4] = 0.0        # class ties -> lowest class
    d = torch.from_numpy(z).to(DEV)
    thr = 0.9
    route, cls, conf = gate.gate(d, thr, class_route=class_route)
    torch.cuda.synchronize()
    route, cls, conf = route.cpu().numpy(), cls.cpu().numpy(), conf.cpu().numpy()
    assert np.array_equal(cls, np.argmax(z[:, :4].astype(np.float64), axis=1))

    def softmax(v):
        e = np.exp(v - v.max(axis=1, keepdims=True))
        return e / e.sum(axis=1, keepdims=True)

    q = softmax(z[:, 4:7].astype(np.float64))
    c = softmax(z[:, :4].astype(np.float64)).max(axis=1)
    ref_conf = np.stack([q[:, 0], q[:, 0] + q[:, 1], c], axis=1)
    np.testing.assert_allclose(conf, ref_conf, rtol=1e-5, atol=1e-7)
    ref_route = np.where(ref_conf[:, 0] >= thr, 0, np.where(ref_conf[:, 1] >= thr, 1, 2))
    if class_route:
        ref_route = np.where(c >= thr, 0, ref_route)
    clear = (np.abs(ref_conf - thr) > 1e-5).all(axis=1)
    assert np.array_equal(route[clear], ref_route[clear])
    assert {0, 1, 2} <= set(np.unique(route))


def test_relative_targets_match_oracle():
    """Class targets relative to the start decision (a permutation of each
    row), bit for bit; start classes read through their low two bits."""
    n = 3001
    rng = np.random.default_rng(SEED + 9)
    prob = rng.dirichlet(np.ones(4), size=n).astype(np.float32)
    start = rng.integers(0, 256, size=n).astype(np.uint8)
    out = gate.relative_targets(torch.from_numpy(start).to(DEV), torch.from_numpy(prob).to(DEV))
    torch.cuda.synchronize()
    ref = cnn.relative_targets(prob, start & 3)
    assert np.array_equal(out.cpu().numpy(), ref)


def test_training_reduces_loss():
    """A few hundred Adam steps on a fixed small set drive the GPU loss down
    (the kernels' gradients are descent directions end to end)."""
    L, B = 5, 256
    syn = torch.from_numpy(uniform_syndromes(L, B, SEED + 9, density=0.1)).to(DEV)
    p = torch.from_numpy(uniform_rates(B, SEED + 10)).to(DEV)
    t, b = cnn_targets(B, SEED + 11)
    # learnable targets: class = parity of the lit stars, budget from p
    t = np.zeros((B, 4), dtype=np.float32)
    star = syn[:, :L * (L - 1)].sum(dim=1).cpu().numpy()
    t[np.arange(B), star % 4] = 1.0
    b = (p.cpu().numpy() > 0.115).astype(np.int32)
    tt, bb = torch.from_numpy(t).to(DEV), torch.from_numpy(b).to(DEV)
    net = gate.GateNet(L, cnn_init(L, SEED + 12), device=DEV)
    first = float(net.train_step(syn, p, tt, bb, lr=2e-3).mean())
    for _ in range(300):
        last = net.train_step(syn, p, tt, bb, lr=2e-3)
    last = float(last.mean())
    say(f"loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first


@pytest.mark.parametrize("L,B", [(2, 1), (3, 37), (5, 70), (13, 23), (13, 1001), (25, 3)])
def test_fused_inference_matches_layered_forward(L, B):
    """The fused kernel runs the layered forward's operations in the same
    order: identical logits, bit for bit, on ragged batches (partial sample
    groups, partial 16-pixel tiles)."""
    props = torch.cuda.get_device_properties(0)
    say(f"infer L={L} B={B} (LDS per block {getattr(props, 'shared_memory_per_block', '?')})")
    syn = torch.from_numpy(uniform_syndromes(L, B, SEED + 31 * L + B, density=0.15)).to(DEV)
    p = torch.from_numpy(uniform_rates(B, SEED + 5 + B)).to(DEV)
    prm = cnn_init(L, SEED + 6)
    rng = np.random.default_rng(SEED + 7)
    prm += rng.normal(0.0, 0.05, size=prm.size).astype(np.float32)   # non-zero biases
    d_prm = torch.from_numpy(prm).to(DEV)
    ref, _ = gate.forward(L, d_prm, syn, p)
    got, _ = gate.infer(L, d_prm, syn, p)
    torch.cuda.synchronize()
    assert torch.equal(got[:, :7], ref[:, :7])


# ---------------------------------------------------------------- training support
@pytest.mark.parametrize("L", [3, 13])
def test_init_params_match_oracle(L):
    """mcmc_cnn_init against the oracle's Box-Muller draws from the same
    Philox words: both compute in double and round to float; the device's
    log and cos may differ from the host's in the last place of the double,
    which reaches the float only at a rounding boundary (1 ulp allowed)."""
    say(f"cnn init L={L}")
    g = gate.init_params(L, 99).cpu().numpy()
    o = cnn.he_init(L, 99)
    np.testing.assert_allclose(g, o, rtol=2 ** -23, atol=0)
    assert (g == o).mean() > 0.999


@pytest.mark.parametrize("n", [1, 5, 64, 1000, 4097, 100000])
def test_epoch_permutation_matches_oracle(n):
    say(f"cnn permutation n={n}")
    g = gate.permutation(n, 0xABC, 3).cpu().numpy()
    if n <= 4097:
        assert np.array_equal(g, cnn.epoch_permutation(n, 0xABC, 3))
    assert np.array_equal(np.sort(g), np.arange(n))


def test_budget_labels_match_oracle():
    say("budget labels")
    rng = np.random.default_rng(4)
    d = [torch.from_numpy(rng.integers(0, 4, 5000).astype(np.uint8)).to(DEV) for _ in range(3)]
    g = gate.budget_labels(*d).cpu().numpy()
    o = cnn.budget_labels(*(x.cpu().numpy() for x in d))
    assert np.array_equal(g, o)


def test_train_epochs_equal_the_step_sequence():
    """mcmc_cnn_train_epoch equals its definition run from the single-step
    entry points: each epoch's shuffle, mini-batches in that order, forward,
    backward, one Adam step at the scheduled rate; parameters, moments and the
    epoch loss sums bit for bit."""
    say("train epoch vs steps")
    L, n, B, epochs, lr = 5, 700, 128, 2, 2e-3
    syn = torch.from_numpy(uniform_syndromes(L, n, seed=31, density=0.2)).to(DEV)
    p = torch.from_numpy(uniform_rates(n, 32)).to(DEV)
    t_np, b_np = cnn_targets(n, 33)
    tgt = torch.from_numpy(t_np).to(DEV)
    bud = torch.from_numpy(b_np).to(DEV)
    init = gate.init_params(L, 7)
    net = gate.GateNet(L, init, device=DEV)
    hist = gate.train(net, syn, p, tgt, bud, epochs=epochs, batch=B, lr=lr, seed=21)
    # the definition, step by step
    prm = init.clone()
    m = torch.zeros_like(prm)
    v = torch.zeros_like(prm)
    total = epochs * (n // B)
    t = 0
    ref_hist = []
    for e in range(epochs):
        perm = torch.from_numpy(cnn.epoch_permutation(n, 21, e)).to(DEV)
        acc = 0.0
        for s in range(0, n - B + 1, B):
            idx = perm[s:s + B]
            logits, ws = gate.forward(L, prm, syn[idx], p[idx])
            grads, loss = gate.backward(L, prm, logits, tgt[idx], bud[idx], ws, 0.5)
            lo, hi = np.float64(np.float32(lr)), np.float64(np.float32(lr / 10.0))
            rate = np.float32(lo + (hi - lo) * (t / max(1, total - 1)))
            t += 1
            gate.adam_step(prm, grads, m, v, t, lr=float(rate))
            bs = 0.0
            for x in loss.double().cpu().numpy():
                bs += x
            acc += bs
        ref_hist.append(acc / ((n // B) * B))
    torch.cuda.synchronize()
    assert torch.equal(prm, net.params)
    assert torch.equal(m, net.m) and torch.equal(v, net.v)
    assert hist == ref_hist
    assert net.step_count == total
