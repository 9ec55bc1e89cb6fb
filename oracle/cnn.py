"""Float64 reference of the gate network (not part of the paper: the learned
budget gate grown on the decoder), forward and backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network over an L x L grid, channels last:
  input  3 planes: lit stars (i, j) at (y, x) = (i, j) (row L-1 empty), lit
         plaquettes (i, j) at (i, j) (column L-1 empty), and p everywhere
  conv1  3 -> 32, 3x3, zero padding, bias, ReLU
  conv2  32 -> 32, same
  conv3  32 -> 32, same
  head   linear over the flattened conv3 output (feature f = pixel*32 + c)
         -> 7 logits: 4 class logits, 3 budget logits ({0, L, L^2} sweeps)
Tap t = (dy+1)*3 + (dx+1).  Weights: W[c_out][tap][c_in].

Loss per sample: soft cross-entropy of the class logits against the MCMC
class probabilities, plus w_b times the cross-entropy of the budget logits
against the budget label; averaged over the batch.

`bf16=True` reproduces the rounding points of the GPU kernels (operands of
every matrix product in bfloat16, round-to-nearest-even; accumulation exact
here): input p, all weights used in products, the ReLU outputs, and the
back-propagated pre-activation gradients of the three convolutions.  With
bf16=False everything is plain float64 (used for the finite-difference pin).
"""

import numpy as np

C = 32
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def to_bf16(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits, ties
    to even) and return them as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def param_shapes(L):
    return [("W1", (C, 9, 3)), ("b1", (C,)), ("W2", (C, 9, C)), ("b2", (C,)),
            ("W3", (C, 9, C)), ("b3", (C,)), ("Wh", (7, L * L * C)), ("bh", (7,))]


def unflatten(L, flat):
    out, off = {}, 0
    for name, shape in param_shapes(L):
        size = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + size], dtype=np.float64).reshape(shape)
        off += size
    return out


def flatten(L, params):
    return np.concatenate([np.asarray(params[n], dtype=np.float64).reshape(-1)
                           for n, _ in param_shapes(L)])


def encode(L, syndromes, p):
    """[B, L, L, 3] float64 input planes (before any rounding)."""
    syn = np.asarray(syndromes, dtype=np.float64)
    B = syn.shape[0]
    ns = L * (L - 1)
    x = np.zeros((B, L, L, 3))
    x[:, :L - 1, :, 0] = syn[:, :ns].reshape(B, L - 1, L)
    x[:, :, :L - 1, 1] = syn[:, ns:].reshape(B, L, L - 1)
    x[:, :, :, 2] = np.asarray(p, dtype=np.float64)[:, None, None]
    return x


def _shift(x, dy, dx):
    """out[b, y, x] = x[b, y+dy, x+dx] with zeros outside."""
    B, H, W, Cc = x.shape
    out = np.zeros_like(x)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    out[:, ys:ye, xs:xe] = x[:, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv(x, W, b):
    """y[b,y,x,co] = sum_{tap,ci} x[b, y+dy, x+dx, ci] W[co, tap, ci] + b[co]."""
    y = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        y += _shift(x, dy, dx) @ W[:, t, :].T
    return y + b


def forward(L, params, syndromes, p, bf16=True):
    r = to_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    P = {k: (r(v) if k.startswith("W") else np.asarray(v, dtype=np.float64))
         for k, v in params.items()}
    x0 = r(encode(L, syndromes, p))
    a1 = r(np.maximum(conv(x0, P["W1"], P["b1"]), 0.0))
    a2 = r(np.maximum(conv(a1, P["W2"], P["b2"]), 0.0))
    a3 = r(np.maximum(conv(a2, P["W3"], P["b3"]), 0.0))
    B = x0.shape[0]
    flat = a3.reshape(B, -1)
    logits = flat @ P["Wh"].T + P["bh"]
    return logits, dict(x0=x0, a1=a1, a2=a2, a3=a3, P=P)


def _softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_dlogits(logits, class_target, budget_target, budget_weight):
    B = logits.shape[0]
    pc = _softmax(logits[:, :4])
    pb = _softmax(logits[:, 4:7])
    t = np.asarray(class_target, dtype=np.float64)
    y = np.asarray(budget_target, dtype=np.int64)
    lc = -(t * np.log(pc)).sum(axis=1)
    lb = -np.log(pb[np.arange(B), y])
    loss = (lc + budget_weight * lb).mean()
    dz = np.zeros_like(logits)
    dz[:, :4] = (pc - t) / B
    onehot = np.zeros((B, 3))
    onehot[np.arange(B), y] = 1.0
    dz[:, 4:7] = budget_weight * (pb - onehot) / B
    return loss, dz, lc + budget_weight * lb


def _conv_backward(x, dpre, W):
    """Gradients of conv(x, W, b) given dL/d(pre-activation)."""
    dW = np.zeros_like(W)
    for t, (dy, dx) in enumerate(TAPS):
        xs = _shift(x, dy, dx)
        dW[:, t, :] = np.einsum("byxo,byxi->oi", dpre, xs)
    db = dpre.sum(axis=(0, 1, 2))
    dx_ = np.zeros(x.shape)
    for t, (dy, dx) in enumerate(TAPS):
        dx_ += _shift(dpre, -dy, -dx) @ W[:, t, :]
    return dW, db, dx_


def backward(L, params, syndromes, p, class_target, budget_target, budget_weight=0.5, bf16=True):
    """(loss, per-sample losses, grads dict, logits)."""
    r = to_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    logits, st = forward(L, params, syndromes, p, bf16)
    loss, dz, per = loss_and_dlogits(logits, class_target, budget_target, budget_weight)
    P = st["P"]
    B = logits.shape[0]
    a3f = st["a3"].reshape(B, -1)
    g = {"Wh": dz.T @ a3f, "bh": dz.sum(axis=0)}
    da3 = (dz @ P["Wh"]).reshape(st["a3"].shape)
    dpre3 = r(da3 * (st["a3"] > 0))
    g["W3"], g["b3"], da2 = _conv_backward(st["a2"], dpre3, P["W3"])
    dpre2 = r(da2 * (st["a2"] > 0))
    g["W2"], g["b2"], da1 = _conv_backward(st["a1"], dpre2, P["W2"])
    dpre1 = r(da1 * (st["a1"] > 0))
    g["W1"], g["b1"], _ = _conv_backward(st["x0"], dpre1, P["W1"])
    return loss, per, g, logits


def adam(params, grads, m, v, lr, beta1, beta2, eps, step):
    """One Adam step (bias-corrected), element by element, float64."""
    out_p, out_m, out_v = {}, {}, {}
    for k in params:
        mm = beta1 * m[k] + (1 - beta1) * grads[k]
        vv = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = mm / (1 - beta1 ** step)
        vh = vv / (1 - beta2 ** step)
        out_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
        out_m[k], out_v[k] = mm, vv
    return out_p, out_m, out_v


# ---------------------------------------------------------------------------
# Training support: initial parameters, budget labels, relative class
# targets, the epoch shuffle.
# Philox4x32-10 with key = seed, fourth counter word 3<<30 | 3<<28 | field<<20
# (field 0xFE: initial weights, 0xFD: shuffle).
# ---------------------------------------------------------------------------
def _ctr3(field):
    return (3 << 30) | (3 << 28) | (field << 20)


def he_init(L, seed):
    """Initial parameters (float32 [param_count]): weight i of a block with
    fan-in f is sqrt(-2 ln u1) cos(2 pi u2) sqrt(2/f) (Box-Muller), u1 =
    (a + 1) / 2^32, u2 = b / 2^32, (a, b) = words 2(i&1), 2(i&1)+1 of Philox
    at counter (i >> 1, 0, 0, ctr3(0xFE)); biases zero.  Blocks: W1 [32][9][3]
    (f = 27), b1, W2 [32][9][32] (f = 288), b2, W3 (f = 288), b3,
    Wh [7][32 L^2] (f = 32 L^2), bh."""
    from . import philox
    sizes = [(C * 9 * 3, 27), (C, 0), (C * 9 * C, 9 * C), (C, 0), (C * 9 * C, 9 * C), (C, 0),
             (7 * L * L * C, L * L * C), (7, 0)]
    total = sum(s for s, _ in sizes)
    fan = np.zeros(total)
    at = 0
    for size, f in sizes:
        fan[at:at + size] = f
        at += size
    i = np.arange(total, dtype=np.uint64)
    k0, k1 = philox.seed_key(seed)
    w = philox.philox4x32_10(i >> np.uint64(1), 0, 0, _ctr3(0xFE), k0, k1)
    odd = (i & np.uint64(1)).astype(bool)
    a = np.where(odd, w[2], w[0]).astype(np.float64)
    b = np.where(odd, w[3], w[1]).astype(np.float64)
    u1 = (a + 1.0) * 2.0 ** -32
    u2 = b * 2.0 ** -32
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    out = np.where(fan > 0, z * np.sqrt(2.0 / np.maximum(fan, 1)), 0.0)
    return out.astype(np.float32)


def budget_labels(d_zero, d_short, d_full):
    """0 if the no-sweep decision is the full-budget one, else 1 if the short
    budget's is, else 2."""
    d_zero, d_short, d_full = (np.asarray(v) for v in (d_zero, d_short, d_full))
    return np.where(d_zero == d_full, 0, np.where(d_short == d_full, 1, 2)).astype(np.int32)


# The start-weight gap route (a rule beside the network, not in the paper):
# the decision from the class starts alone is taken when the gap between the
# lightest and the second-lightest class start reaches a threshold that
# depends on the error rate.  The rate axis is cut into GAP_BINS bins of
# GAP_BIN_WIDTH; GAP_NEVER marks a bin whose threshold no gap reaches.
GAP_BINS = 50
GAP_BIN_WIDTH = 0.01
GAP_NEVER = 255


def start_weight_gap(weights):
    """int64 [n]: second-smallest minus smallest of each row of the [n][4]
    class start weights."""
    w = np.sort(np.asarray(weights, dtype=np.int64), axis=1)
    return w[:, 1] - w[:, 0]


def gap_bin(p):
    """int64 [n]: the rate bin floor(p * 100), computed in fp32 as the gate
    kernel does (p as fp32, the product rounded to fp32), capped at
    GAP_BINS - 1."""
    q = np.asarray(p, dtype=np.float32) * np.float32(1.0 / GAP_BIN_WIDTH)
    return np.minimum(np.floor(q).astype(np.int64), GAP_BINS - 1)


def fit_gap_table(p, weights, budget, max_miss, min_count):
    """uint8 [GAP_BINS]: per rate bin, the smallest gap threshold G such that
    among the bin's samples with gap >= G at least min_count remain and the
    fraction whose budget label is not 0 (the no-sweep decision differs from
    the full-budget one) is at most max_miss; GAP_NEVER if no G < GAP_NEVER
    qualifies.  Written out by the definition, G by G."""
    gap = start_weight_gap(weights)
    b = gap_bin(p)
    miss = np.asarray(budget) != 0
    table = np.full(GAP_BINS, GAP_NEVER, dtype=np.uint8)
    for k in range(GAP_BINS):
        gk, mk = gap[b == k], miss[b == k]
        for G in range(GAP_NEVER):
            sel = gk >= G
            cnt = int(sel.sum())
            if cnt < min_count:
                break
            if int(mk[sel].sum()) <= max_miss * cnt:
                table[k] = G
                break
    return table


def gap_route(p, weights, table):
    """bool [n]: the gap route takes the syndrome (gap >= its bin's
    threshold, a GAP_NEVER threshold never)."""
    t = np.asarray(table, dtype=np.int64)[gap_bin(p)]
    return (t != GAP_NEVER) & (start_weight_gap(weights) >= t)


def relative_targets(class_prob, start_class):
    """Class targets read relative to the start decision: out[i][k] =
    class_prob[i][k ^ start_class[i]].  A class is bx + 2 bz with bx, bz the
    parities of the two logical operators (geometry.class_index), so
    composing an error with a class-c operator maps class e to e ^ c, and
    entry 0 is the probability that the start decision is the right class."""
    prob = np.asarray(class_prob)
    s = np.asarray(start_class).astype(np.int64)
    k = np.arange(4)
    return prob[np.arange(prob.shape[0])[:, None], k[None, :] ^ s[:, None]]


def epoch_permutation(n, seed, epoch):
    """int64 [n]: position i -> a 4-round Feistel network on b bits (b the
    smallest even number >= 2 with 2^b >= n, halves of h = b/2 bits,
    (l, r) -> (r, l xor F_k(r)), F_k(r) = low h bits of Philox word 0 at
    counter (r, k, epoch, ctr3(0xFD))), repeated until the value is below n."""
    from . import philox
    b = 2
    while (1 << b) < n:
        b += 2
    h = b // 2
    mask = (1 << h) - 1
    k0, k1 = philox.seed_key(seed)

    def f(k, r):
        return int(philox.philox4x32_10(r, k, epoch, _ctr3(0xFD), k0, k1)[0]) & mask

    def net(x):
        left, right = x >> h, x & mask
        for k in range(4):
            left, right = right, left ^ f(k, right)
        return (left << h) | right

    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        y = net(i)
        while y >= n:
            y = net(y)
        out[i] = y
    return out
