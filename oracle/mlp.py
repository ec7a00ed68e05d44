"""FP64 CPU oracle of the learned subspace selection's network (numpy).

TEST INFRASTRUCTURE ONLY: imported by tests/. The HIP library and its binding never import it.

Not part of the paper's method: the learned selection replaces the Gamma row of Section 5.6 by
a network's softmax mixed with that row. What is fixed here is the interface both sides share:
  * 9 input features per query (position scaled to the scene box, shading normal, unit direction
    toward the previous eye vertex), each encoded as
    [f, sin(2^0 pi f), cos(2^0 pi f), ..., sin(2^11 pi f), cos(2^11 pi f)] -> 225 values,
    zero-padded to 256;
  * three hidden layers of 64 ReLU units and n_out logits, h_{l+1} = relu(h_l W_l + b_l),
    logits = h_3 W_4 + b_4;
  * parameters as one flat vector W1[256][64], b1, W2[64][64], b2, W3[64][64], b3,
    W4[64][n_out], b4 (row-major, input index first);
  * loss = sum_i w_i CE(softmax(logits_i), S_i) / sum_i w_i;
  * Adam (Kingma and Ba, 2015) with bias corrections.
Everything is written out in plain matrix form; no fusion.

The network's stated precision is BF16 storage with FP32 accumulation. With bf16=True the
forward and backward passes round to BF16 (round to nearest even) where that format stores
values: the encoded inputs, the weight matrices, the hidden activations, the logit gradient and
every hidden pre-activation gradient; products and sums stay in FP64 (the accumulation error is
far below the storage rounding). Biases stay in their FP32 values. The encoding's arguments are
formed in FP32 as well (FP32 features: fp32(f pi), then exact doublings), since at 2^11 pi the
argument's FP32 rounding moves about one encoded input in a hundred to the neighbouring BF16
value, which the gradient feels.
"""
import numpy as np

N_IN = 256
N_ENC = 225
N_H = 64
BANDS = 12


def round_bf16(x):
    """Round to the nearest BF16 value (ties to even), through FP32 (NaN and infinity not handled)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def encode(feat, fp32_args=False):
    """feat [n, 9] -> [n, 256] in the order raw, (sin, cos) per band, per feature. fp32_args: the
    argument of band b is fp32(fp32(f) fp32(pi)) 2^b (doubling is exact), then sin/cos exactly."""
    feat = np.asarray(feat, dtype=np.float64)
    n = feat.shape[0]
    X = np.zeros((n, N_IN))
    col = 0
    for j in range(9):
        X[:, col] = feat[:, j]
        col += 1
        base = (feat[:, j].astype(np.float32) * np.float32(np.pi)).astype(np.float64) if fp32_args else \
            np.pi * feat[:, j]
        for b in range(BANDS):
            a = (2.0 ** b) * base
            X[:, col] = np.sin(a)
            X[:, col + 1] = np.cos(a)
            col += 2
    assert col == N_ENC
    return X


def layout(n_out):
    """(name, shape) of every parameter block in the flat vector's order."""
    return [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
            ("W3", (N_H, N_H)), ("b3", (N_H,)), ("W4", (N_H, n_out)), ("b4", (n_out,))]


def count(n_out):
    return sum(int(np.prod(s)) for _, s in layout(n_out))


def unpack(params, n_out):
    params = np.asarray(params, dtype=np.float64)
    assert params.size == count(n_out)
    out, o = {}, 0
    for name, shape in layout(n_out):
        k = int(np.prod(shape))
        out[name] = params[o:o + k].reshape(shape)
        o += k
    return out


def pack(blocks, n_out):
    return np.concatenate([np.asarray(blocks[name], dtype=np.float64).ravel() for name, _ in layout(n_out)])


def _store(bf16):
    return round_bf16 if bf16 else (lambda a: a)


def weights(params, n_out, bf16=False):
    """Parameter blocks as the passes use them (weight matrices in BF16 when bf16)."""
    P = unpack(params, n_out)
    if bf16:
        P = {k: (round_bf16(v) if k.startswith("W") else v) for k, v in P.items()}
    return P


def forward(params, n_out, feat, bf16=False):
    """Logits [n, n_out] and the intermediate values (for the backward pass)."""
    st = _store(bf16)
    P = weights(params, n_out, bf16)
    X = st(encode(feat, fp32_args=bf16))
    Z1 = X @ P["W1"] + P["b1"]
    H1 = st(np.maximum(Z1, 0.0))
    Z2 = H1 @ P["W2"] + P["b2"]
    H2 = st(np.maximum(Z2, 0.0))
    Z3 = H2 @ P["W3"] + P["b3"]
    H3 = st(np.maximum(Z3, 0.0))
    L = H3 @ P["W4"] + P["b4"]
    return L, dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, Z3=Z3, H3=H3)


def log_softmax(L):
    m = L.max(axis=1, keepdims=True)
    return L - m - np.log(np.exp(L - m).sum(axis=1, keepdims=True))


def loss(params, n_out, feat, label, weight):
    """Weighted mean cross entropy."""
    L, _ = forward(params, n_out, feat)
    lp = log_softmax(L)
    w = np.asarray(weight, dtype=np.float64)
    return float(-(w * lp[np.arange(L.shape[0]), np.asarray(label)]).sum() / w.sum())


def grad(params, n_out, feat, label, weight, bf16=False):
    """Gradient of loss() by the chain rule, layer by layer (flat vector, same layout)."""
    st = _store(bf16)
    P = weights(params, n_out, bf16)
    L, a = forward(params, n_out, feat, bf16)
    w = np.asarray(weight, dtype=np.float64)
    n = L.shape[0]
    # d loss / d logits = w_i / W (softmax_i - onehot(S_i))
    G4 = np.exp(log_softmax(L))
    G4[np.arange(n), np.asarray(label)] -= 1.0
    G4 = st(G4 * (w / w.sum())[:, None])
    g = {"W4": a["H3"].T @ G4, "b4": G4.sum(axis=0)}
    dH3 = G4 @ P["W4"].T
    dZ3 = st(dH3 * (a["Z3"] > 0))
    g["W3"] = a["H2"].T @ dZ3
    g["b3"] = dZ3.sum(axis=0)
    dH2 = dZ3 @ P["W3"].T
    dZ2 = st(dH2 * (a["Z2"] > 0))
    g["W2"] = a["H1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2 @ P["W2"].T
    dZ1 = st(dH1 * (a["Z1"] > 0))
    g["W1"] = a["X"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return pack(g, n_out)


def grad_scale(params, n_out, feat, label, weight):
    """Per block, sqrt(sum_i ||per-sample gradient_i||^2) of the loss's gradient (each sample's term
    of a weight block is the outer product of that layer's input and output gradient, so its
    Frobenius norm is the product of the two vectors' norms). This is the scale of the error of
    a gradient whose per-sample terms each carry a small relative error and whose sum cancels."""
    P = unpack(params, n_out)
    L, a = forward(params, n_out, feat)
    w = np.asarray(weight, dtype=np.float64)
    n = L.shape[0]
    G4 = np.exp(log_softmax(L))
    G4[np.arange(n), np.asarray(label)] -= 1.0
    G4 *= (w / w.sum())[:, None]
    rows = lambda M: np.sqrt((M * M).sum(axis=1))  # noqa: E731
    out = {"W4": np.sqrt(((rows(a["H3"]) * rows(G4)) ** 2).sum()), "b4": np.sqrt((rows(G4) ** 2).sum())}
    dZ = G4
    for l, (h, z) in zip((4, 3, 2), (("H2", "Z3"), ("H1", "Z2"), ("X", "Z1"))):
        dZ = (dZ @ P[f"W{l}"].T) * (a[z] > 0)
        out[f"W{l - 1}"] = np.sqrt(((rows(a[h]) * rows(dZ)) ** 2).sum())
        out[f"b{l - 1}"] = np.sqrt((rows(dZ) ** 2).sum())
    return out


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
