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

The proxy-retrace direction head: when n_out = n_spec + 40, the outputs after the n_spec logits are
an 8-lobe von Mises-Fisher mixture over directions on the unit sphere, 5 values per lobe: the mean
direction (3 values, normalised), the log concentration (clamped to [LOG_KAPPA_MIN, LOG_KAPPA_MAX])
and the lobe's mixture logit. A lobe's density is the vMF density
    p(w) = kappa / (2 pi (1 - exp(-2 kappa))) exp(-kappa (1 - mu.w)),
with 1 - mu.w written as |mu - w|^2 / 2 (equal for unit vectors, and free of cancellation near
mu). It is trained on the weighted negative log-likelihood of the retrace directions of the
proxy contributions: loss_vmf = -sum_i w_i log p_mix(w_i | x_i) / sum_i w_i, added to the cross
entropy of the subspace rows.

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
N_LOBES = 8
VMF_OUT = 5 * N_LOBES
LOG_KAPPA_MIN, LOG_KAPPA_MAX = -3.0, 10.0


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


# ------------------------------------------------------------------ vMF retrace-direction head
def vmf_lobes(R):
    """Raw outputs R [n, 40] (bias included) -> per lobe: unit mean mu [n, 8, 3], concentration kappa
    [n, 8], mixture weight pi [n, 8] (softmax of the lobe logits), the norm of the raw direction
    [n, 8] and whether the log concentration lies strictly inside its clamp range [n, 8]."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, N_LOBES, 5)
    m = R[..., :3]
    nrm = np.sqrt((m * m).sum(-1))
    # a vanishing raw direction gives the +z axis
    mu = np.where((nrm > 1e-20)[..., None], m / np.maximum(nrm, 1e-300)[..., None], np.array([0.0, 0.0, 1.0]))
    s = R[..., 3]
    inside = (s > LOG_KAPPA_MIN) & (s < LOG_KAPPA_MAX)
    kappa = np.exp(np.clip(s, LOG_KAPPA_MIN, LOG_KAPPA_MAX))
    lg = R[..., 4]
    e = np.exp(lg - lg.max(-1, keepdims=True))
    return mu, kappa, e / e.sum(-1, keepdims=True), nrm, inside


def vmf_lobe_pdf(mu, kappa, w):
    """The von Mises-Fisher density on the unit sphere (solid-angle measure)."""
    d = mu - w
    h = 0.5 * (d * d).sum(-1)            # 1 - mu.w for unit vectors
    return kappa / (2.0 * np.pi * -np.expm1(-2.0 * kappa)) * np.exp(-kappa * h)


def vmf_pdf(R, w):
    """Mixture density of the raw outputs R [n, 40] at the unit directions w [n, 3]."""
    mu, kappa, pi, _, _ = vmf_lobes(R)
    return (pi * vmf_lobe_pdf(mu, kappa, np.asarray(w, dtype=np.float64)[:, None, :])).sum(-1)


def vmf_nll_grad(R, w):
    """d(-log p_mix(w)) / dR [n, 40] by the chain rule, with responsibilities r_k = pi_k p_k / p_mix:
    lobe logit pi_k - r_k; log concentration -r_k (1 - 2 kappa / (exp(2 kappa) - 1) - kappa h)
    (zero where the clamp is active), with h = 1 - mu.w; raw direction m:
    -r_k kappa (w - (mu.w) mu) / |m|."""
    w = np.asarray(w, dtype=np.float64)
    mu, kappa, pi, nrm, inside = vmf_lobes(R)
    ww = w[:, None, :]
    v = vmf_lobe_pdf(mu, kappa, ww)
    r = pi * v / (pi * v).sum(-1, keepdims=True)
    h = 0.5 * ((mu - ww) ** 2).sum(-1)
    two_k = 2.0 * kappa
    ratio = np.where(two_k < 700.0, two_k / np.expm1(np.minimum(two_k, 700.0)), 0.0)
    G = np.zeros(mu.shape[:2] + (5,))
    G[..., 4] = pi - r
    G[..., 3] = np.where(inside, -r * (1.0 - ratio - kappa * h), 0.0)
    cosw = (mu * ww).sum(-1)
    G[..., :3] = np.where((nrm > 1e-20)[..., None],
                          -(r * kappa / np.maximum(nrm, 1e-300))[..., None] * (ww - cosw[..., None] * mu), 0.0)
    return G.reshape(-1, VMF_OUT)


def vmf_sample(R, u):
    """Directions drawn from the mixtures of R [n, 40] with uniforms u [n, 4]: the lobe by inverse CDF
    of pi (u0), then 1 - mu.w = -log(u1 + (1 - u1) exp(-2 kappa)) / kappa (the inverse CDF of the
    vMF's cosine) and the azimuth 2 pi u2 about mu."""
    mu, kappa, pi, _, _ = vmf_lobes(R)
    u = np.asarray(u, dtype=np.float64)
    n = mu.shape[0]
    k = np.minimum((np.cumsum(pi, -1) <= u[:, :1]).sum(-1), N_LOBES - 1)
    m, kp = mu[np.arange(n), k], kappa[np.arange(n), k]
    h = -np.log(u[:, 1] + (1.0 - u[:, 1]) * np.exp(-2.0 * kp)) / kp
    st = np.sqrt(np.maximum(h * (2.0 - h), 0.0))
    a = np.where(np.abs(m[:, 0:1]) > 0.9, [[0.0, 1.0, 0.0]], [[1.0, 0.0, 0.0]])
    t = np.cross(m, a)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    b = np.cross(m, t)
    ph = 2.0 * np.pi * u[:, 2]
    return (1.0 - h)[:, None] * m + st[:, None] * (np.cos(ph)[:, None] * t + np.sin(ph)[:, None] * b)


# ------------------------------------------------------------------ losses and gradients
def _output_grad(L, n_spec, n_ce, label, w_ce, dirs, w_v):
    """d loss / d outputs [n_ce + n_v, n_out]: the cross-entropy rows over the first n_spec columns,
    then the vMF rows over the 40 columns after them."""
    G = np.zeros_like(L)
    if n_ce:
        lp = log_softmax(L[:n_ce, :n_spec])
        Gc = np.exp(lp)
        Gc[np.arange(n_ce), np.asarray(label)] -= 1.0
        G[:n_ce, :n_spec] = Gc * (w_ce / w_ce.sum())[:, None]
    if dirs is not None and len(dirs):
        G[n_ce:, n_spec:n_spec + VMF_OUT] = vmf_nll_grad(L[n_ce:, n_spec:n_spec + VMF_OUT], dirs) * \
            (w_v / w_v.sum())[:, None]
    return G


def _rows(feat, vmf):
    f = [np.asarray(feat, dtype=np.float64).reshape(-1, 9)] if feat is not None else [np.zeros((0, 9))]
    if vmf is not None:
        f.append(np.asarray(vmf[0], dtype=np.float64).reshape(-1, 9))
    return np.concatenate(f, axis=0)


def loss(params, n_out, feat, label, weight, n_spec=None, vmf=None):
    """Weighted mean cross entropy of the subspace rows (softmax over the first n_spec outputs;
    n_spec = n_out without the direction head), plus, given vmf = (feat, dirs, weight), the
    weighted mean negative log-likelihood of the directions under the vMF mixture."""
    n_spec = n_out if n_spec is None else n_spec
    total = 0.0
    if feat is not None and len(feat):
        L, _ = forward(params, n_out, feat)
        lp = log_softmax(L[:, :n_spec])
        w = np.asarray(weight, dtype=np.float64)
        total += float(-(w * lp[np.arange(L.shape[0]), np.asarray(label)]).sum() / w.sum())
    if vmf is not None and len(vmf[0]):
        L, _ = forward(params, n_out, vmf[0])
        wv = np.asarray(vmf[2], dtype=np.float64)
        p = vmf_pdf(L[:, n_spec:n_spec + VMF_OUT], vmf[1])
        total += float(-(wv * np.log(p)).sum() / wv.sum())
    return total


def grad(params, n_out, feat, label, weight, bf16=False, n_spec=None, vmf=None):
    """Gradient of loss() by the chain rule, layer by layer (flat vector, same layout). The
    cross-entropy rows and the direction rows (vmf) pass through the network as one batch."""
    n_spec = n_out if n_spec is None else n_spec
    st = _store(bf16)
    P = weights(params, n_out, bf16)
    rows = _rows(feat, vmf)
    n_ce = 0 if feat is None else len(feat)
    L, a = forward(params, n_out, rows, bf16)
    w_ce = np.asarray(weight, dtype=np.float64) if n_ce else None
    dirs, w_v = (vmf[1], np.asarray(vmf[2], dtype=np.float64)) if vmf is not None else (None, None)
    G4 = st(_output_grad(L, n_spec, n_ce, label, w_ce, dirs, w_v))
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


def grad_scale(params, n_out, feat, label, weight, n_spec=None, vmf=None):
    """Per block, sqrt(sum_i ||per-sample gradient_i||^2) of the loss's gradient (each sample's term
    of a weight block is the outer product of that layer's input and output gradient, so its
    Frobenius norm is the product of the two vectors' norms). This is the scale of the error of
    a gradient whose per-sample terms each carry a small relative error and whose sum cancels."""
    n_spec = n_out if n_spec is None else n_spec
    P = unpack(params, n_out)
    rows = _rows(feat, vmf)
    n_ce = 0 if feat is None else len(feat)
    L, a = forward(params, n_out, rows)
    w_ce = np.asarray(weight, dtype=np.float64) if n_ce else None
    dirs, w_v = (vmf[1], np.asarray(vmf[2], dtype=np.float64)) if vmf is not None else (None, None)
    G4 = _output_grad(L, n_spec, n_ce, label, w_ce, dirs, w_v)
    rn = lambda M: np.sqrt((M * M).sum(axis=1))  # noqa: E731
    out = {"W4": np.sqrt(((rn(a["H3"]) * rn(G4)) ** 2).sum()), "b4": np.sqrt((rn(G4) ** 2).sum())}
    dZ = G4
    for l, (h, z) in zip((4, 3, 2), (("H2", "Z3"), ("H1", "Z2"), ("X", "Z1"))):
        dZ = (dZ @ P[f"W{l}"].T) * (a[z] > 0)
        out[f"W{l - 1}"] = np.sqrt(((rn(a[h]) * rn(dZ)) ** 2).sum())
        out[f"b{l - 1}"] = np.sqrt((rn(dZ) ** 2).sum())
    return out


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
