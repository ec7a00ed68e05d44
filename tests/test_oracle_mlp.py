"""Pins of the FP64 network oracle (oracle/mlp.py) against facts that do not come from it:
closed forms of the encoding, the loss and Adam, central finite differences and an independent
reverse-mode differentiation (torch.autograd in float64 on the CPU)."""
import numpy as np
import pytest

from oracle import mlp

N_OUT = 24


def _params(rng, n_out=N_OUT, scale=1.0):
    blocks = {}
    for name, shape in mlp.layout(n_out):
        fan = shape[0] if len(shape) == 2 else 1
        blocks[name] = rng.normal(0.0, scale / np.sqrt(fan), size=shape) if len(shape) == 2 else \
            rng.normal(0.0, 0.1, size=shape)
    return mlp.pack(blocks, n_out)


def _data(rng, n, n_out=N_OUT):
    feat = rng.uniform(-1.0, 1.0, size=(n, 9))
    label = rng.integers(0, n_out, size=n)
    weight = rng.exponential(1.0, size=n)
    return feat, label, weight


def test_encoding_closed_form():
    f = np.zeros((3, 9))
    f[1, :] = 0.5
    f[2, 4] = 0.25
    X = mlp.encode(f)
    assert X.shape == (3, 256)
    assert np.all(X[:, 225:] == 0.0)
    # f = 0: raw 0, sin 0, cos 1 in every band
    row = X[0, :25]
    assert row[0] == 0.0 and np.all(row[1::2] == 0.0) and np.all(row[2::2] == 1.0)
    # f = 1/2: band 0 -> (1, 0), band 1 -> (0, -1), bands >= 2 -> (0, 1)
    row = X[1, 25:50]
    assert row[0] == 0.5
    np.testing.assert_allclose(row[1:3], [1.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(row[3:5], [0.0, -1.0], atol=1e-12)
    np.testing.assert_allclose(row[5::2], 0.0, atol=1e-9)
    np.testing.assert_allclose(row[6::2], 1.0, atol=1e-12)
    # feature 4 at 1/4 occupies columns 100..124: band 0 -> (sqrt(1/2), sqrt(1/2)), band 1 -> (1, 0)
    row = X[2, 100:125]
    assert row[0] == 0.25
    np.testing.assert_allclose(row[1:3], [np.sqrt(0.5), np.sqrt(0.5)], atol=1e-12)
    np.testing.assert_allclose(row[3:5], [1.0, 0.0], atol=1e-12)


def test_parameter_count():
    assert mlp.count(N_OUT) == 256 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * N_OUT + N_OUT


def test_loss_uniform_logits_is_log_n():
    rng = np.random.default_rng(1)
    p = mlp.unpack(_params(rng), N_OUT)
    p = {k: v.copy() for k, v in p.items()}
    p["W4"][:] = 0.0
    p["b4"][:] = 0.0
    feat, label, weight = _data(rng, 17)
    assert mlp.loss(mlp.pack(p, N_OUT), N_OUT, feat, label, weight) == pytest.approx(np.log(N_OUT), rel=1e-14)
    # with uniform logits the bias gradient is sum_i w_i (1/N - onehot) / W
    g = mlp.unpack(mlp.grad(mlp.pack(p, N_OUT), N_OUT, feat, label, weight), N_OUT)
    expect = np.full(N_OUT, 1.0 / N_OUT)
    for i in range(17):
        expect[label[i]] -= weight[i] / weight.sum()
    np.testing.assert_allclose(g["b4"], expect, atol=1e-14)


def test_known_linear_network():
    """A network that passes one input straight through: logits depend on f_0 as written."""
    blocks = {name: np.zeros(shape) for name, shape in mlp.layout(3)}
    blocks["W1"][0, 0] = 1.0        # h1_0 = relu(f_0)
    blocks["W2"][0, 0] = 2.0        # h2_0 = 2 relu(f_0)
    blocks["W3"][0, 0] = 1.0
    blocks["W4"][0, :] = [1.0, -1.0, 0.0]
    blocks["b4"][:] = [0.0, 0.0, 0.5]
    f = np.zeros((2, 9))
    f[0, 0] = 0.75
    f[1, 0] = -0.75
    L, _ = mlp.forward(mlp.pack(blocks, 3), 3, f)
    np.testing.assert_allclose(L, [[1.5, -1.5, 0.5], [0.0, 0.0, 0.5]], atol=1e-15)


def test_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    params = _params(rng)
    feat, label, weight = _data(rng, 9)
    g = mlp.grad(params, N_OUT, feat, label, weight)
    eps = 1e-6
    for _ in range(6):
        d = rng.normal(size=params.size)
        d /= np.linalg.norm(d)
        fd = (mlp.loss(params + eps * d, N_OUT, feat, label, weight) -
              mlp.loss(params - eps * d, N_OUT, feat, label, weight)) / (2 * eps)
        assert fd == pytest.approx(float(g @ d), rel=1e-6, abs=1e-12)
    # single coordinates of every block
    off = 0
    for name, shape in mlp.layout(N_OUT):
        k = int(np.prod(shape))
        idx = off + int(rng.integers(0, k if name != "W1" else 225 * 64))
        e = np.zeros(params.size)
        e[idx] = 1.0
        fd = (mlp.loss(params + eps * e, N_OUT, feat, label, weight) -
              mlp.loss(params - eps * e, N_OUT, feat, label, weight)) / (2 * eps)
        assert fd == pytest.approx(float(g[idx]), rel=1e-5, abs=1e-10), name
        off += k


def test_gradient_against_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    params = _params(rng)
    feat, label, weight = _data(rng, 31)
    g = mlp.grad(params, N_OUT, feat, label, weight)
    blocks = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(params, N_OUT).items()}
    # the encoding written independently with torch ops
    f = torch.tensor(feat, dtype=torch.float64)
    cols = []
    for j in range(9):
        cols.append(f[:, j:j + 1])
        for b in range(12):
            a = f[:, j:j + 1] * (np.pi * 2.0 ** b)
            cols += [torch.sin(a), torch.cos(a)]
    X = torch.cat(cols + [torch.zeros(f.shape[0], 31, dtype=torch.float64)], dim=1)
    h = X
    for l in (1, 2, 3):
        h = torch.relu(h @ blocks[f"W{l}"] + blocks[f"b{l}"])
    logits = h @ blocks["W4"] + blocks["b4"]
    w = torch.tensor(weight, dtype=torch.float64)
    ce = torch.nn.functional.cross_entropy(logits, torch.tensor(label), reduction="none")
    ((w * ce).sum() / w.sum()).backward()
    ref = np.concatenate([blocks[name].grad.numpy().ravel() for name, _ in mlp.layout(N_OUT)])
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


def test_adam_closed_form():
    # with a constant gradient g the bias-corrected moments are g and g^2 at every step, so each
    # step moves w by -lr g / (|g| + eps)
    rng = np.random.default_rng(4)
    w0 = rng.normal(size=50)
    g = rng.normal(size=50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        w, m, v = mlp.adam_step(w, g, m, v, t, lr=1e-3)
        np.testing.assert_allclose(w, w0 - t * 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
    # first step with zero gradient leaves w unchanged
    w1, _, _ = mlp.adam_step(w0, np.zeros(50), np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_array_equal(w1, w0)


def test_grad_scale_single_sample_is_the_gradient_norm():
    # with one sample there is no cancellation: the scale equals each block's gradient norm
    rng = np.random.default_rng(5)
    params = _params(rng)
    feat, label, weight = _data(rng, 1)
    g = mlp.unpack(mlp.grad(params, N_OUT, feat, label, weight), N_OUT)
    sc = mlp.grad_scale(params, N_OUT, feat, label, weight)
    for name, _ in mlp.layout(N_OUT):
        assert sc[name] == pytest.approx(np.linalg.norm(g[name]), rel=1e-12), name
    # and with many samples it bounds the norm of the sum (triangle inequality with Cauchy-Schwarz)
    feat, label, weight = _data(rng, 40)
    g = mlp.unpack(mlp.grad(params, N_OUT, feat, label, weight), N_OUT)
    sc = mlp.grad_scale(params, N_OUT, feat, label, weight)
    for name, _ in mlp.layout(N_OUT):
        assert np.linalg.norm(g[name]) <= sc[name] * np.sqrt(40) * (1 + 1e-12), name


def test_bf16_rounding():
    # BF16 keeps 8 significant bits: spacing 2^-7 in [1, 2); halfway cases go to the even neighbour
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7 + 2.0 ** -9, -2.5, 3.0e-3, 65504.0])
    r = mlp.round_bf16(x)
    np.testing.assert_array_equal(r[:4], [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7])
    assert r[4] == -2.5
    # relative error at most 2^-8 for normal numbers
    assert np.all(np.abs(r[5:] - x[5:]) <= 2.0 ** -8 * np.abs(x[5:]))
    rng = np.random.default_rng(6)
    y = rng.normal(size=10000) * 10.0 ** rng.uniform(-3, 3, size=10000)
    ry = mlp.round_bf16(y)
    assert np.all(np.abs(ry - y) <= 2.0 ** -8 * np.abs(y) * (1 + 1e-6))
    # idempotent, and values with 8 significant bits are kept exactly
    np.testing.assert_array_equal(mlp.round_bf16(ry), ry)


def test_bf16_mode_on_a_known_network():
    """The pass-through network of test_known_linear_network: every value is a BF16 value, so the
    bf16 mode gives the exact logits; a weight of 1 + 2^-9 (below the halfway point to the next
    BF16 value) is stored as 1 and the logits follow."""
    blocks = {name: np.zeros(shape) for name, shape in mlp.layout(3)}
    blocks["W1"][0, 0] = 1.0
    blocks["W2"][0, 0] = 2.0
    blocks["W3"][0, 0] = 1.0
    blocks["W4"][0, :] = [1.0, -1.0, 0.0]
    blocks["b4"][:] = [0.0, 0.0, 0.5]
    f = np.zeros((2, 9))
    f[0, 0] = 0.75
    f[1, 0] = -0.75
    L16, _ = mlp.forward(mlp.pack(blocks, 3), 3, f, bf16=True)
    np.testing.assert_array_equal(L16, [[1.5, -1.5, 0.5], [0.0, 0.0, 0.5]])
    blocks["W1"][0, 0] = 1.0 + 2.0 ** -9
    L64, _ = mlp.forward(mlp.pack(blocks, 3), 3, f)
    L16, _ = mlp.forward(mlp.pack(blocks, 3), 3, f, bf16=True)
    np.testing.assert_allclose(L64[0, :2], [1.5 * (1 + 2.0 ** -9), -1.5 * (1 + 2.0 ** -9)], rtol=1e-15)
    np.testing.assert_array_equal(L16[0], [1.5, -1.5, 0.5])
    # the gradient in bf16 mode: with uniform weights and these exact values the logit gradient
    # (softmax - onehot) / n is rounded once; W4's gradient is h3^T G4 with h3 = (1.5, 0, ...)
    label = np.array([2, 2])
    g16 = mlp.unpack(mlp.grad(mlp.pack(blocks, 3), 3, f, label, np.ones(2), bf16=True), 3)
    Lr = np.array([1.5, -1.5, 0.5])
    sm = np.exp(Lr - Lr.max()) / np.exp(Lr - Lr.max()).sum()
    G0 = mlp.round_bf16((sm - np.array([0, 0, 1.0])) / 2)
    np.testing.assert_allclose(g16["W4"][0], 1.5 * G0, rtol=1e-15)


def test_fp32_argument_encoding():
    # fp32 arguments: exact for features whose products with pi round the same way (f = 0),
    # and within the FP32 rounding of f pi (2^-24 relative), times 2^b, of the exact argument
    f = np.zeros((1, 9))
    np.testing.assert_array_equal(mlp.encode(f, fp32_args=True), mlp.encode(f))
    rng = np.random.default_rng(8)
    f = rng.uniform(0, 1, size=(200, 9)).astype(np.float32).astype(np.float64)
    X, X32 = mlp.encode(f), mlp.encode(f, fp32_args=True)
    for b in range(12):
        cols = [1 + 25 * j + 2 * b for j in range(9)]
        # fp32(pi) and the product each round by at most half an ulp (2^-24 relative)
        bound = 2.0 ** b * np.pi * 2 * 2.0 ** -24 * 1.01 + 1e-15
        assert np.all(np.abs(X32[:, cols] - X[:, cols]) <= bound)


# ------------------------------------------------------------------ vMF retrace-direction head
def _unit(rng, n):
    w = rng.normal(size=(n, 3))
    return w / np.linalg.norm(w, axis=1, keepdims=True)


@pytest.mark.parametrize("log_kappa", [-3.0, 0.0, np.log(30.0), np.log(2.0e4)])
def test_vmf_lobe_density_integrates_to_one(log_kappa):
    """The lobe density, evaluated at directions on the sphere, integrates to one over the sphere
    (quadrature in the polar angle about a tilted mean, uniform in azimuth; dense near the mean
    for large concentrations), and its mixture with identical lobes is that lobe."""
    from scipy import integrate
    kappa = float(np.exp(log_kappa))
    mu = np.array([0.3, -0.5, 0.8])
    mu /= np.linalg.norm(mu)
    a = np.cross(mu, [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(mu, a)

    def ring(theta):
        ph = np.linspace(0.0, 2 * np.pi, 64, endpoint=False)
        w = (np.cos(theta) * mu[None, :] + np.sin(theta) * (np.cos(ph)[:, None] * a + np.sin(ph)[:, None] * b))
        return float(mlp.vmf_lobe_pdf(mu[None, :], np.full(64, kappa), w).mean()) * 2 * np.pi * np.sin(theta)

    pts = [t for t in (0.5 / np.sqrt(kappa), 2 / np.sqrt(kappa), 8 / np.sqrt(kappa)) if t < np.pi]
    tot, _ = integrate.quad(ring, 0.0, np.pi, points=pts, limit=400, epsabs=1e-12, epsrel=1e-10)
    assert tot == pytest.approx(1.0, rel=1e-7)
    # a mixture of eight copies of the lobe is the lobe
    R = np.zeros((5, 40))
    for k in range(8):
        R[:, 5 * k:5 * k + 3] = mu * 2.5
        R[:, 5 * k + 3] = log_kappa
        R[:, 5 * k + 4] = 0.7 * k
    w = _unit(np.random.default_rng(1), 5)
    np.testing.assert_allclose(mlp.vmf_pdf(R, w), mlp.vmf_lobe_pdf(mu[None, :], np.full(5, kappa), w), rtol=1e-13)


def test_vmf_sampling_matches_its_density():
    """Samples of one lobe: the cosine to the mean has the vMF's law (CDF (1 - exp(-kappa h)) /
    (1 - exp(-2 kappa)) of h = 1 - mu.w, Kolmogorov-Smirnov) and mean coth(kappa) - 1/kappa; the
    azimuth is uniform; the lobes of a mixture are drawn with their weights."""
    from scipy import stats
    rng = np.random.default_rng(2)
    n = 200_000
    for kappa in (0.2, 5.0, 3000.0):
        mu = np.array([0.0, 0.6, 0.8])
        R = np.zeros((n, 40))
        R[:, 0:3] = mu * 3.0
        R[:, 3] = np.log(kappa)
        R[:, 4] = 50.0          # the first lobe only
        w = mlp.vmf_sample(R, rng.uniform(size=(n, 4)))
        np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-12)
        h = 1.0 - w @ mu
        cdf = lambda x: -np.expm1(-kappa * x) / -np.expm1(-2 * kappa)  # noqa: E731
        assert stats.kstest(h, cdf).pvalue > 1e-4
        m = float((w @ mu).mean())
        assert abs(m - (1 / np.tanh(kappa) - 1 / kappa)) < 5 * (w @ mu).std() / np.sqrt(n)
    # lobe frequencies under distinct, well separated means
    R = np.zeros((n, 40))
    logits = np.array([0.0, 1.0, -1.0, 0.5, 2.0, -2.0, 0.0, 0.3])
    means = _unit(np.random.default_rng(3), 8)
    for k in range(8):
        R[:, 5 * k:5 * k + 3] = means[k]
        R[:, 5 * k + 3] = np.log(5000.0)
        R[:, 5 * k + 4] = logits[k]
    w = mlp.vmf_sample(R, rng.uniform(size=(n, 4)))
    k = (w @ means.T).argmax(1)
    pi = np.exp(logits) / np.exp(logits).sum()
    counts = np.bincount(k, minlength=8)
    assert stats.chisquare(counts, pi * n).pvalue > 1e-4


def test_vmf_nll_gradient_by_finite_differences():
    """d(-log p_mix)/dR against central differences of the mixture density, on raw outputs whose
    log concentrations lie inside the clamp (and zero for the clamped ones)."""
    rng = np.random.default_rng(4)
    n = 6
    R = rng.normal(size=(n, 40))
    R[:, 3::5] = rng.uniform(-2.5, 4.0, size=(n, 8))
    R[0, 3] = 11.0          # clamped: no gradient through it
    w = _unit(rng, n)
    G = mlp.vmf_nll_grad(R, w)
    eps = 1e-6
    for j in range(40):
        d = np.zeros_like(R)
        d[:, j] = eps
        fd = (-np.log(mlp.vmf_pdf(R + d, w)) + np.log(mlp.vmf_pdf(R - d, w))) / (2 * eps)
        np.testing.assert_allclose(G[:, j], fd, rtol=1e-5, atol=1e-8, err_msg=str(j))
    assert G[0, 3] == 0.0


def test_network_gradient_with_direction_rows():
    """The whole network's gradient with subspace rows and direction rows in one batch, against
    central differences of loss() and against torch.autograd (float64) of the same loss written
    with torch ops (the vMF log-density from its closed form)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    n_spec = 12
    n_out = n_spec + mlp.VMF_OUT
    params = _params(rng, n_out)
    feat, label, weight = _data(rng, 7, n_spec)
    fv = rng.uniform(-1.0, 1.0, size=(5, 9))
    dv = _unit(rng, 5)
    wv = rng.exponential(1.0, size=5)
    vmf = (fv, dv, wv)
    g = mlp.grad(params, n_out, feat, label, weight, n_spec=n_spec, vmf=vmf)
    eps = 1e-6
    for _ in range(6):
        d = rng.normal(size=params.size)
        d /= np.linalg.norm(d)
        fd = (mlp.loss(params + eps * d, n_out, feat, label, weight, n_spec=n_spec, vmf=vmf) -
              mlp.loss(params - eps * d, n_out, feat, label, weight, n_spec=n_spec, vmf=vmf)) / (2 * eps)
        assert fd == pytest.approx(float(g @ d), rel=1e-6, abs=1e-12)
    blocks = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(params, n_out).items()}

    def net(f):
        f = torch.tensor(f, dtype=torch.float64)
        cols = []
        for j in range(9):
            cols.append(f[:, j:j + 1])
            for b in range(12):
                a = f[:, j:j + 1] * (np.pi * 2.0 ** b)
                cols += [torch.sin(a), torch.cos(a)]
        h = torch.cat(cols + [torch.zeros(f.shape[0], 31, dtype=torch.float64)], dim=1)
        for l in (1, 2, 3):
            h = torch.relu(h @ blocks[f"W{l}"] + blocks[f"b{l}"])
        return h @ blocks["W4"] + blocks["b4"]

    Lc = net(feat)[:, :n_spec]
    w = torch.tensor(weight, dtype=torch.float64)
    ce = torch.nn.functional.cross_entropy(Lc, torch.tensor(label), reduction="none")
    R = net(fv)[:, n_spec:].reshape(5, 8, 5)
    mu = R[..., :3] / R[..., :3].norm(dim=-1, keepdim=True)
    kap = torch.exp(torch.clamp(R[..., 3], mlp.LOG_KAPPA_MIN, mlp.LOG_KAPPA_MAX))
    logpi = torch.log_softmax(R[..., 4], dim=-1)
    wt = torch.tensor(dv, dtype=torch.float64)[:, None, :]
    logv = torch.log(kap) - np.log(2 * np.pi) - torch.log(-torch.expm1(-2 * kap)) - kap * (1 - (mu * wt).sum(-1))
    nll = -torch.logsumexp(logpi + logv, dim=-1)
    wvt = torch.tensor(wv, dtype=torch.float64)
    ((w * ce).sum() / w.sum() + (wvt * nll).sum() / wvt.sum()).backward()
    ref = np.concatenate([blocks[name].grad.numpy().ravel() for name, _ in mlp.layout(n_out)])
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-13)
