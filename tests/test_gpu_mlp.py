"""GPU tests of the learned subspace selection's network (BF16 MFMA, FP32 accumulation) against
the FP64 oracle of oracle/mlp.py, through the C ABI.

Tolerances: operands are rounded to BF16 (unit roundoff u = 2^-8) at every layer's input and
weights, so each layer's products carry a relative error of about u / sqrt(2) per factor pair,
accumulating to a few 1e-3 over four layers on random data; the forward test allows 2e-2
(rel-L2) with cosine similarity above 0.999.

Gradients: a gradient block is a sum over samples whose terms cancel, and BF16 storage of the
weights, inputs and activations moves it by several per cent of sqrt(sum_i ||term_i||^2) (the
oracle's grad_scale) on random networks. The oracle's bf16 mode rounds at the same storage
points, so the GPU gradient is compared with it at 1 % of that scale (what remains is FP32
accumulation order and the rare ReLU whose sign the order flips), and with the FP64 gradient
within 1.5 times the bf16 model's own distance from it plus 1 % of the scale. A transposed
operand, a wrong MFMA lane layout or a lost split-K chunk gives errors of order 10-100 %."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp  # noqa: E402
from synth import scenes  # noqa: E402

pytestmark = pytest.mark.gpu
N_SPEC = 24
N_OUT = N_SPEC + mlp.VMF_OUT   # logits, then the direction head's mixture


@pytest.fixture(scope="module")
def scene():
    from paper_2503_23412_amd import pt
    s = pt.Scene(scenes.cornell_glass(64, 64), max_light_paths=4096)
    s.build_subspaces(n_eye=16, n_spec=N_SPEC)
    yield s
    s.release()


def _params(rng, n_out=N_OUT):
    blocks = {}
    for name, shape in mlp.layout(n_out):
        if len(shape) == 2:
            fan = 225 if name == "W1" else shape[0]
            blocks[name] = rng.uniform(-1, 1, size=shape) * np.sqrt(6.0 / fan)
        else:
            blocks[name] = rng.normal(0.0, 0.1, size=shape)
    blocks["W1"][225:] = 0.0
    return mlp.pack(blocks, n_out).astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _cos(a, b):
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [1, 16, 1037])
def test_forward_matches_oracle(scene, n):
    rng = np.random.default_rng(10 + n)
    p = _params(rng)
    assert scene.mlp_param_count() == p.size == mlp.count(N_OUT)
    scene.mlp_set_params(p)
    np.testing.assert_array_equal(scene.mlp_get_params(), p)
    feat = rng.uniform(0.0, 1.0, size=(n, 9))
    feat[:, 3:9] = rng.normal(size=(n, 6))
    feat[:, 3:6] /= np.linalg.norm(feat[:, 3:6], axis=1, keepdims=True)
    feat[:, 6:9] /= np.linalg.norm(feat[:, 6:9], axis=1, keepdims=True)
    fd = torch.tensor(feat, dtype=torch.float32, device="cuda")
    out = torch.full((n, N_OUT), float("nan"), dtype=torch.float32, device="cuda")
    scene.mlp_forward(fd, out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    ref, _ = mlp.forward(p.astype(np.float64), N_OUT, feat.astype(np.float32).astype(np.float64))
    print(f"forward n={n}: rel-L2 {_rel(got, ref):.2e}", flush=True)
    assert np.all(np.isfinite(got))
    assert _rel(got, ref) < 2e-2
    assert _cos(got.ravel(), ref.ravel()) > 0.999


def _unit(rng, n):
    w = rng.normal(size=(n, 3))
    return w / np.linalg.norm(w, axis=1, keepdims=True)


@pytest.mark.parametrize("n,n_dir", [(300, 0), (5003, 0), (0, 2000), (5003, 4001)])
def test_gradient_and_adam_match_oracle(scene, n, n_dir):
    """Subspace rows (cross entropy of the logits) and direction rows (negative log-likelihood under
    the vMF mixture) in one training batch, against the oracle's gradient of the same loss."""
    rng = np.random.default_rng(20 + n + 7 * n_dir)
    p = _params(rng)
    scene.mlp_set_params(p)
    feat = rng.uniform(0.0, 1.0, size=(n, 9))
    label = rng.integers(0, N_SPEC, size=n)
    weight = rng.exponential(1.0, size=n)
    fv = rng.uniform(0.0, 1.0, size=(n_dir, 9))
    dv = _unit(rng, n_dir)
    wv = rng.exponential(1.0, size=n_dir)
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda") if len(a) else None  # noqa: E731
    lr = 1e-3
    g = scene.mlp_train_step(dev(feat, torch.float32), dev(label, torch.int32), dev(weight, torch.float32), lr,
                             feat_dir=dev(fv, torch.float32), dirs=dev(dv, torch.float32),
                             weight_dir=dev(wv, torch.float32), want_grad=True)
    c = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    f64, w64 = c(feat), c(weight)
    vmf = (c(fv), c(dv), c(wv)) if n_dir else None
    fe = f64 if n else None
    kw = dict(n_spec=N_SPEC, vmf=vmf)
    ref = mlp.grad(p.astype(np.float64), N_OUT, fe, label, w64, **kw)
    scale = mlp.grad_scale(p.astype(np.float64), N_OUT, fe, label, w64, **kw)
    ref16 = mlp.grad(p.astype(np.float64), N_OUT, fe, label, w64, bf16=True, **kw)
    off, bad = 0, []
    for name, shape in mlp.layout(N_OUT):
        k = int(np.prod(shape))
        a, b, b16 = g[off:off + k].astype(np.float64), ref[off:off + k], ref16[off:off + k]
        e64, e16, model = (float(np.linalg.norm(a - b)), float(np.linalg.norm(a - b16)),
                           float(np.linalg.norm(b16 - b)))
        print(f"grad {name}: vs fp64 {e64 / scale[name]:.2e}, vs bf16 model {e16 / scale[name]:.2e}, "
              f"model vs fp64 {model / scale[name]:.2e} (of scale); cos vs fp64 {_cos(a, b):.5f}", flush=True)
        if not (np.all(np.isfinite(a)) and e16 <= 1e-2 * scale[name] and e64 <= 1.5 * model + 1e-2 * scale[name]):
            bad.append(name)
        if name == "W1":
            assert np.all(a.reshape(shape)[225:] == 0.0)
        off += k
    assert not bad, bad
    # one Adam step from zero moments: w - lr g / (|g| + eps), with the GPU's own gradient
    p1 = scene.mlp_get_params()
    g32 = g.astype(np.float32)
    expect = p - np.float32(lr) * g32 / (np.abs(g32) + np.float32(1e-8))
    np.testing.assert_allclose(p1, expect, rtol=1e-6, atol=1e-8)


def test_vmf_sampler_matches_its_density():
    """The retrace's vMF mixture sampler on the device: its reported density equals the oracle's
    mixture density at the drawn direction; a single lobe's draws follow the vMF law of the cosine to
    the mean (Kolmogorov-Smirnov against (1 - exp(-kappa h)) / (1 - exp(-2 kappa)), h = 1 - mu.w);
    the lobes of a mixture are drawn with their weights."""
    from paper_2503_23412_amd import pt
    from scipy import stats
    rng = np.random.default_rng(40)
    n = 1 << 18
    raw = np.zeros((n, 40), np.float32)
    for k in range(8):
        raw[:, 5 * k:5 * k + 3] = _unit(rng, n) * rng.uniform(0.5, 3.0, size=(n, 1))
        raw[:, 5 * k + 3] = rng.uniform(-2.5, 9.5, size=n)
        raw[:, 5 * k + 4] = rng.normal(size=n)
    rd = torch.tensor(raw, device="cuda")
    dirs = torch.empty((n, 3), device="cuda")
    pdf = torch.empty(n, device="cuda")
    pt.vmf_sample(rd, 11, dirs, pdf)
    torch.cuda.synchronize()
    w, pg = dirs.double().cpu().numpy(), pdf.double().cpu().numpy()
    np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-6)
    po = mlp.vmf_pdf(raw.astype(np.float64), w)
    rel = np.abs(pg - po) / po
    print(f"vmf density: max rel {rel.max():.2e} median {np.median(rel):.2e}", flush=True)
    assert np.quantile(rel, 0.999) < 1e-4 and rel.max() < 1e-3
    for kappa in (0.2, 5.0, 3000.0):
        mu = np.array([0.0, 0.6, 0.8])
        raw1 = np.zeros((n, 40), np.float32)
        raw1[:, 0:3] = mu * 2.0
        raw1[:, 3] = np.log(kappa)
        raw1[:, 4] = 60.0
        pt.vmf_sample(torch.tensor(raw1, device="cuda"), 12, dirs, pdf)
        torch.cuda.synchronize()
        w = dirs.double().cpu().numpy()
        h = np.maximum(1.0 - w @ mu, 0.0)
        cdf = lambda x: -np.expm1(-kappa * x) / -np.expm1(-2 * kappa)  # noqa: E731
        pv = stats.kstest(h, cdf).pvalue
        print(f"vmf lobe kappa {kappa}: KS p {pv:.3g}", flush=True)
        assert pv > 1e-4
    means = _unit(np.random.default_rng(41), 8)
    logits = np.array([0.0, 1.0, -1.0, 0.5, 2.0, -2.0, 0.0, 0.3], np.float32)
    raw2 = np.zeros((n, 40), np.float32)
    for k in range(8):
        raw2[:, 5 * k:5 * k + 3] = means[k]
        raw2[:, 5 * k + 3] = np.log(5000.0)
        raw2[:, 5 * k + 4] = logits[k]
    pt.vmf_sample(torch.tensor(raw2, device="cuda"), 13, dirs, pdf)
    torch.cuda.synchronize()
    k = (dirs.double().cpu().numpy() @ means.T).argmax(1)
    pi = np.exp(logits.astype(np.float64)) / np.exp(logits.astype(np.float64)).sum()
    assert stats.chisquare(np.bincount(k, minlength=8), pi * n).pvalue > 1e-4
