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


@pytest.fixture(scope="module")
def scene():
    from paper_2503_23412_amd import pt
    s = pt.Scene(scenes.cornell_glass(64, 64), max_light_paths=4096)
    s.build_subspaces(n_eye=16, n_spec=N_SPEC)
    yield s
    s.release()


def _params(rng, n_out=N_SPEC):
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
    assert scene.mlp_param_count() == p.size == mlp.count(N_SPEC)
    scene.mlp_set_params(p)
    np.testing.assert_array_equal(scene.mlp_get_params(), p)
    feat = rng.uniform(0.0, 1.0, size=(n, 9))
    feat[:, 3:9] = rng.normal(size=(n, 6))
    feat[:, 3:6] /= np.linalg.norm(feat[:, 3:6], axis=1, keepdims=True)
    feat[:, 6:9] /= np.linalg.norm(feat[:, 6:9], axis=1, keepdims=True)
    fd = torch.tensor(feat, dtype=torch.float32, device="cuda")
    out = torch.full((n, N_SPEC), float("nan"), dtype=torch.float32, device="cuda")
    scene.mlp_forward(fd, out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    ref, _ = mlp.forward(p.astype(np.float64), N_SPEC, feat.astype(np.float32).astype(np.float64))
    print(f"forward n={n}: rel-L2 {_rel(got, ref):.2e}", flush=True)
    assert np.all(np.isfinite(got))
    assert _rel(got, ref) < 2e-2
    assert _cos(got.ravel(), ref.ravel()) > 0.999


@pytest.mark.parametrize("n", [300, 5003])
def test_gradient_and_adam_match_oracle(scene, n):
    rng = np.random.default_rng(20 + n)
    p = _params(rng)
    scene.mlp_set_params(p)
    feat = rng.uniform(0.0, 1.0, size=(n, 9))
    label = rng.integers(0, N_SPEC, size=n)
    weight = rng.exponential(1.0, size=n)
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")  # noqa: E731
    lr = 1e-3
    g = scene.mlp_train_step(dev(feat, torch.float32), dev(label, torch.int32), dev(weight, torch.float32), lr,
                             want_grad=True)
    ref = mlp.grad(p.astype(np.float64), N_SPEC, feat.astype(np.float32).astype(np.float64), label,
                   weight.astype(np.float32).astype(np.float64))
    f64, w64 = feat.astype(np.float32).astype(np.float64), weight.astype(np.float32).astype(np.float64)
    scale = mlp.grad_scale(p.astype(np.float64), N_SPEC, f64, label, w64)
    ref16 = mlp.grad(p.astype(np.float64), N_SPEC, f64, label, w64, bf16=True)
    off, bad = 0, []
    for name, shape in mlp.layout(N_SPEC):
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
