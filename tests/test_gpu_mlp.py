"""GPU tests of the learned subspace selection's network (BF16 MFMA, FP32 accumulation) against
the FP64 oracle of oracle/mlp.py, through the C ABI.

Tolerances: operands are rounded to BF16 (unit roundoff 2^-8) at every layer's input and
weights, so each layer's products carry a relative error of about 2^-8 / sqrt(2) per factor
pair, accumulating to a few 1e-3 over four layers on random data; the tests allow 2e-2 (rel-L2)
with cosine similarity above 0.999, which a transposed operand or a wrong MFMA lane layout
(errors of order 1) cannot meet."""
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
    off = 0
    for name, shape in mlp.layout(N_SPEC):
        k = int(np.prod(shape))
        a, b = g[off:off + k].astype(np.float64), ref[off:off + k]
        print(f"grad {name}: rel-L2 {_rel(a, b):.2e} cos {_cos(a, b):.6f}", flush=True)
        assert np.all(np.isfinite(a)), name
        assert _rel(a, b) < 5e-2 and _cos(a, b) > 0.999, name
        if name == "W1":
            assert np.all(a.reshape(shape)[225:] == 0.0)
        off += k
    # one Adam step from zero moments: w - lr g / (|g| + eps), with the GPU's own gradient
    p1 = scene.mlp_get_params()
    g32 = g.astype(np.float32)
    expect = p - np.float32(lr) * g32 / (np.abs(g32) + np.float32(1e-8))
    np.testing.assert_allclose(p1, expect, rtol=1e-6, atol=1e-8)
