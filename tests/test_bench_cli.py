"""Host logic of the benchmark scripts: one GPU only, and the photon-plane CPU baseline leg."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    for script in ("bench.py", "bench_planes.py"):
        p = subprocess.run([sys.executable, os.path.join(ROOT, script), "--gpus", "2"], capture_output=True,
                           text=True, timeout=120)
        assert p.returncode == 2, (script, p.stderr)
        assert "one GPU" in p.stderr, (script, p.stderr)


def test_planes_cpu_baseline_is_bounded(oracle):
    import bench_planes
    from synth import scenes
    out = bench_planes.cpu_baseline(scenes.planes_scene(8, 8), 16, budget_s=0.2)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "ray-plane tests/s"
    assert out["value"] > 0 and "8x8" in out["sample"]
