#!/usr/bin/env python3
"""Batched serving benchmark (config 4): 16 seeded scenes of uneven size (10^3 .. 2 10^6 triangles,
256^2 .. 1920x1080 pixels, mirror/glass/glossy materials, depth 16, 2,000 eye and specular
subspaces each) rendered together, one HIP graph holding one iteration of every scene on its own
branch (pt_render_scenes), with the first stage of every scene's reciprocal chains in one
persistent launch over a shared work queue, replayed per iteration.

Reports one JSON line: aggregate full-path samples/s over all scenes (pixels x iterations / wall
time), and the per-scene iteration latency from the device's wall clock (first to last kernel of
each scene's iteration, pt_iteration_times): p50 and p99 over every scene and timed iteration.

  python bench_serving.py [--iters 16] [--warmup 2] [--plain] [--res-cap R] [--max-tris T]

--plain switches the learned proposal off (the default renders every scene with it); --res-cap and
--max-tris shrink the batch for quick runs.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain", action="store_true")
    ap.add_argument("--res-cap", type=int, default=None)
    ap.add_argument("--max-tris", type=int, default=2_000_000)
    ap.add_argument("--subspaces", type=int, default=2000)
    a = ap.parse_args()
    import numpy as np
    import torch
    from paper_2503_23412_amd import pt
    from synth import scenes

    t0 = time.time()
    batch = scenes.serving_batch(max_tris=a.max_tris, res_cap=a.res_cap)
    log(f"generated {len(batch)} scenes in {time.time() - t0:.1f} s")
    flags = (pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_MIS | pt.PT_FLAG_GAMMA | pt.PT_FLAG_TILES |
             pt.PT_FLAG_SPC | pt.PT_FLAG_LT)
    if not a.plain:
        flags |= pt.PT_FLAG_MLP | pt.PT_FLAG_MLP_DIR
    S, acc, prm, pix, tris = [], [], [], [], []
    for i, (sc, spec) in enumerate(batch):
        W, H = sc["width"], sc["height"]
        # light sub-paths and candidates in the proportions of config 2 (a quarter of the pixels;
        # 1 / 25 of the light paths)
        M = max(4096, (W * H) // 4)
        s = pt.Scene(sc, max_light_paths=M)
        ns = min(a.subspaces, 4096)
        s.build_subspaces(n_eye=ns, n_spec=ns)
        S.append(s)
        acc.append(torch.zeros(W * H * 3, device="cuda"))
        prm.append(dict(max_depth=16, n_light=M, cand_cap=max(64, M // 25), seed=i, flags=flags, train_iters=1 << 30,
                        mlp_mix=0.9, mlp_lr=1e-3))
        pix.append(W * H)
        tris.append(int(sc["tri"].shape[0]))
        log(f"scene {i}: {tris[-1]} tris, {W}x{H}, M={M}")
    torch.cuda.synchronize()
    it = 0
    for _ in range(a.warmup):
        pt.render_scenes(S, acc, None, 1, [dict(q, iteration=it) for q in prm])
        it += 1
    torch.cuda.synchronize()
    log("warmup done")
    first = it
    t0 = time.perf_counter()
    for k in range(a.iters):
        pt.render_scenes(S, acc, None, 1, [dict(q, iteration=it) for q in prm])
        it += 1
        if k % 4 == 3:
            torch.cuda.synchronize()
            log(f"iteration {k + 1}/{a.iters}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat = np.concatenate([s.iteration_times(first, a.iters) for s in S])
    per_scene = [float(np.median(s.iteration_times(first, a.iters))) for s in S]
    tot = [s.totals() for s in S]
    for s in S:
        s.release()
    lat = lat[lat >= 0]
    out = {
        "metric": "aggregate full-path samples/s (16-scene serving batch)",
        "value": sum(pix) * a.iters / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "iters": a.iters,
        "ms_per_batch_iteration": dt / a.iters * 1e3,
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
        "latency_ms_median_per_scene": per_scene,
        "scenes": [{"tris": t, "pixels": p} for t, p in zip(tris, pix)],
        "learned": not a.plain,
        "n_nan": sum(t["n_nan"] for t in tot),
        "n_recip_truncated": sum(t["n_recip_truncated"] for t in tot),
        "dtype": "f32",
        "data": "synthetic",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
