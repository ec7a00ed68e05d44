"""Benchmark of the proxy-sampling BDPT hot path on one MI355X.

A step is one rendering iteration (1 sample per pixel through every strategy: light pass,
candidates, reciprocal estimates, eye pass with next-event estimation and proxy connections,
accumulation) of the projector caustic workload (512 x 512, depth 12, 500,000 light
sub-paths per iteration, 20,000 expected candidates). Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(sc, params, budget_s=20.0):
    """The FP64 oracle (O2, proxy-sampling BDPT) on a bounded sample of the same workload:
    the projector scene at the same depth and light-path budget, on a pixel window of the
    full-resolution camera (the oracle renders rows independently), timed on the host."""
    import numpy as np
    from oracle import oracle as O
    from synth import scenes
    threads = os.cpu_count() or 1
    # a 64 x 64 crop of the 512 x 512 image keeps the camera rays of the full render
    small = scenes.projector(64, 64)
    small["cam"] = sc["cam"]
    S = O.Scene(small)
    t0 = time.time()
    n = 0
    M = max(1000, params["n_light"] // 64)
    while time.time() - t0 < budget_s and n < 64:
        S.render(method=1, n_iter=1, first_iter=n, max_depth=params["max_depth"], n_light=M,
                 cand_cap=max(40, params["cand_cap"] // 64), threads=threads, seed=1)
        n += 1
    dt = time.time() - t0
    return {"value": 64 * 64 * n / dt, "unit": "full-path samples/s", "cores": threads, "kind": "oracle",
            "sample": f"O2 on the projector scene, {n} iterations of a 64x64 pixel window with M={M} light "
                      f"sub-paths (1/64 of the pixels and light paths per iteration)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--config", type=int, default=1)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build has no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2503_23412_amd import pt
    from synth import scenes

    cfg = scenes.config(args.config)
    sc = cfg["scene"]
    W, H = sc["width"], sc["height"]
    params = dict(max_depth=cfg["max_depth"], n_light=cfg["n_light"], cand_cap=cfg["cand_cap"], seed=cfg["seed"])
    torch.cuda.set_device(0)
    log(f"upload: {sc['tri'].shape[0]} tris, {W}x{H}")
    S = pt.Scene(sc, max_light_paths=cfg["n_light"])
    S.build_subspaces(n_eye=cfg["n_subspaces"], n_spec=cfg["n_spec"])
    acc = torch.zeros(W * H * 3, device="cuda")
    acc2 = torch.zeros_like(acc)
    stream = torch.cuda.current_stream()
    for k in range(args.warmup):
        S.render_iteration(acc, acc2, iteration=k, **params)
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    for k in range(args.steps):
        S.render_iteration(acc, acc2, iteration=args.warmup + k, **params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt:.3f} s")
    # one iteration with counters for ray totals and traversal work, one with extension timing
    it = args.warmup + args.steps
    st = S.render_iteration(acc, acc2, stats=True, iteration=it, **params)
    stc = S.render_iteration(acc, acc2, stats=True, iteration=it + 1,
                             flags=pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_COUNT, **params)
    times = []
    for j in range(4):
        stt = S.render_iteration(acc, acc2, stats=True, iteration=it + 2 + j,
                                 flags=pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_TIMING, **params)
        times.append(stt["ms_extend"])
    ms_ext = float(np.mean(times))
    rays = st["rays_extend_eye"] + st["rays_extend_light"] + st["rays_shadow"] + st["rays_proxy"] + st["rays_recip"]
    # algorithmic bytes of the eye extension launches: every visited 128-byte node, every tested
    # 48-byte triangle, the ray (32 B) and queue index (4 B) read, the hit (16 B) written
    eye_rays = stc["rays_extend_eye"]
    traffic_alg = stc["node_visits"] * 128 + stc["tri_tests"] * 48 + eye_rays * (32 + 4 + 16)
    n_launch = params["max_depth"]
    achieved = (traffic_alg / n_launch) / (ms_ext / n_launch * 1e-3) / 1e9
    value = W * H * args.steps / dt
    out = {
        "metric": "full-path samples/s",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "projector caustic (config 1): 512x512, 8,206 tris, depth 12, "
                               "M=500,000 light sub-paths, 20,000 expected candidates, plain method",
                   "spp_per_step": 1, "max_depth": params["max_depth"], "n_light": params["n_light"]},
        "mrays_per_s": rays * args.steps / dt / 1e6,
        "rays_per_step": rays,
        "ray_breakdown": {k: st[k] for k in ("rays_extend_eye", "rays_extend_light", "rays_shadow", "rays_proxy",
                                             "rays_recip")},
        "proxy": {k: st[k] for k in ("n_cand", "n_kept", "n_recip_samples", "n_recip_truncated",
                                     "n_proxy_attempts", "n_proxy_valid", "n_nan")},
        "roofline": {"kernel": "k_extend (eye closest hit)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_step": traffic_alg, "ms_per_step": ms_ext,
                     "nodes_per_ray": stc["node_visits"] / max(eye_rays, 1),
                     "tris_per_ray": stc["tri_tests"] / max(eye_rays, 1)},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, params)
    S.release()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
