"""Benchmark of the proxy-sampling BDPT hot path on one MI355X.

A step is one rendering iteration (1 sample per pixel through every strategy: light pass,
connection pool, candidates, reciprocal estimates, eye pass with emission hits, next-event
estimation and probabilistic connections, light tracing, proxy connections, accumulation) of
the projector caustic workload (512 x 512, depth 12, 500,000 light sub-paths per iteration,
20,000 expected candidates). Prints one JSON line.

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
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (256 CUs, 2.4 GHz, packed FMA)
# algorithmic FP32 operations per unit of traversal work (an FMA counts two):
# a 4-wide node visit is four slab tests, each 6 FMAs for the six plane distances, 6 min/max
# for the entry distance, 6 for the exit distance and 1 compare (25 per child);
# a triangle test is Moller-Trumbore: two cross products (18), four dot products (20), one
# reciprocal, the translation (3), three scalings by the reciprocal (3), 7 for the determinant,
# barycentric and distance bounds (52)
FLOP_NODE = 100
FLOP_TRI = 52
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_k_recip_projector_512.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_23412_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(csrc, "*.hip")),
                    key=os.path.basename):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per k_recip launch from the committed hardware-counter summary, or None when
    the kernel sources no longer hash to the value the counters were taken with."""
    try:
        txt = open(PMC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        line = line.strip()
        for key in ("traffic_bytes_per_launch:", "source_sha256:"):
            if line.startswith(key):
                vals[key] = line[len(key):].strip()
    if vals.get("source_sha256:") != kernel_source_hash() or "traffic_bytes_per_launch:" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch:"])


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
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB: the reference kernel of "
                         "known size for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library has no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2503_23412_amd import pt
    from synth import scenes

    cfg = scenes.config(args.config)
    sc = cfg["scene"]
    W, H = sc["width"], sc["height"]
    # the plain method: every strategy of the iteration, no learned selection
    flags = (pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_MIS | pt.PT_FLAG_GAMMA | pt.PT_FLAG_TILES |
             pt.PT_FLAG_SPC | pt.PT_FLAG_LT)
    params = dict(max_depth=cfg["max_depth"], n_light=cfg["n_light"], cand_cap=cfg["cand_cap"], seed=cfg["seed"])
    torch.cuda.set_device(0)
    log(f"upload: {sc['tri'].shape[0]} tris, {W}x{H}")
    S = pt.Scene(sc, max_light_paths=cfg["n_light"])
    S.build_subspaces(n_eye=cfg["n_subspaces"], n_spec=cfg["n_spec"])
    acc = torch.zeros(W * H * 3, device="cuda")
    acc2 = torch.zeros_like(acc)
    # warmup: the reciprocal-chain schedule autotuner (its timed iterations render like any other),
    # then plain iterations
    tune = S.autotune(acc, acc2, iteration=0, flags=flags, **params)
    log(f"autotune: {tune}")
    k0 = tune["iterations_rendered"]
    for k in range(args.warmup):
        S.render_iteration(acc, acc2, iteration=k0 + k, flags=flags, **params)
    torch.cuda.synchronize()
    log("warmup done")
    first = k0 + args.warmup
    t0 = time.perf_counter()
    for k in range(args.steps):
        S.render_iteration(acc, acc2, iteration=first + k, flags=flags, **params)
        if k % 16 == 15:
            log(f"step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt:.3f} s")
    # one iteration with traversal counters, then timed ones (HIP events recorded on the stream the
    # kernels are launched on, inside the library)
    it = first + args.steps
    stc = S.render_iteration(acc, acc2, stats=True, iteration=it, flags=flags | pt.PT_FLAG_COUNT, **params)
    tim = [S.render_iteration(acc, acc2, stats=True, iteration=it + 1 + j, flags=flags | pt.PT_FLAG_TIMING, **params)
           for j in range(4)]
    ms_ext = float(np.mean([t["ms_extend"] for t in tim]))
    ms_a = float(np.mean([t["ms_recip_stage_a"] for t in tim]))
    ms_rec = float(np.mean([t["ms_recip"] for t in tim]))
    st = tim[-1]
    rays = st["rays_extend_eye"] + st["rays_extend_light"] + st["rays_shadow"] + st["rays_proxy"] + st["rays_recip"]
    n_launch = params["max_depth"]
    # algorithmic work of the two traversal kernels: FP32 operations of every node visit and
    # triangle test (FLOP_NODE, FLOP_TRI); the bytes of every visited 128-byte node and tested
    # 48-byte triangle record are reported beside them (those reads are served from the caches:
    # the measured HBM traffic is the `traffic` field)
    ext_flops = stc["node_visits"] * FLOP_NODE + stc["tri_tests"] * FLOP_TRI
    a_flops = stc["node_visits_stage_a"] * FLOP_NODE + stc["tri_tests_stage_a"] * FLOP_TRI
    ext_bytes = stc["node_visits"] * 128 + stc["tri_tests"] * 48
    a_bytes = stc["node_visits_stage_a"] * 128 + stc["tri_tests_stage_a"] * 48
    cands = [
        {"kernel": "k_extend (eye closest hit)", "ms_per_step": ms_ext, "launches": n_launch, "flops": ext_flops,
         "bytes": ext_bytes, "traffic": None},
        {"kernel": "k_recip (reciprocal chains, stage A)", "ms_per_step": ms_a, "launches": 1, "flops": a_flops,
         "bytes": a_bytes, "traffic": recorded_traffic() if args.config == 1 else None},
    ]
    dom = max(cands, key=lambda c: c["ms_per_step"])
    per_launch_s = dom["ms_per_step"] / dom["launches"] * 1e-3
    achieved = dom["flops"] / dom["launches"] / per_launch_s / 1e12 if per_launch_s > 0 else 0.0
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
        "config": {"workload": f"projector caustic (config 1): {W}x{H}, {sc['tri'].shape[0]:,} tris, depth "
                               f"{params['max_depth']}, M={params['n_light']:,} light sub-paths, "
                               f"{params['cand_cap']:,} expected candidates; plain method (PT, NEE, probabilistic "
                               f"connections, light tracing, proxy connections with variance-aware MIS, Gamma, tiles)",
                   "spp_per_step": 1, "max_depth": params["max_depth"], "n_light": params["n_light"]},
        "mrays_per_s": rays * args.steps / dt / 1e6,
        "rays_per_step": rays,
        "ray_breakdown": {k: st[k] for k in ("rays_extend_eye", "rays_extend_light", "rays_shadow", "rays_proxy",
                                             "rays_recip")},
        "proxy": {k: st[k] for k in ("n_cand", "n_kept", "n_recip_samples", "n_recip_truncated",
                                     "n_proxy_attempts", "n_proxy_valid", "n_pool", "n_connections", "n_lt_splats",
                                     "n_nan", "chain_len_max")},
        "ms_breakdown": {"eye_extension": ms_ext, "reciprocal_block": ms_rec, "reciprocal_stage_a": ms_a},
        "schedule": {"stage_a_budget": tune["stage_a_budget"], "round_grid": tune["round_grid"],
                     "autotune_iterations": k0, "ms_tuned": tune["ms_best"], "ms_default": tune["ms_previous"]},
        "roofline": {"kernel": dom["kernel"], "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": dom["traffic"],
                     "flops_per_launch": dom["flops"] / dom["launches"],
                     "ms_per_launch": dom["ms_per_step"] / dom["launches"],
                     "node_tri_bytes_per_launch": dom["bytes"] / dom["launches"],
                     "node_tri_GBs": dom["bytes"] / dom["launches"] / per_launch_s / 1e9 if per_launch_s > 0 else 0.0,
                     "hbm_frac_of_traffic": (dom["traffic"] / per_launch_s / 1e9 / HBM_PEAK_GBS
                                             if dom["traffic"] and per_launch_s > 0 else None)},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, params)
    S.release()
    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"reference copy: {args.copy_mib} MiB read, {args.copy_mib} MiB written")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
