"""Benchmark of the proxy-sampling BDPT hot path on one MI355X.

A step is one rendering iteration (1 sample per pixel through every strategy: light pass,
connection pool, candidates, reciprocal estimates, eye pass with emission hits, next-event
estimation and probabilistic connections, light tracing, proxy connections, accumulation).
Default workload: the glossy/specular procedural scene (config 2: 1024 x 1024, 198,740 tris,
depth 12, 262,144 light sub-paths per iteration, 10,486 expected candidates, 1,000 / 100
subspaces). --config 1 times the projector caustic scene (512 x 512). Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--no-cpu]
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
NODE_BYTES = 128           # one 4-wide BVH node (one 128-byte line)
TRI_BYTES = 48             # one intersection triangle record
# algorithmic FP32 operations per unit of traversal work (an FMA counts two):
# a 4-wide node visit is four slab tests, each 6 FMAs for the six plane distances, 6 min/max
# for the entry distance, 6 for the exit distance and 1 compare (25 per child);
# a triangle test is Moller-Trumbore: two cross products (18), four dot products (20), one
# reciprocal, the translation (3), three scalings by the reciprocal (3), 7 for the determinant,
# barycentric and distance bounds (52)
FLOP_NODE = 100
FLOP_TRI = 52
PMC_FILES = {2: os.path.join(ROOT, "profiles", "pmc_glossy_1024.txt")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the headers that hold the device code of the render iteration's kernels (the photon-plane
# kernels and the host file are not among them)
KERNEL_SOURCES = ("pt_device.h", "pt_kernels.h", "pt_layout.h", "pt_mlp.h", "pt_subspace.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_23412_amd", "csrc")
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(config, kernel):
    """HBM bytes per launch of `kernel` from the committed hardware-counter summary of this
    workload, or None when there is none or the kernel sources no longer hash to the value the
    counters were taken with. Lines: `source_sha256: <hex>` and `traffic_bytes_per_launch <kernel>: <bytes>`."""
    try:
        txt = open(PMC_FILES[config]).read()
    except (OSError, KeyError):
        return None
    sha, val = None, None
    for line in txt.splitlines():
        line = line.strip()
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith(f"traffic_bytes_per_launch {kernel}:"):
            val = float(line.split(":", 1)[1])
    if sha != kernel_source_hash():
        return None
    return val


def cpu_baseline(config, sc, params, budget_s=20.0):
    """The FP64 oracle (O2, proxy-sampling BDPT) on a bounded sample of the same workload: the
    same scene, camera view and depth rendered at 64 x 64 pixels (each pixel sample traces the
    same kind of paths as at full resolution) with 1/64 of the light sub-paths and candidates per
    iteration, timed on the host's cores."""
    from oracle import oracle as O
    from synth import scenes
    threads = os.cpu_count() or 1
    small = scenes.config(config)["scene"]
    small["width"], small["height"] = 64, 64
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
            "sample": f"O2 on the same scene and view at 64x64 pixels (full image {sc['width']}x{sc['height']}), "
                      f"{n} iterations with M={M} light sub-paths (1/64 of the light paths per iteration)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--tris", type=int, default=0,
                    help="configs 2 and 3: triangle budget of the glossy scene instead of 200,000 (8,000,000 gives "
                         "4.2 M triangles, 285 MB of nodes and triangle records, beyond the 256 MB Infinity Cache)")
    ap.add_argument("--bvh-width", type=int, default=0, choices=(0, 4, 8),
                    help="BVH width of the walks: 4, 8, or 0 to upload both trees and let the autotuner pick")
    ap.add_argument("--pilot", type=int, default=None,
                    help="pilot samples per candidate (default 16; 0 takes B and beta from the (class, u, S, C) "
                         "bucket statistics of earlier iterations alone, Section 5.5)")
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
    if args.tris and args.config in (2, 3):
        cfg["scene"] = scenes.glossy_procedural(1024, 1024, target_tris=args.tris)
    sc = cfg["scene"]
    W, H = sc["width"], sc["height"]
    # the plain method: every strategy of the iteration; config 3 adds the learned proposal (both
    # heads, trained online in every iteration)
    flags = (pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_MIS | pt.PT_FLAG_GAMMA | pt.PT_FLAG_TILES |
             pt.PT_FLAG_SPC | pt.PT_FLAG_LT)
    params = dict(max_depth=cfg["max_depth"], n_light=cfg["n_light"], cand_cap=cfg["cand_cap"], seed=cfg["seed"])
    if args.pilot is not None:
        params["pilot"] = args.pilot
    if cfg.get("mlp"):
        flags |= pt.PT_FLAG_MLP | pt.PT_FLAG_MLP_DIR
        params.update(mlp_mix=cfg["mlp_mix"], mlp_lr=cfg["mlp_lr"], train_iters=cfg["train_iters"])
    torch.cuda.set_device(0)
    log(f"upload: {sc['tri'].shape[0]} tris, {W}x{H}")
    S = pt.Scene(sc, max_light_paths=cfg["n_light"], bvh_width=args.bvh_width)
    S.build_subspaces(n_eye=cfg["n_subspaces"], n_spec=cfg["n_spec"])
    acc = torch.zeros(W * H * 3, device="cuda")
    acc2 = torch.zeros_like(acc)
    # warmup: 48 iterations, past the 40 in which Gamma, Q and the tile shares learn (their
    # statistics, and with them the chains' cost, settle there, and a tuner timing its choices
    # one after another while the cost still falls would favour whichever it times last); then the
    # schedule autotuner (its timed iterations render like any other); then plain iterations
    settle = 48
    for k in range(settle):
        S.render_iteration(acc, acc2, iteration=k, flags=flags, **params)
    tune = S.autotune(acc, acc2, iteration=settle, flags=flags, **params)
    log(f"autotune: {tune}")
    k0 = settle + tune["iterations_rendered"]
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
    # Roofline of the dominant traversal kernel in the units of the traversal roof (HBM bytes):
    # `achieved` = the algorithmic bytes of one launch (every visited 128-byte node and every
    # tested 48-byte triangle record, from the traversal counters of a counting iteration) over
    # the launch's average duration (HIP events recorded on the launch stream inside the library);
    # `traffic` = the bytes the hardware counters saw move between L2 and memory for one launch,
    # when a summary of the current sources exists. The FP32 operations of the same work are
    # reported beside them (FLOP_NODE, FLOP_TRI) against the vector FP32 peak.
    ext_flops = stc["node_visits"] * FLOP_NODE + stc["tri_tests"] * FLOP_TRI
    a_flops = stc["node_visits_stage_a"] * FLOP_NODE + stc["tri_tests_stage_a"] * FLOP_TRI
    ext_bytes = stc["node_visits"] * NODE_BYTES + stc["tri_tests"] * TRI_BYTES
    a_bytes = stc["node_visits_stage_a"] * NODE_BYTES + stc["tri_tests_stage_a"] * TRI_BYTES
    cands = [
        {"kernel": "k_extend", "what": "eye closest hit", "ms_per_step": ms_ext, "launches": n_launch,
         "flops": ext_flops, "bytes": ext_bytes},
        {"kernel": "k_recip", "what": "reciprocal chains, stage A", "ms_per_step": ms_a, "launches": 1,
         "flops": a_flops, "bytes": a_bytes},
    ]
    dom = max(cands, key=lambda c: c["ms_per_step"])
    per_launch_s = dom["ms_per_step"] / dom["launches"] * 1e-3
    bytes_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_launch / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
    traffic = recorded_traffic(args.config, dom["kernel"]) if not args.tris else None
    flops_tf = dom["flops"] / dom["launches"] / per_launch_s / 1e12 if per_launch_s > 0 else 0.0
    value = W * H * args.steps / dt
    wl = {1: "projector caustic (config 1)", 2: "glossy/specular procedural (config 2)",
          3: "glossy/specular procedural with the learned proposal (config 3)"}.get(args.config, f"config {args.config}")
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
        "config": {"workload": f"{wl}: {W}x{H}, {sc['tri'].shape[0]:,} tris, depth {params['max_depth']}, "
                               f"M={params['n_light']:,} light sub-paths, {params['cand_cap']:,} expected candidates; "
                               + ("learned proposal (subspace softmax and vMF retrace directions, 10 % "
                                  "defensive, trained online) on " if cfg.get("mlp") else "") +
                               f"plain method (PT, NEE, probabilistic connections, light tracing, proxy connections "
                               f"with variance-aware MIS, Gamma, tiles)",
                   "spp_per_step": 1, "max_depth": params["max_depth"], "n_light": params["n_light"],
                   "pilot": params.get("pilot", 16)},
        "mrays_per_s": rays * args.steps / dt / 1e6,
        "rays_per_step": rays,
        "ray_breakdown": {k: st[k] for k in ("rays_extend_eye", "rays_extend_light", "rays_shadow", "rays_proxy",
                                             "rays_recip")},
        "proxy": {k: st[k] for k in ("n_cand", "n_kept", "n_recip_samples", "n_recip_truncated",
                                     "n_proxy_attempts", "n_proxy_valid", "n_pool", "n_connections", "n_lt_splats",
                                     "n_nan", "chain_len_max")},
        "ms_breakdown": {"eye_extension": ms_ext, "reciprocal_block": ms_rec, "reciprocal_stage_a": ms_a},
        # stage A of the chains in the counting iteration: lanes busy in its traversal loops (node
        # visits over 64 x the wavefronts' loop trips) and the f/q samples it drew against those the
        # chains used
        "stage_a": {"simd_efficiency": stc["node_visits_stage_a"] / max(64.0 * stc["wave_trips_stage_a"], 1.0),
                    "samples_drawn": stc["n_drawn_stage_a"], "samples_used": stc["n_samples_stage_a"],
                    "pilot_samples_drawn": stc["n_drawn_pilot"]},
        "schedule": {"stage_a_budget": tune["stage_a_budget"], "round_grid": tune["round_grid"],
                     "bvh_width": tune["bvh_width"], "extension_workgroup": tune["ext_wg"],
                     "queue_chunk": tune["queue_chunk"], "stage_a_ahead": tune["stage_a_ahead"],
                     "stage_a_refill": tune["stage_a_refill"],
                     "autotune_iterations": k0, "ms_tuned": tune["ms_best"],
                     "ms_default": tune["ms_previous"]},
        "roofline": {"kernel": f"{dom['kernel']} ({dom['what']})", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "ms_per_launch": dom["ms_per_step"] / dom["launches"],
                     "traffic_GBs": traffic / per_launch_s / 1e9 if traffic and per_launch_s > 0 else None,
                     "fp32_TFLOPs": flops_tf, "fp32_frac": flops_tf / FP32_PEAK_TFLOPS,
                     "kernels": {c["kernel"]: {"ms_per_launch": c["ms_per_step"] / c["launches"],
                                               "GBs": (c["bytes"] / c["ms_per_step"] / 1e6 if c["ms_per_step"] > 0
                                                       else 0.0)} for c in cands}},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.config, sc, params)
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
