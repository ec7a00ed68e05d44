"""Photon-plane workload (Section 6.7: reciprocal estimation as the CMIS weight of photon planes).

One step = one iteration of pt_planes_render: n_planes photon planes drawn from the light and
gathered by every pixel's centre ray of the image, each ray-plane hit weighted by one chain of the
RRS reciprocal estimator. Prints one JSON line: ray-plane tests per second, the roofline of the
gather kernel (bound by FP32 ALU work: the algorithmic operations of the tests, hits and chain
samples over the kernel time from HIP events on the launch stream), and the FP64 oracle's rate
on a bounded sample (the same estimator with the exact reciprocal by quadrature, one host thread).

usage: python bench_planes.py [--steps K] [--warmup W] [--width 512 --height 512 --planes 8192] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic FP32 operations (an add, a multiply, a division or a comparison one each, an FMA
# two): one ray-plane test (the plane's normal against the ray, the division for t, two
# comparisons), one hit (the chord and sweep coordinates, the light point, m = w x d, its in-plane
# part, the cache cell) and one chain sample (the chord length through y, cos and sin, f, q, g and
# the node update)
FLOP_TEST = 8
FLOP_HIT = 74
FLOP_SAMPLE = 50
# vector FP32 peak of the build: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz; the library
# is compiled without packed FP32 instructions, so one FMA per lane per cycle
PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(sc_small, n_planes, budget_s=15.0):
    """The oracle's photon-plane estimator (exact 1/J by quadrature, FP64, one thread) on a bounded
    sample: as many iterations as fit the budget at 64 x 64 pixels and n_planes planes."""
    from oracle import oracle as O
    O.build(force=False)
    W, H = sc_small["width"], sc_small["height"]
    n_it, t_used = 0, 0.0
    while t_used < budget_s and n_it < 64:
        t0 = time.perf_counter()
        O.planes_render(sc_small, n_planes, 1, seed=100 + n_it)
        t_used += time.perf_counter() - t0
        n_it += 1
    return {"value": W * H * n_planes * n_it / t_used, "unit": "ray-plane tests/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle estimator with the exact reciprocal at {W}x{H} pixels, {n_planes} planes, "
                      f"{n_it} iterations"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--height", type=int, default=512)
    ap.add_argument("--planes", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench_planes.py measures one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2503_23412_amd import pt
    from synth import scenes
    torch.cuda.set_device(0)
    sc = scenes.planes_scene(args.width, args.height)
    W, H, M = sc["width"], sc["height"], args.planes
    P = pt.Planes(sc, max_planes=M)
    acc = torch.zeros(W * H * 3, device="cuda")
    acc2 = torch.zeros_like(acc)
    for k in range(args.warmup):
        P.render(acc, acc2, M, iteration=k, seed=1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        P.render(acc, acc2, M, iteration=args.warmup + k, seed=1)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_iter = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    log(f"timed {args.steps} steps in {dt:.3f} s ({ms_iter:.3f} ms per iteration from events)")
    # one iteration with counters (it synchronises) for the algorithmic operation count
    st = P.render(acc, acc2, M, iteration=args.warmup + args.steps, seed=1, stats=True)
    P.release()
    tests = float(W * H * M)
    flops = tests * FLOP_TEST + st["n_hits"] * FLOP_HIT + st["n_samples"] * FLOP_SAMPLE
    achieved = flops / (ms_iter * 1e-3) / 1e12
    out = {
        "metric": "ray-plane tests/s", "value": tests * args.steps / dt, "unit": "tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"photon planes, single scattering: {W}x{H} pixel-centre rays, {M} planes per "
                               f"iteration, rectangular light, homogeneous medium (sigma_s {sc['sigma_s']}, "
                               f"sigma_t {sc['sigma_t']}), CMIS weight by one RRS chain per hit"},
        "roofline": {"kernel": "k_planes_gather (with k_planes_gen, k_fill_u64: one iteration)", "bound": "alu",
                     "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS,
                     "traffic": None, "flops_per_launch": flops, "ms_per_launch": ms_iter},
        "hits_per_iteration": st["n_hits"], "chain_samples_per_iteration": st["n_samples"],
        "samples_per_hit": st["n_samples"] / max(st["n_hits"], 1.0), "n_truncated": st["n_truncated"],
        "n_nan": st["n_nan"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(scenes.planes_scene(64, 64), 256)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
