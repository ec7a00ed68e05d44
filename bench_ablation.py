#!/usr/bin/env python3
"""Convergence ablations of two choices of the method, as MAPE over rendering time on one GPU.

  rr     The roulette of the reciprocal chains: the method's RRS function (Section 4.2, optimal r(x)
         of the appendix) against Booth's roulette, which goes on with probability
         min(1, prod |1 - f/(Bq)| / r) for a hand-set r and never splits (the baseline of the RR
         ablation, Section 6.5), at several r. Same B for both.
         Scored by the whole image under MIS (rr) or by the paths proxy sampling builds with
         the other strategies switched off (rr_proxy), where the variance of the 1/P estimates
         reaches the image undiluted by the other strategies and unweighted by the MIS.
  gamma  The choice of the incomplete light sub-path that a proxy connection completes: by the
         subspace matrix Gamma[T, S] against uniformly (Section 6.3). Only the paths that proxy
         sampling builds are scored (the other strategies are switched off), as in that section.

Measures, per variant and checkpoint (iterations 2^k, wall time from the first iteration with a
device synchronisation at each checkpoint):
  mape_ref  mean over pixels and RGB of |I - R| / (R + 0.01) against the stored CPU reference
            image of the workload (written by the reference renderer; its own noise sets a floor);
  mape_se   the MAPE that the per-pixel standard errors predict, mean sqrt(2/pi) SE / (R + 0.01),
            with R the reference, or the pooled mean of every variant where there is none. It has
            no floor, but understates an estimator whose variance is infinite or heavy-tailed
            (Booth's roulette with a small r), so both are reported where a reference exists.
  eff       1 / (mape^2 x seconds) at the last checkpoint: equal-time efficiency, larger is better;
  samples/cand  f/q samples the reciprocal chains consumed per kept candidate, last iteration;
  tmean/first   the variant's image mean, its brightest 0.1 % of values left out so that a single
                firefly does not decide it, over the same for the first variant: an estimator whose
                samples rarely reach its expectation shows up as a ratio well below 1, with a small
                mape_se that then says nothing about its error.

Prints one JSON line per variant and checkpoint, then a summary table. Needs the built HIP
library; nothing here falls back to the CPU.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
GOLD = os.path.join(ROOT, "tests", "golden")
EPS = 0.01

# workload: scene builder, path depth, light sub-paths per iteration, expected candidates,
# (eye subspaces, specular subspaces), stored reference
WORKLOADS = {
    "cornell_glass_64": (lambda s: s.cornell_glass(64, 64), 8, 4096, 400, (64, 64), "cfg0_o1_ref.npz"),
    "projector_128": (lambda s: s.projector(128, 128), 12, 65536, 2600, (256, 100), "cfg1_128_o3_ref.npz"),
    "projector_512": (lambda s: s.projector(512, 512), 12, 500_000, 20_000, (1000, 100), None),
    "glossy_1024": (lambda s: s.glossy_procedural(1024, 1024), 12, 262_144, 10_486, (1000, 100), None),
}


def variants(study, pt):
    full = (pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_MIS | pt.PT_FLAG_GAMMA | pt.PT_FLAG_TILES |
            pt.PT_FLAG_SPC | pt.PT_FLAG_LT)
    proxy = pt.PT_FLAG_NEE | pt.PT_FLAG_PROXY | pt.PT_FLAG_ONLY_PROXY_CLASS
    if study in ("rr", "rr_proxy"):
        base = full if study == "rr" else proxy | pt.PT_FLAG_GAMMA
        out = [("rrs", base, 1.0)]
        out += [(f"booth_r={r:g}", base | pt.PT_FLAG_BOOTH, r) for r in (0.01, 0.1, 1.0, 10.0, 100.0, 1000.0)]
        return out
    return [("gamma", proxy | pt.PT_FLAG_GAMMA, 1.0), ("uniform", proxy, 1.0)]


def trimmed_mean(m):
    """Mean of every value but the brightest 0.1 %."""
    v = np.sort(m.ravel())
    return float(v[:max(1, int(0.999 * v.size))].mean())


def run_variant(torch, pt, sc, wl, flags, booth_r, n_iter, seed):
    _, depth, n_light, cand_cap, subs, _ = wl
    W, H = sc["width"], sc["height"]
    params = dict(max_depth=depth, n_light=n_light, cand_cap=cand_cap, seed=seed, flags=flags, booth_r=booth_r)
    S = pt.Scene(sc, max_light_paths=n_light)
    S.build_subspaces(n_eye=subs[0], n_spec=subs[1])
    acc = torch.zeros(W * H * 3, device="cuda")
    acc2 = torch.zeros_like(acc)
    S.autotune(torch.zeros_like(acc), torch.zeros_like(acc), iteration=1 << 30, **params)
    torch.cuda.synchronize()
    checks, snaps = set(2 ** k for k in range(20) if 2 ** k <= n_iter) | {n_iter}, []
    trunc, last = 0.0, {}
    t0 = time.perf_counter()
    for k in range(n_iter):
        stats = k in (0, n_iter - 1)
        st = S.render_iteration(acc, acc2, stats=stats, iteration=k, **params)
        if st:
            trunc += st["n_recip_truncated"]
            last = st
        if k + 1 in checks:
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            m = (acc / (k + 1)).double().cpu().numpy().reshape(H, W, 3)
            v = np.maximum((acc2 / (k + 1)).double().cpu().numpy().reshape(H, W, 3) - m * m, 0) / (k + 1)
            snaps.append((k + 1, t, m, v))
            t0 += time.perf_counter() - t - t0   # copies out of the timed time
    S.release()
    return snaps, trunc, last["n_recip_samples"] / max(1.0, last["n_kept"])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--study", choices=("rr", "rr_proxy", "gamma"), default="rr")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="cornell_glass_64")
    ap.add_argument("--iters", type=int, default=256)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=None, help="also write the JSON lines to this file")
    a = ap.parse_args()

    import torch
    from paper_2503_23412_amd import pt
    from synth import scenes
    if not torch.cuda.is_available():
        sys.exit("bench_ablation.py needs a GPU")
    wl = WORKLOADS[a.workload]
    sc = wl[0](scenes)
    ref = np.load(os.path.join(GOLD, wl[5]))["mean"] if wl[5] and a.study == "rr" else None

    runs = []
    for name, flags, booth_r in variants(a.study, pt):
        print(f"# {a.study} {a.workload}: {name}, {a.iters} iterations", flush=True)
        snaps, trunc, spc = run_variant(torch, pt, sc, wl, flags, booth_r, a.iters, a.seed)
        runs.append((name, snaps, trunc, spc))
    # denominators: the reference, else the pooled mean of every variant at its last checkpoint
    R = ref if ref is not None else np.mean([s[-1][2] for _, s, _, _ in runs], axis=0)
    lines, table = [], []
    first_mean = trimmed_mean(runs[0][1][-1][2])
    for name, snaps, trunc, spc in runs:
        for n, t, m, v in snaps:
            rec = {"study": a.study, "workload": a.workload, "variant": name, "iters": n, "seconds": round(t, 4),
                   "mape_se": float(np.mean(math.sqrt(2 / math.pi) * np.sqrt(v) / (R + EPS)))}
            if ref is not None:
                rec["mape_ref"] = float(np.mean(np.abs(m - ref) / (ref + EPS)))
            rec["image_mean"] = float(m.mean())
            rec["image_tmean"] = trimmed_mean(m)
            lines.append(rec)
            print(json.dumps(rec), flush=True)
        last = lines[-1]
        mape = last.get("mape_ref", last["mape_se"])
        table.append((name, last["iters"], last["seconds"], last.get("mape_ref"), last["mape_se"],
                      1.0 / (mape * mape * last["seconds"]), trunc, spc,
                      last["image_tmean"] / first_mean))
    if a.out:
        with open(a.out, "w") as f:
            for rec in lines:
                f.write(json.dumps(rec) + "\n")
    print(f"\n{a.study} on {a.workload}, {a.iters} iterations, seed {a.seed}")
    print(f"{'variant':<16}{'iters':>7}{'seconds':>10}{'mape_ref':>10}{'mape_se':>10}{'eff':>10}{'trunc':>8}{'samples/cand':>14}{'tmean/first':>13}")
    for name, n, t, mr, ms, eff, trunc, spc, rel in table:
        mr_s = f"{mr:10.4f}" if mr is not None else f"{'-':>10}"
        print(f"{name:<16}{n:>7}{t:>10.3f}{mr_s}{ms:>10.4f}{eff:>10.1f}{trunc:>8.0f}{spc:>14.1f}{rel:>13.4f}")


if __name__ == "__main__":
    main()
