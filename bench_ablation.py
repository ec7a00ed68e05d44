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
  learned  The learned proposal (network softmax over the specular subspaces, vMF mixture for the
         first retrace direction at glossy vertices; 10 % defensive plain sampling, trained online
         by the library's kernels) against the plain method, every strategy on, at EQUAL GPU TIME
         (--seconds per variant). The reference is the plain method run for --ref-seconds on the same
         scene; images are compared as 4 x 4 block means (a block of the full camera covers one pixel
         of the same camera at a quarter of the resolution), which the reference's per-block standard
         error turns into the floor mape_ref_floor reported beside the MAPE.

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
    if study == "learned":
        return [("plain", full, 1.0), ("learned", full | pt.PT_FLAG_MLP | pt.PT_FLAG_MLP_DIR, 1.0),
                ("learned_selection", full | pt.PT_FLAG_MLP, 1.0)]
    return [("gamma", proxy | pt.PT_FLAG_GAMMA, 1.0), ("uniform", proxy, 1.0)]


def run_timed(torch, pt, sc, wl, flags, seconds, seed, n_checks=4):
    """Iterations until `seconds` of rendering (device-synchronised wall time, set-up and autotuning
    excluded); per checkpoint (seconds / 2^j), the mean image as 4 x 4 block means and the variance
    of its mean from per-iteration block images."""
    _, depth, n_light, cand_cap, subs, _ = wl
    W, H = sc["width"], sc["height"]
    params = dict(max_depth=depth, n_light=n_light, cand_cap=cand_cap, seed=seed, flags=flags, booth_r=1.0,
                  train_iters=1 << 30, mlp_mix=0.9, mlp_lr=1e-3)
    S = pt.Scene(sc, max_light_paths=n_light)
    S.build_subspaces(n_eye=subs[0], n_spec=subs[1])
    img = torch.zeros(W * H * 3, device="cuda")
    S.autotune(torch.zeros_like(img), None, iteration=1 << 29, **params)
    s1 = torch.zeros((H // 4) * (W // 4) * 3, dtype=torch.float64, device="cuda")
    s2 = torch.zeros_like(s1)
    torch.cuda.synchronize()
    checks = sorted(seconds / 2 ** j for j in range(n_checks))
    snaps, k, t_run, t_say = [], 0, 0.0, 30.0
    while checks:
        if t_run >= t_say:
            print(f"#   {k} iterations, {t_run:.0f} s", flush=True)
            t_say += 30.0
        t0 = time.perf_counter()
        img.zero_()
        S.render_iteration(img, None, iteration=k, **params)
        torch.cuda.synchronize()
        t_run += time.perf_counter() - t0
        b = img.view(H // 4, 4, W // 4, 4, 3).double().mean(dim=(1, 3)).reshape(-1)
        s1 += b
        s2 += b * b
        k += 1
        if t_run >= checks[0]:
            checks.pop(0)
            m = (s1 / k).cpu().numpy().reshape(H // 4, W // 4, 3)
            v = np.maximum((s2 / k).cpu().numpy().reshape(H // 4, W // 4, 3) - m * m, 0) / max(k - 1, 1)
            snaps.append((k, t_run, m, v))
    tot = S.totals()
    S.release()
    return snaps, tot


def learned_study(a, torch, pt, sc, wl):
    """Equal-time MAPE of the learned proposal against the plain method (see the module docstring)."""
    print(f"# reference: plain method, {a.ref_seconds} s", flush=True)
    ref_snaps, ref_tot = run_timed(torch, pt, sc, wl, variants("learned", pt)[0][1], a.ref_seconds, a.seed + 1000,
                                   n_checks=1)
    _, _, R, VR = ref_snaps[-1]
    floor = float(np.mean(math.sqrt(2 / math.pi) * np.sqrt(VR) / (R + EPS)))
    lines = []
    for name, flags, _ in variants("learned", pt):
        print(f"# learned study {a.workload}: {name}, {a.seconds} s", flush=True)
        snaps, tot = run_timed(torch, pt, sc, wl, flags, a.seconds, a.seed)
        for n, t, m, v in snaps:
            rec = {"study": "learned", "workload": a.workload, "variant": name, "iters": n, "seconds": round(t, 3),
                   "mape_ref": float(np.mean(np.abs(m - R) / (R + EPS))),
                   "mape_se": float(np.mean(math.sqrt(2 / math.pi) * np.sqrt(v) / (R + EPS))),
                   "mape_ref_floor": floor, "ref_iters": ref_snaps[-1][0], "ref_seconds": round(ref_snaps[-1][1], 2),
                   "image_mean": float(m.mean()), "n_nan": tot["n_nan"], "n_recip_truncated": tot["n_recip_truncated"]}
            lines.append(rec)
            print(json.dumps(rec), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            for rec in lines:
                f.write(json.dumps(rec) + "\n")
    print(f"\nlearned vs plain on {a.workload} at {a.seconds} s each, seed {a.seed}; reference {a.ref_seconds} s "
          f"(MAPE floor {floor:.4f})")
    print(f"{'variant':<20}{'iters':>7}{'seconds':>10}{'mape_ref':>10}{'mape_se':>10}")
    for rec in lines:
        print(f"{rec['variant']:<20}{rec['iters']:>7}{rec['seconds']:>10.2f}{rec['mape_ref']:>10.4f}{rec['mape_se']:>10.4f}")


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
    ap.add_argument("--study", choices=("rr", "rr_proxy", "gamma", "learned"), default="rr")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="cornell_glass_64")
    ap.add_argument("--iters", type=int, default=256)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=None, help="also write the JSON lines to this file")
    ap.add_argument("--seconds", type=float, default=20.0, help="learned study: rendering time per variant")
    ap.add_argument("--ref-seconds", type=float, default=240.0, help="learned study: rendering time of the reference")
    a = ap.parse_args()

    import torch
    from paper_2503_23412_amd import pt
    from synth import scenes
    if not torch.cuda.is_available():
        sys.exit("bench_ablation.py needs a GPU")
    wl = WORKLOADS[a.workload]
    sc = wl[0](scenes)
    if a.study == "learned":
        learned_study(a, torch, pt, sc, wl)
        return
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
