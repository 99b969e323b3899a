"""Benchmark of the hard-sphere collision step on one MI355X.

Workload (default): 16,000,000 polydisperse spheres (lognormal radii, median 1,
log-sd 0.25, clamped to [0.5, 2], m = r^3) at volume fraction 0.3 in a periodic
cube, N(0, 1) velocities, e = 0.8, dt = 0.4; seeded random sequential
placement.  A step is the whole path: validation and reach, binning, the
pair-test sweep, partner selection and resolve sweeps until none is left, free
flight and wrap.  Every timed step starts from the configured input: the
positions and velocities are restored from a device copy (inside the timed
region) before each step, so each step processes the same batch.

Prints one JSON line: particles stepped per second (value), pair tests per
second of the detect kernel, the detect kernel's ALU roofline fraction, and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair tests/s + particles stepped/s at 16M; FP32+recheck vs FP64 at equal pair set"
# FP64 arithmetic operations of one pair test in the detect kernel (separation 3,
# relative velocity 3, s 1, b 5, c 7, the cheap reject bound 1); compares excluded
OPS_PER_PAIR_TEST = 20
# 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz: non-FMA binary64 operations per second
PEAK_FP64_OPS = 256 * 4 * 16 * 2.4e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(args):
    import workloads
    if args.n:
        box = workloads.config(3, n=args.n)
    else:
        box = workloads.config(3)
    return box


def cpu_baseline(args):
    """The oracle (plain FP64 C, OpenMP) on a bounded sample: the same recipe at
    1M spheres (same density and velocity law, so the per-sphere cost matches)."""
    import oracle
    import workloads
    n = args.cpu_sample
    box = workloads.make_box(n, seed=103, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)
    t0 = time.perf_counter()
    res = oracle.step(box)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": n / dt, "unit": "particles/s", "cores": cores, "kind": "oracle",
        "sample": f"one step of {n} spheres, same recipe (lognormal r, phi 0.3, e 0.8, dt 0.4), "
                  f"seed 103; {dt:.2f} s; {res.n_pairs} pairs in {res.n_sweeps} sweeps",
        "pair_tests_per_s": res.pair_tests / dt,
        "seconds": dt,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="override N (default 16M)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--form", choices=["both", "fp64", "fp32"], default="both",
                    help="plain FP64 path, FP32 filter + FP64 recheck, or both (value = fp64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: the collision step is a single-GPU build; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2501_05340_amd as pc

    t0 = time.perf_counter()
    box = make_workload(args)
    log(f"workload {box.n} spheres, L={box.L[0]:.3f}, generated in {time.perf_counter() - t0:.1f} s")
    p0 = pc.Particles.from_box(box)

    def run_form(fp32: int):
        """K timed steps of one form, each from the configured input."""
        p = p0.clone()
        ctx = pc.Context(box.n, pc.pcol_default_opts(timing=1, fp32_filter=fp32))
        partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
        tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")

        def restore():
            for t, t_0 in zip(p.tensors()[:6], p0.tensors()[:6]):
                t.copy_(t_0)

        name = "fp32+recheck" if fp32 else "fp64"
        for k in range(args.warmup):
            restore()
            st = pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll)
            log(f"[{name}] warmup {k}: {st['n_pairs']} pairs, {st['n_sweeps']} sweeps, "
                f"detect {st['ms_detect']:.3f} ms")
        torch.cuda.synchronize()
        stats = []
        t_start = time.perf_counter()
        for k in range(args.steps):
            restore()
            stats.append(pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        for k, st in enumerate(stats):
            log(f"[{name}] step {k}: pairs {st['n_pairs']} sweeps {st['n_sweeps']} tests "
                f"{st['pair_tests']} rechecks {st['n_recheck']} bin {st['ms_bin']:.3f} detect "
                f"{st['ms_detect']:.3f} sweeps {st['ms_sweeps']:.3f} advance {st['ms_advance']:.3f} ms")
        out = {"p": p, "partner": partner, "stats": stats, "wall": wall}
        ctx.close()
        return out

    forms = {}
    if args.form in ("both", "fp64"):
        forms["fp64"] = run_form(0)
    if args.form in ("both", "fp32"):
        forms["fp32"] = run_form(1)
    main_form = "fp64" if "fp64" in forms else "fp32"
    R = forms[main_form]
    stats, wall = R["stats"], R["wall"]
    ms_step = wall * 1e3 / args.steps
    det_ms = [st["ms_detect"] for st in stats]
    tests = sum(st["pair_tests"] for st in stats)
    det_total = sum(det_ms) * 1e-3
    achieved = tests * OPS_PER_PAIR_TEST / det_total
    out = {
        "metric": METRIC,
        "value": box.n * args.steps / wall,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{box.name}: {box.n} polydisperse spheres, phi 0.3, e {box.e}, "
                               f"dt {box.dt}, periodic cube L={box.L[0]:.4f}",
                   "n": box.n, "form": "plain_fp64" if main_form == "fp64" else "fp32_filter+fp64_recheck"},
        "pair_tests_per_s": tests / det_total,
        "detect_ms_median": statistics.median(det_ms),
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "sweeps_per_step": statistics.mean(st["n_sweeps"] for st in stats),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_OPS, "traffic": None,
                     "kernel": "k_detect_half",
                     "note": f"{OPS_PER_PAIR_TEST} non-FMA FP64 ops per unordered pair test"},
    }
    if "fp64" in forms and "fp32" in forms:
        A, B = forms["fp64"], forms["fp32"]
        mismatch = int((A["partner"] != B["partner"]).sum().item())
        errs = []
        for f in ("vx", "vy", "vz"):
            a, b = getattr(A["p"], f), getattr(B["p"], f)
            errs.append(((a - b).abs() / a.abs().clamp_min(1e-300)).max().item())
        sb = B["stats"]
        dm32 = [st["ms_detect"] for st in sb]
        out["fp32_form"] = {
            "value": box.n * args.steps / B["wall"], "unit": "particles/s",
            "ms_per_step": B["wall"] * 1e3 / args.steps,
            "speedup_vs_fp64": A["wall"] / B["wall"],
            "detect_ms_median": statistics.median(dm32),
            "detect_speedup_vs_fp64": statistics.median(det_ms) / statistics.median(dm32),
            "pair_set_mismatch": mismatch,
            "max_rel_velocity_error": max(errs),
            "band": sb[0]["band"],
            "rechecks_per_step": statistics.mean(st["n_recheck"] for st in sb),
        }
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_sample} spheres")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
