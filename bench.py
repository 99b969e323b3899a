"""Benchmark of the hard-sphere collision step on one MI355X.

Workload (default): 16,000,000 polydisperse spheres (lognormal radii, median 1,
log-sd 0.25, clamped to [0.5, 2], m = r^3) at volume fraction 0.3 in a periodic
cube, N(0, 1) velocities, e = 0.8, dt = 0.4; seeded random sequential
placement.  A step is the whole path: validation and reach, binning, the
pair-test sweep, partner selection and resolve sweeps until none is left, free
flight and wrap.  Every timed step starts from the configured input: the
positions and velocities are restored from a device copy before each step,
outside its timed interval (each interval is bracketed by device
synchronisations), so each step processes the same batch.

Prints one JSON line: particles stepped per second (value); pair tests per
second on the reference grid (cell side L / floor(L / reach), the 27 cells
around each sphere, unordered pairs, one full detection pass) for the GPU and
for the CPU oracle; the detect kernel's FP64 issue fraction with its counted and
algorithmic HBM fractions; every phase's time and fraction of the HBM peak on
its algorithmic bytes; and the CPU oracle timed on a bounded sample of the same
workload (median of 3, all host threads, with single-thread times).  Beside the
plain FP64 path it reports the binary32 filter form on the same input (its
survivors are decided by the binary64 rule, so both compute the same step
bitwise) and both forms' pair-set mismatch against the oracle on the sample;
the batched form (512 uneven boxes, about 8M spheres, one captured graph per
step, against a loop of single-box steps); the literal collision order; the
friction, walls and cell-ordered forms; the deposition; and the adjoint form
(10-step rollout of 1M spheres, forward and backward).
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
# FP64 vector operations of one pair test in the detect kernel's filter, the
# Gram form alpha_i + <P_j, Q_i> <= tol - beta_j: seven FMAs from alpha_i (the
# compare excluded; per-sphere terms and the candidate's threshold are formed
# once per sphere or chunk, not per pair).  An FMA is one operation here (two
# flops): 7 operations, 14 flops.
OPS_PER_PAIR_TEST = 7
FLOPS_PER_PAIR_TEST = 14
# 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz: binary64 vector operations per
# second (an FMA is one; the published 78.6 TFLOP/s counts it as two flops)
PEAK_FP64_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8e12  # bytes/s


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step_poly16M_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2501_05340_amd", "csrc", f)
                  for f in ("pcol_kernels.hip", "pcol_internal.h")]


def measured_traffic():
    """Counted HBM bytes from the committed counter summary of one 16M FP64 step
    (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy calibration): the detect
    kernel's bytes per launch, each phase's bytes per step and the bytes of one
    stored-order deposition call, or None when the kernel sources changed since
    the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        vals = dict(line.split(" = ", 1) for line in text.splitlines() if " = " in line)
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()
        if vals.get("kernel_sources_sha256", "").strip() != sha:
            return None
        return {"detect_launch": float(vals["traffic_bytes_per_launch"]),
                "phases": {k.split(".", 1)[1]: float(v) for k, v in vals.items()
                           if k.startswith("phase_counted_bytes.")},
                "deposition_call": float(vals["deposition_counted_bytes_per_call"])}
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ref_grid_pair_tests(x, y, z, L, reach, active=None) -> int:
    """Unordered candidate pairs among the active spheres in the 27-cell stencil of
    the reference grid, cell side L_k / floor(L_k / reach) (at least 3 cells per
    axis): the pairs a plain cell-list search with cells of the reach tests,
    whatever grid a code actually uses, so that GPU and oracle are counted alike."""
    import numpy as np
    nc = [int(np.floor(L[a] / reach)) for a in range(3)]
    assert min(nc) >= 3, "reference grid needs 3 cells per axis"
    keep = slice(None) if active is None else np.asarray(active, dtype=bool)
    c = [np.minimum(np.floor(np.asarray(p)[keep] / (L[a] / nc[a])).astype(np.int64), nc[a] - 1)
         for a, p in enumerate((x, y, z))]
    cnt = np.bincount((c[2] * nc[1] + c[1]) * nc[0] + c[0],
                      minlength=nc[0] * nc[1] * nc[2]).reshape(nc[2], nc[1], nc[0])
    total = int((cnt * (cnt - 1) // 2).sum())
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz, dy, dx) <= (0, 0, 0):
                    continue  # 13 forward neighbours: every unordered cell pair once
                total += int((cnt * np.roll(cnt, (-dz, -dy, -dx), axis=(0, 1, 2))).sum())
    return total


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def make_workload(args):
    import workloads
    if args.n:
        box = workloads.config(3, n=args.n)
    else:
        box = workloads.config(3)
    return box


SINGLE_THREAD = """
import json, statistics, sys, time
sys.path.insert(0, {root!r})
import oracle, workloads
out = {{}}
for name, box in (("config1", workloads.config(1)), ("config2_recipe_50k", workloads.config(2, n=50000))):
    ts = []
    for k in range(3):
        t0 = time.perf_counter()
        r = oracle.step(box)
        ts.append(time.perf_counter() - t0)
    t = statistics.median(ts)
    out[name] = {{"n": box.n, "seconds_median_of_3": t, "particles_per_s": box.n / t,
                  "pairs": r.n_pairs, "threads": oracle.max_threads()}}
print(json.dumps(out))
"""


def cpu_baseline(args):
    """The oracle (plain FP64 C, OpenMP) on a bounded sample: the same recipe at
    1M spheres (same density and velocity law, so the per-sphere cost matches),
    the whole step and one full detection pass each timed as the median of 3 runs
    on all host threads; single-thread times of configs 1 (2,000 spheres) and 2
    (its recipe at 50,000 spheres) in a child process with one OpenMP thread."""
    import subprocess
    import oracle
    import workloads
    n = args.cpu_sample
    box = workloads.make_box(n, seed=103, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)
    times, res = [], None
    for k in range(3):
        t0 = time.perf_counter()
        res = oracle.step(box)
        times.append(time.perf_counter() - t0)
    t_step = statistics.median(times)
    dtimes = []
    for k in range(3):
        t0 = time.perf_counter()
        _, _, tests = oracle.earliest(box)
        dtimes.append(time.perf_counter() - t0)
    t_det = statistics.median(dtimes)
    ref = ref_grid_pair_tests(box.x, box.y, box.z, box.L, res.reach)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    single = None
    try:
        r = subprocess.run([sys.executable, "-c", SINGLE_THREAD.format(root=ROOT)],
                           capture_output=True, text=True, env=env, timeout=300)
        single = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        single = None
    threads = oracle.max_threads()
    return {
        "value": n / t_step, "unit": "particles/s", "cores": threads, "kind": "oracle",
        "sample": f"one step of {n} spheres, same recipe (lognormal r, phi 0.3, e 0.8, dt 0.4), "
                  f"seed 103; median of 3 runs {t_step:.2f} s ({', '.join(f'{t:.2f}' for t in times)}); "
                  f"{res.n_pairs} pairs in {res.n_sweeps} sweeps",
        "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
        "seconds_median": t_step, "seconds_runs": times,
        # one full detection pass (every sphere active) on the oracle's grid, which is
        # the reference grid: its pair tests per second, as the GPU's below
        "pair_tests_per_s": ref / t_det, "ref_grid_pair_tests_per_pass": ref,
        "oracle_grid_pair_tests_per_pass": tests, "detect_pass_seconds_median": t_det,
        # the whole step: pair tests of every sweep (each sweep re-tests the active set)
        "step_pair_tests_all_sweeps": res.pair_tests,
        "step_pair_tests_per_s": res.pair_tests / t_step,
        "single_thread": single,
        "_box": box, "_res": res,
    }


def oracle_parity(pc, torch, cpu):
    """Both filter forms on the CPU baseline's sample against the oracle's step:
    spheres whose partner differs, contact times and states."""
    import numpy as np
    box, res = cpu["_box"], cpu["_res"]
    p0 = pc.Particles.from_box(box)
    out = {}
    for name, flt in (("fp64", 0), ("fp32", 1)):
        p = p0.clone()
        ctx = pc.Context(box.n, pc.pcol_default_opts(filter=flt))
        partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
        tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
        pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll)
        torch.cuda.synchronize()
        ctx.close()
        part = partner.cpu().numpy().astype(np.int64)
        tc = tcoll.cpu().numpy()
        err, nonbit = 0.0, 0
        for f in ("x", "y", "z", "vx", "vy", "vz"):
            a, b = getattr(p, f).cpu().numpy(), getattr(res, f)
            err = max(err, float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b))))))
            nonbit += int(np.count_nonzero(a.view(np.uint64) != b.view(np.uint64)))
        out[name] = {"pair_set_mismatch_vs_oracle": int(np.count_nonzero(part != res.partner)),
                     "tcoll_bitwise_equal": bool(np.array_equal(tc, res.tcoll, equal_nan=True)),
                     "max_rel_state_error_vs_oracle": err, "state_values_not_bitwise": nonbit,
                     "n": box.n, "pairs": res.n_pairs}
    return out


def batched_leg(args, pc, torch):
    """Batching workload: 512 periodic boxes, N_b log-uniform in [1k, 64k], phi_b
    uniform in [0.05, 0.35], radius 1, e 0.9, dt 0.4; all boxes stepped by one
    pcol_step_batched call per step (autotuned on its first call), against the
    same boxes stepped one pcol_step call at a time."""
    import numpy as np
    import workloads
    t0 = time.perf_counter()
    boxes = workloads.config(4)
    off = np.cumsum([0] + [b.n for b in boxes]).astype(np.int64)
    n = int(off[-1])
    cat = lambda f: torch.as_tensor(np.concatenate([getattr(b, f) for b in boxes]),
                                    dtype=torch.float64).cuda().contiguous()
    p0 = pc.Particles(*[cat(f) for f in ("x", "y", "z", "vx", "vy", "vz", "r", "m")])
    log(f"batched workload: {len(boxes)} boxes, {n} spheres, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    Ls = [b.L for b in boxes]
    dt, e = boxes[0].dt, boxes[0].e
    p = p0.clone()
    partner = torch.empty(n, dtype=torch.int32, device="cuda")

    def restore():
        for t, t_0 in zip(p.tensors()[:6], p0.tensors()[:6]):
            t.copy_(t_0)

    ctx = pc.Context(n, pc.pcol_default_opts(autotune=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st0 = pc.pcol_step_batched(ctx, p, off, Ls, dt, e, partner, None)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    log(f"[batched] first call {first_ms:.1f} ms (plan, tune={st0['tuned']}, capture): "
        f"cell_mult {st0['cell_mult']} home cells/workgroup {st0['home_cells']}")
    for k in range(args.warmup):
        restore()
        pc.pcol_step_batched(ctx, p, off, Ls, dt, e, partner, None)
    stats = []
    wall = 0.0
    for k in range(args.steps):  # each step from the configured input, restored untimed
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(pc.pcol_step_batched(ctx, p, off, Ls, dt, e, partner, None))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    for k, st in enumerate(stats):
        log(f"[batched] step {k}: pairs {st['n_pairs']} sweeps {st['n_sweeps']} replanned "
            f"{st['replanned']} host-finished {st['finished_on_host']}")
    # the same step as a loop of single-box calls
    ctx1 = pc.Context(max(b.n for b in boxes))
    q = p0.clone()
    part1 = torch.empty(n, dtype=torch.int32, device="cuda")
    views = []
    for b in range(len(boxes)):
        lo, hi = int(off[b]), int(off[b + 1])
        views.append((pc.Particles(*[t[lo:hi] for t in q.tensors()]), part1[lo:hi], boxes[b].L))

    def loop_step():
        for t, t_0 in zip(q.tensors()[:6], p0.tensors()[:6]):
            t.copy_(t_0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sub, pt, L in views:
            pc.pcol_step(ctx1, sub, L, dt, e, pt, None, stats=False)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    loop_step()
    nloop = max(1, min(args.steps, 3))
    loop_wall = sum(loop_step() for k in range(nloop)) / nloop
    # pair sets agree (loop partners are box-local)
    loc = torch.empty_like(partner)
    restore()
    pc.pcol_step_batched(ctx, p, off, Ls, dt, e, partner, None)
    for b in range(len(boxes)):
        lo, hi = int(off[b]), int(off[b + 1])
        pt = part1[lo:hi]
        loc[lo:hi] = torch.where(pt >= 0, pt + lo, pt)
    torch.cuda.synchronize()
    mismatch = int((loc != partner).sum().item())
    same_state = all(torch.equal(getattr(p, f).view(torch.int64), getattr(q, f).view(torch.int64))
                     for f in ("x", "y", "z", "vx", "vy", "vz"))
    ms = wall * 1e3 / args.steps
    out = {
        "value": n * args.steps / wall, "unit": "particles/s", "ms_per_step": ms,
        "n_boxes": len(boxes), "n": n,
        "box_loop_ms_per_step": loop_wall * 1e3,
        "speedup_vs_box_loop": loop_wall * 1e3 / ms,
        "pair_set_mismatch_vs_box_loop": mismatch, "state_bitwise_equal_to_box_loop": same_state,
        "first_call_ms": first_ms, "tuned_on_first_call": bool(st0["tuned"]),
        "cell_mult": st0["cell_mult"], "home_cells": st0["home_cells"],
        "total_cells": st0["total_cells"],
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "sweeps_per_step": statistics.mean(st["n_sweeps"] for st in stats),
        "replans_in_timed_steps": sum(st["replanned"] for st in stats),
    }
    ctx.close()
    ctx1.close()
    return out


def friction_leg(args, pc, torch, box, p0, ref):
    """The 16M step with spins and Coulomb friction (pcol_step_spin, mu 0.3, spins
    N(0, 1) / r per component, seed 17), each step from the configured input and
    spins, restored outside the timed interval; its pair set against the plain step's."""
    import numpy as np
    mu = 0.3
    rng = np.random.default_rng(17)
    w0 = [torch.as_tensor(rng.normal(size=box.n) / box.r).cuda() for _ in range(3)]
    p = p0.clone()
    w = [t.clone() for t in w0]
    ctx = pc.Context(box.n, pc.pcol_default_opts(timing=1))
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")

    def restore():
        for t, t_0 in zip(list(p.tensors()[:6]) + w, list(p0.tensors()[:6]) + w0):
            t.copy_(t_0)

    for k in range(args.warmup):
        restore()
        pc.pcol_step_spin(ctx, p, w, box.L, box.dt, box.e, mu, partner)
    stats, wall = [], 0.0
    for k in range(args.steps):
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(pc.pcol_step_spin(ctx, p, w, box.L, box.dt, box.e, mu, partner))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    changed = int((w[0] != w0[0]).sum().item())
    out = {
        "value": box.n * args.steps / wall, "unit": "particles/s",
        "ms_per_step": wall * 1e3 / args.steps, "mu": mu,
        "ms_per_step_over_plain": (wall / args.steps) / (ref["wall"] / args.steps),
        "pair_set_mismatch_vs_plain": int((partner != ref["partner"]).sum().item()),
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "spins_changed": changed,
        "sweeps_ms_median": statistics.median(st["ms_sweeps"] for st in stats),
    }
    ctx.close()
    log(f"[friction] {out['ms_per_step']:.3f} ms per step, {changed} spins changed")
    return out


def cell_order_leg(args, pc, torch, box, p0, ref):
    """The same 16M step with the spheres stored in cell order (sorted by the cell of a
    106^3 grid over the box, z slowest: a caller that keeps its particles sorted by
    element), permuted before timing; the pair count must equal the stored-order step's."""
    nc = 106
    cell = [torch.clamp(torch.floor(t / (box.L[d] / nc)), max=nc - 1).long()
            for d, t in enumerate((p0.x, p0.y, p0.z))]
    perm = torch.argsort((cell[2] * nc + cell[1]) * nc + cell[0], stable=True)
    q0 = pc.Particles(*[t[perm].contiguous() for t in p0.tensors()])
    del cell, perm
    p = q0.clone()
    ctx = pc.Context(box.n, pc.pcol_default_opts(timing=1))

    def restore():
        for t, t_0 in zip(p.tensors()[:6], q0.tensors()[:6]):
            t.copy_(t_0)

    for k in range(args.warmup):
        restore()
        pc.pcol_step(ctx, p, box.L, box.dt, box.e)
    stats, wall = [], 0.0
    for k in range(args.steps):
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(pc.pcol_step(ctx, p, box.L, box.dt, box.e))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    out = {
        "value": box.n * args.steps / wall, "unit": "particles/s",
        "ms_per_step": wall * 1e3 / args.steps,
        "ms_per_step_over_stored_order": (wall / args.steps) / (ref["wall"] / args.steps),
        "bin_ms_median": statistics.median(st["ms_bin"] for st in stats),
        "advance_ms_median": statistics.median(st["ms_advance"] for st in stats),
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "pairs_per_step_stored_order": statistics.mean(st["n_pairs"] for st in ref["stats"]),
    }
    ctx.close()
    log(f"[cell order] {out['ms_per_step']:.3f} ms per step, bin {out['bin_ms_median']:.3f} ms")
    return out


def literal_leg(args, pc, torch, box, p0, ref):
    """The 16M step in the paper's collision order taken literally (opts.order = 1:
    elements along the Morton curve, first eligible contact found), each step from
    the configured input; against the earliest-partner step on the same input: pairs,
    kinetic energy dissipated, spheres whose partner differs, mean contact time."""
    p = p0.clone()
    ctx = pc.Context(box.n, pc.pcol_default_opts(timing=1, order=1))
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")

    def restore():
        for t, t_0 in zip(p.tensors()[:6], p0.tensors()[:6]):
            t.copy_(t_0)

    for k in range(args.warmup):
        restore()
        pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll)
    stats, wall = [], 0.0
    for k in range(args.steps):
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    ke = lambda q: 0.5 * float((q.m * (q.vx * q.vx + q.vy * q.vy + q.vz * q.vz)).sum().item())
    ke0 = ke(p0)
    lit = {"loss": ke0 - ke(p), "partner": partner.clone(), "tcoll": tcoll.clone()}
    ctx.close()
    # the earliest-partner step's result on the same input (the plain leg's last step)
    rp, rt = ref["partner"], ref["tcoll"]
    erl_loss = ke0 - ke(ref["p"])
    hit_l, hit_e = lit["partner"] >= 0, rp >= 0
    out = {
        "value": box.n * args.steps / wall, "unit": "particles/s",
        "ms_per_step": wall * 1e3 / args.steps,
        "ms_per_step_over_plain": (wall / args.steps) / (ref["wall"] / args.steps),
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "pairs_per_step_earliest_rule": statistics.mean(st["n_pairs"] for st in ref["stats"]),
        "sweeps_per_step": statistics.mean(st["n_sweeps"] for st in stats),
        "ke_dissipated": lit["loss"], "ke_dissipated_earliest_rule": erl_loss,
        "colliding_spheres_with_other_partner": int(((lit["partner"] != rp) & hit_l & hit_e).sum().item()),
        "colliding_spheres": int(hit_l.sum().item()),
        "mean_contact_time": float(lit["tcoll"][hit_l].mean().item()),
        "mean_contact_time_earliest_rule": float(rt[hit_e].mean().item()),
    }
    log(f"[literal] {out['ms_per_step']:.3f} ms per step, {out['pairs_per_step']:.0f} pairs "
        f"({out['pairs_per_step_earliest_rule']:.0f} earliest rule), {out['sweeps_per_step']:.1f} sweeps")
    return out


def walls_leg(args, pc, torch, box, p0, ref):
    """The 16M step between reflective walls on all three axes (pcol_step_walls), each
    step from the configured input, restored outside the timed interval."""
    walls = (1, 1, 1)
    p = p0.clone()
    ctx = pc.Context(box.n)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")

    def restore():
        for t, t_0 in zip(p.tensors()[:6], p0.tensors()[:6]):
            t.copy_(t_0)

    for k in range(args.warmup):
        restore()
        pc.pcol_step_walls(ctx, p, box.L, walls, box.dt, box.e, partner)
    stats, wall = [], 0.0
    for k in range(args.steps):
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(pc.pcol_step_walls(ctx, p, box.L, walls, box.dt, box.e, partner))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    out = {
        "value": box.n * args.steps / wall, "unit": "particles/s",
        "ms_per_step": wall * 1e3 / args.steps, "walls": list(walls),
        "ms_per_step_over_plain": (wall / args.steps) / (ref["wall"] / args.steps),
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "pairs_per_step_plain": statistics.mean(st["n_pairs"] for st in ref["stats"]),
        "partners_differing_from_plain": int((partner != ref["partner"]).sum().item()),
    }
    ctx.close()
    log(f"[walls] {out['ms_per_step']:.3f} ms per step, {out['pairs_per_step']:.0f} pairs")
    return out


def deposition_leg(args, pc, torch, box, p0):
    """Deposition of four source components (momentum and energy; standard normal,
    seed 3) of the 16M spheres at their start positions onto the corner nodes of a
    160^3 periodic grid over the same box (3.9 spheres per element), pcol_deposit per
    call: position check with its readback, counting sort by element, then element
    corner sums and node sums per tile of nodes."""
    import workloads
    comp, nc = 4, (160, 160, 160)
    a = torch.as_tensor(workloads.deposit_case(box.n, seed=3, L=box.L, comp=comp)[3]).cuda()
    ctx = pc.Context(1)
    nnode = nc[0] * nc[1] * nc[2]
    out = torch.empty((nc[2], nc[1], nc[0], comp), dtype=torch.float64, device="cuda")

    def timed(x, y, z, src):
        for k in range(args.warmup):
            pc.pcol_deposit(ctx, x, y, z, src, nc, box.L, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            pc.pcol_deposit(ctx, x, y, z, src, nc, box.L, out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    # the same spheres stored in element order (as a code that keeps its particles
    # sorted by host element holds them), permuted before timing
    cell = [torch.clamp(torch.floor(t / (box.L[d] / nc[d])), max=nc[d] - 1).long()
            for d, t in enumerate((p0.x, p0.y, p0.z))]
    perm = torch.argsort((cell[2] * nc[1] + cell[1]) * nc[0] + cell[0])
    xs, ys, zs = p0.x[perm].contiguous(), p0.y[perm].contiguous(), p0.z[perm].contiguous()
    as_ = a[:, perm].contiguous()
    wall_sorted = timed(xs, ys, zs, as_)
    sorted_out = out.clone()
    wall = timed(p0.x, p0.y, p0.z, a)
    sorted_diff = float((sorted_out - out).abs().max().item())
    del xs, ys, zs, as_, perm, cell
    # algorithmic bytes: positions and sources read once, the node array written once
    # (the operator's own traffic, whatever the scratch of the sort)
    alg = box.n * (24 + 8 * comp) + nnode * comp * 8
    counted = measured_traffic()
    traffic = counted["deposition_call"] if counted else None
    res = {
        "value": box.n / wall, "unit": "particles/s", "ms_per_call": wall * 1e3,
        "nc": list(nc), "comp": comp, "spheres_per_element": box.n / nnode,
        "corner_terms_per_s": box.n * 8 * comp / wall,
        "algorithmic_bytes": alg, "algorithmic_GBps": alg / wall / 1e9,
        # the whole call (sort and sums) against the HBM peak, on its algorithmic bytes
        "roofline": {"bound": "hbm", "achieved": alg / wall / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": alg / wall / 8e12, "traffic": traffic,
                     "traffic_unit": "bytes per call",
                     "hbm_frac_counted": traffic / wall / 8e12 if traffic else None,
                     "kernel": "pcol_deposit (k_dep_count, scan, k_dep_scatter, k_dep_tile)"},
        "element_sorted_ms_per_call": wall_sorted * 1e3,
        "element_sorted_max_abs_diff": sorted_diff,
        "conservation_rel_error": float(
            ((out.sum(dim=(0, 1, 2)) - a.sum(dim=1)).abs().max() / a.abs().sum(dim=1).max()).item()),
    }
    ctx.close()
    log(f"[deposition] {res['ms_per_call']:.3f} ms per call ({wall_sorted * 1e3:.3f} ms in element "
        f"order), "
        f"{res['corner_terms_per_s'] / 1e9:.1f} G corner terms/s")
    return res


def adjoint_leg(args, pc, torch):
    """Differentiation workload: 1M spheres (phi 0.2, radius 1, e 0.9 learnable),
    10 FP64 steps through the autograd rollout, loss = sum |v|^2 at the end;
    forward (steps plus checkpoints) and backward (recompute plus adjoint) timed."""
    import workloads
    box = workloads.config(5)
    n = box.n
    ctx = pc.Context(n)
    p0 = pc.Particles.from_box(box)
    nsteps = 10

    def run():
        ts = [getattr(p0, f).clone().requires_grad_(True) for f in ("x", "y", "z", "vx", "vy", "vz")]
        e = torch.tensor(box.e, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = pc.Rollout.apply(*ts, e, p0.r, p0.m, box.L, box.dt, nsteps, ctx, 1)
        loss = (out[3] * out[3] + out[4] * out[4] + out[5] * out[5]).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3, e.grad.item()

    run()
    fw, bw, ge = [], [], None
    for k in range(max(1, min(args.steps, 3))):
        a, b, ge = run()
        fw.append(a)
        bw.append(b)
    ctx.close()
    return {"n": n, "steps": nsteps, "forward_ms": statistics.median(fw),
            "backward_ms": statistics.median(bw),
            "backward_over_forward": statistics.median(bw) / statistics.median(fw),
            "checkpoint_every": 1, "dloss_de": ge}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="override N (default 16M)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--form", choices=["all", "fp64", "fp32"], default="all",
                    help="filter form(s) to time: binary64 or binary32 (value = fp64 when it runs)")
    ap.add_argument("--split-quantile", type=float, default=None,
                    help="extent split quantile of the single-box path (default: the library's)")
    ap.add_argument("--cell-mult", type=float, default=None,
                    help="cell side factor of the single-box path (default: the library's)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-form leg")
    ap.add_argument("--no-friction", action="store_true", help="skip the friction-and-spin leg")
    ap.add_argument("--no-deposition", action="store_true", help="skip the deposition leg")
    ap.add_argument("--no-walls", action="store_true", help="skip the walls leg")
    ap.add_argument("--no-literal", action="store_true",
                    help="skip the leg in the paper's literal collision order")
    ap.add_argument("--no-cell-order", action="store_true",
                    help="skip the leg with the spheres stored in cell order")
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

    def run_form(name: str, flt: int, split):
        """W warm-up and K timed steps of one filter form, each from the configured
        input: the input is restored before a step, outside its timed interval
        (a step is bracketed by device synchronisations), so every timed step is
        the configured workload and nothing else."""
        p = p0.clone()
        kw = {}
        if split is not None:
            kw["split_quantile"] = split
        if args.cell_mult is not None:
            kw["cell_mult"] = args.cell_mult
        ctx = pc.Context(box.n, pc.pcol_default_opts(timing=1, filter=flt, **kw))
        partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
        tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")

        def restore():
            for t, t_0 in zip(p.tensors()[:6], p0.tensors()[:6]):
                t.copy_(t_0)

        for k in range(args.warmup):
            restore()
            st = pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll)
            log(f"[{name}] warmup {k}: {st['n_pairs']} pairs, {st['n_sweeps']} sweeps, "
                f"detect {st['ms_detect']:.3f} ms, nc {st['nc']}, wide {st['n_wide']}, "
                f"rho_c {st['rho_c']:.4f}, reach {st['reach']:.4f}")
        stats = []
        wall = 0.0
        for k in range(args.steps):
            restore()
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            stats.append(pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll))
            torch.cuda.synchronize()
            wall += time.perf_counter() - t_start
        for k, st in enumerate(stats):
            log(f"[{name}] step {k}: pairs {st['n_pairs']} sweeps {st['n_sweeps']} tests "
                f"{st['pair_tests']} rechecks {st['n_recheck']} bin {st['ms_bin']:.3f} detect "
                f"{st['ms_detect']:.3f} sweeps {st['ms_sweeps']:.3f} advance {st['ms_advance']:.3f} ms")
        out = {"p": p, "partner": partner, "tcoll": tcoll, "stats": stats, "wall": wall}
        ctx.close()
        return out

    # filter 0: binary64 Gram filter (the plain FP64 path); 1: binary32 filter whose
    # survivors go to the binary64 rule, so both forms compute the same step bitwise.
    specs = {"fp64": (0, args.split_quantile), "fp32": (1, args.split_quantile)}
    wanted = list(specs) if args.form == "all" else [args.form]
    forms = {k: run_form(k, *specs[k]) for k in wanted}
    main_form = "fp64" if "fp64" in forms else wanted[0]
    R = forms[main_form]
    stats, wall = R["stats"], R["wall"]
    ms_step = wall * 1e3 / args.steps
    det_ms = [st["ms_detect"] for st in stats]
    tests = sum(st["pair_tests"] for st in stats)
    det_total = sum(det_ms) * 1e-3
    achieved = tests * OPS_PER_PAIR_TEST / det_total
    flops = tests * FLOPS_PER_PAIR_TEST / det_total
    # the reference grid's pair tests of one full detection pass (every sphere
    # active), the count the oracle's rate below uses too
    ref_tests = ref_grid_pair_tests(box.x, box.y, box.z, box.L, stats[0]["reach"])
    det_med = statistics.median(det_ms) * 1e-3
    counted = measured_traffic() if main_form == "fp64" else None
    traffic = counted["detect_launch"] if counted else None
    contacts = statistics.mean(st["contacts"] for st in stats)
    pairs = statistics.mean(st["n_pairs"] for st in stats)
    med = lambda key: statistics.median(st[key] for st in stats) * 1e-3
    # algorithmic HBM bytes of each phase (what its kernels must move):
    #  bin: validation, reach and cell ids (one pass on the grid of the last
    #    step) read the 64-B state and write cell and slot (8 B); the scatter
    #    reads 56 + 8 B and writes the 64-B record and the 4-B sorted position;
    #  detect: each first-layer record read once (64 B), a contact count per sphere
    #    (4 B), 12 B per contact side in the slots;
    #  sweeps: per collided sphere its record and its partner's (128 B), two masses,
    #    its key (12 B) and its 64-B output record;
    #  advance: the sorted position (4 B), the output record (64 B), the 48-B start
    #    state read; the 48-B state, partner and time (12 B) written.
    n = box.n
    phase_bytes = {"bin": n * (72 + 132), "detect": n * 68 + contacts * 2 * 12,
                   "sweeps": 2 * pairs * (128 + 16 + 12 + 64), "advance": n * 176}
    phase_ms = {"bin": med("ms_bin"), "detect": det_med, "sweeps": med("ms_sweeps"),
                "advance": med("ms_advance")}
    phases = {k: {"ms": phase_ms[k] * 1e3, "algorithmic_bytes": phase_bytes[k],
                  "hbm_frac_algorithmic": phase_bytes[k] / phase_ms[k] / PEAK_HBM}
              for k in phase_ms}
    # the phase's kernels' counted bytes (one step, from the counter summary) over
    # the phase's time measured here
    for k, ph in phases.items():
        cb = counted["phases"].get(k) if counted else None
        ph["counted_bytes"] = cb
        ph["hbm_frac_counted"] = cb / phase_ms[k] / PEAK_HBM if cb else None
    form_names = {"fp64": "plain_fp64 (binary64 Gram filter)", "fp32": "binary32 filter + binary64 rule"}
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{box.name}: {box.n} polydisperse spheres, phi 0.3, e {box.e}, "
                               f"dt {box.dt}, periodic cube L={box.L[0]:.4f}",
                   "n": box.n, "form": form_names[main_form],
                   "split_quantile": (specs[main_form][1] if specs[main_form][1] is not None
                                      else pc.pcol_default_opts().split_quantile)},
        # pair tests per second on the reference grid (one full pass per detect)
        "pair_tests_per_s": ref_tests / det_med,
        "ref_grid_pair_tests_per_pass": ref_tests,
        # the pairs the kernels actually test (the extent split removes most)
        "pair_tests_split_per_pass": tests / args.steps,
        "pair_tests_split_per_s": tests / det_total,
        "detect_ms_median": statistics.median(det_ms),
        "phases": phases,
        "pairs_per_step": statistics.mean(st["n_pairs"] for st in stats),
        "sweeps_per_step": statistics.mean(st["n_sweeps"] for st in stats),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / PEAK_FP64_OPS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch",
                     # the same launch against the HBM peak: counted bytes (FETCH_SIZE +
                     # WRITE_SIZE, copy-calibrated) and algorithmic bytes
                     "hbm_frac_counted": (traffic / det_med / PEAK_HBM) if traffic else None,
                     "hbm_frac_algorithmic": phase_bytes["detect"] / det_med / PEAK_HBM,
                     "kernel": "k_detect_half64g",
                     "note": f"FP64 vector operations (an FMA counts one): {OPS_PER_PAIR_TEST} per "
                             f"unordered pair test; as flops ({FLOPS_PER_PAIR_TEST} per test) "
                             f"{flops / 1e12:.2f} of 78.6 TFLOP/s"},
    }
    for name in forms:
        if name == main_form:
            continue
        A, B = R, forms[name]
        mismatch = int((A["partner"] != B["partner"]).sum().item())
        state_equal = all(torch.equal(getattr(A["p"], f).view(torch.int64),
                                      getattr(B["p"], f).view(torch.int64))
                          for f in ("x", "y", "z", "vx", "vy", "vz"))
        errs = []
        for f in ("vx", "vy", "vz"):
            a, b = getattr(A["p"], f), getattr(B["p"], f)
            errs.append(((a - b).abs() / a.abs().clamp_min(1e-300)).max().item())
        sb = B["stats"]
        dmb = [st["ms_detect"] for st in sb]
        tb = sum(st["pair_tests"] for st in sb)
        sub = {
            "form": form_names[name],
            "value": box.n * args.steps / B["wall"], "unit": "particles/s",
            "ms_per_step": B["wall"] * 1e3 / args.steps,
            "speedup_vs_" + main_form: A["wall"] / B["wall"],
            "detect_ms_median": statistics.median(dmb),
            "detect_speedup_vs_" + main_form: statistics.median(det_ms) / statistics.median(dmb),
            "pair_tests_per_step": tb / args.steps,
            "pair_tests_per_s": tb / (sum(dmb) * 1e-3),
            "pair_set_mismatch_vs_fp64_gpu": mismatch,
            "state_bitwise_equal_to_fp64_gpu": state_equal,
            "max_rel_velocity_error": max(errs),
            "rechecks_per_step": statistics.mean(st["n_recheck"] for st in sb),
            "split_quantile": (specs[name][1] if specs[name][1] is not None
                               else pc.pcol_default_opts().split_quantile),
        }
        if name == "fp32":
            sub["band"] = sb[0]["band"]
        out[name + "_form"] = sub
    if not args.no_batched:
        out["batched_form"] = batched_leg(args, pc, torch)
    if not args.no_friction and "fp64" in forms:
        out["friction_form"] = friction_leg(args, pc, torch, box, p0, forms["fp64"])
    if not args.no_cell_order and "fp64" in forms:
        out["cell_order_form"] = cell_order_leg(args, pc, torch, box, p0, forms["fp64"])
    if not args.no_walls and "fp64" in forms:
        out["walls_form"] = walls_leg(args, pc, torch, box, p0, forms["fp64"])
    if not args.no_literal and "fp64" in forms:
        out["literal_order_form"] = literal_leg(args, pc, torch, box, p0, forms["fp64"])
    if not args.no_deposition:
        out["deposition"] = deposition_leg(args, pc, torch, box, p0)
    if not args.no_adjoint:
        out["adjoint_form"] = adjoint_leg(args, pc, torch)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_sample} spheres")
        cpu = cpu_baseline(args)
        log("both filter forms against the oracle on its sample")
        par = oracle_parity(pc, torch, cpu)
        out["parity_vs_oracle"] = par
        if "fp32_form" in out:
            out["fp32_form"]["pair_set_mismatch_vs_oracle"] = par["fp32"]["pair_set_mismatch_vs_oracle"]
        out["cpu_baseline"] = {k: v for k, v in cpu.items() if not k.startswith("_")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
