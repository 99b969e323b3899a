"""GPU parity at the edges of the contact rule and of the filters' rounding bounds,
and the paper's kinetic-energy run on the GPU.

The edge box (``tests/edge_cases.py``) holds, inside a dense polydisperse box,
constructed pairs with the contact time exactly dt, a tangent contact (D = 0),
touching (c = 0) and overlapping (c < 0) pairs, b = 0 and a = 0 pairs, grazing
pairs whose closest approach lies within 1e-3 of the contact distance on either
side, slow approaches whose contact falls within 1e-11 of dt on either side (the
pairs whose filter value lies nearest the thresholds of the binary64 and binary32
filters), exact three-sphere ties in both index orders (inside the box, through the
periodic face, and split between the grid's two layers), and spheres at 0 and just
below L.  Every form of the step is compared with the oracle bitwise on it: both
filters, the extent split off, default and at quantile 0.9, one contact slot (the
exact search), walls, friction, the batched form and pcol_detect's keys.  The
designed outcomes are asserted too, so that each edge is known to be exercised.

Sec. "Kinetic Energy Analogy and Preservation": 5,000 spheres of diameter 0.02 in a
periodic cube of side 2, speed 1 in random directions, e = 1, 1,000 steps on the GPU
in lockstep with the oracle (every step bitwise), kinetic energy preserved to
rounding, the velocity components relaxed to the Maxwell-Boltzmann normal law.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.edge_cases import DT, check_designed as _check_designed, edge_box
from tests.gpu_helpers import FIELDS, compare_step, gpu_step, to_host

pytestmark = pytest.mark.gpu

import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def edge():
    box, groups = edge_box()
    return box, groups, oracle.step(box)


@pytest.mark.parametrize("opts", [{}, {"filter": 1}, {"split_quantile": 0.0},
                                  {"split_quantile": 0.9}, {"filter": 1, "split_quantile": 0.9},
                                  {"contact_slots": 1}, {"home_cells": 1}],
                         ids=["plain", "fp32", "nosplit", "split0.9", "fp32split0.9", "slots1",
                              "cells1"])
def test_edge_box_matches_oracle(edge, opts):
    box, groups, orc = edge
    _announce(f"edge box {opts}")
    gpu = gpu_step(box, **opts)
    assert compare_step(box, gpu, orc) == 0
    _check_designed(groups, gpu[1], gpu[2])
    st = gpu[3]
    if opts.get("split_quantile") == 0.9:
        # the large sphere of the split tie is searched separately
        assert st["n_wide"] > 0 and 2.0 + 2.0 * box.dt > st["rho_c"] > 0.0


def test_edge_box_contact_at_dt_rejected_just_below(edge):
    """dt one ulp below 0.5: the pair whose contact time is exactly 0.5 no longer
    collides; everything else as the oracle."""
    box, groups, _ = edge
    b = box.copy()
    b.dt = math.nextafter(DT, 0.0)
    _announce("edge box, dt just below the designed contact time")
    orc = oracle.step(b)
    for flt in (0, 1):
        gpu = gpu_step(b, filter=flt)
        assert compare_step(b, gpu, orc) == 0
        g = next(g for g in groups if g.name == "t_eq_dt")
        assert gpu[1][g.first] == -1 and gpu[1][g.first + 1] == -1
        _check_designed(groups, gpu[1], gpu[2], dt=b.dt)


def test_edge_box_detect_keys(edge):
    """pcol_detect over the edge box, all active and with a random mask, against the
    oracle's earliest partners: the exact ties go to the smaller index."""
    box, groups, _ = edge
    p = pc.Particles.from_box(box)
    rng = np.random.default_rng(8)
    ctx = pc.Context(box.n)
    pc.pcol_bin(ctx, p, box.L, box.dt)
    for act in (None, (rng.random(box.n) < 0.6).astype(np.uint8)):
        a_dev = None if act is None else torch.as_tensor(act).cuda()
        key, tmin = pc.pcol_detect(ctx, p, box.L, box.dt, active=a_dev)
        torch.cuda.synchronize()
        key = key.cpu().numpy().view(np.uint64)
        op, ot, _ = oracle.earliest(box, act)
        none = np.uint64(2 ** 64 - 1)
        kj = np.where(key == none, -1, (key & np.uint64(0xFFFFFFFF)).astype(np.int64))
        assert np.array_equal(kj, op)
        assert np.array_equal(tmin.cpu().numpy(), ot)


def test_edge_box_walls_and_friction(edge):
    box, groups, _ = edge
    walls = (0, 1, 1)  # x stays periodic: the groups through the face x = 0 keep wrapping
    _announce("edge box between walls on y and z")
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step_walls(ctx, p, box.L, walls, box.dt, box.e, partner, tcoll)
    torch.cuda.synchronize()
    gpu = (to_host(p), partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st)
    assert compare_step(box, gpu, oracle.step_walls(box, walls)) == 0
    _announce("edge box with friction and spin")
    rng = np.random.default_rng(19)
    w0 = np.stack([rng.normal(size=box.n) / box.r for _ in range(3)])
    p = pc.Particles.from_box(box)
    w = [torch.as_tensor(w0[k]).cuda() for k in range(3)]
    pc.pcol_step_spin(ctx, p, w, box.L, box.dt, box.e, 0.4, partner, tcoll)
    torch.cuda.synchronize()
    ref = oracle.step_spin(box, w0, 0.4)
    gpu = (to_host(p), partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), None)
    assert compare_step(box, gpu, ref) == 0
    for k, f in enumerate(("wx", "wy", "wz")):
        assert np.array_equal(w[k].cpu().numpy(), getattr(ref, f))


def test_edge_box_in_the_batched_form(edge, tmp_path, monkeypatch):
    """The edge box as one of three boxes of one pcol_step_batched call."""
    box, groups, orc = edge
    monkeypatch.setenv("PCOL_TUNE_CACHE", str(tmp_path / "tune.txt"))
    others = [workloads.make_box(3000, seed=41, phi=0.25, radius=1.0, e=box.e, dt=box.dt),
              workloads.make_box(700, seed=42, phi=0.1, radius=0.8, e=box.e, dt=box.dt)]
    boxes = [others[0], box, others[1]]
    off = np.cumsum([0] + [b.n for b in boxes]).astype(np.int64)
    cat = lambda f: torch.as_tensor(np.concatenate([getattr(b, f) for b in boxes])).cuda()
    p = pc.Particles(*[cat(f) for f in ("x", "y", "z", "vx", "vy", "vz", "r", "m")])
    n = p.n
    ctx = pc.Context(n, pc.pcol_default_opts(autotune=0))
    partner = torch.empty(n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(n, dtype=torch.float64, device="cuda")
    _announce("edge box in the batched form")
    pc.pcol_step_batched(ctx, p, off, [b.L for b in boxes], box.dt, box.e, partner, tcoll)
    torch.cuda.synchronize()
    part = partner.cpu().numpy().astype(np.int64)
    tc = tcoll.cpu().numpy()
    st = to_host(p)
    for b, bx in enumerate(boxes):
        lo, hi = int(off[b]), int(off[b + 1])
        ref = orc if bx is box else oracle.step(bx)
        local = np.where(part[lo:hi] >= 0, part[lo:hi] - lo, -1)
        gpu = ({f: st[f][lo:hi] for f in FIELDS}, local, tc[lo:hi], None)
        assert compare_step(bx, gpu, ref) == 0, f"box {b}"
    _check_designed(groups, np.where(part[off[1]:off[2]] >= 0, part[off[1]:off[2]] - off[1], -1),
                    tc[off[1]:off[2]])


def test_kinetic_energy_run_in_lockstep_with_oracle():
    """The paper's kinetic-energy run (5,000 spheres, d = 0.02, side 2, |v| = 1, e = 1)
    for 1,000 steps of dt = 0.0764 (about 2e5 collisions, the paper's count): every
    GPU step equals the oracle's step from the same state bitwise, the kinetic energy
    is preserved to 1e-13 relative, and the velocity components end normal with
    variance 1/3 (Kolmogorov-Smirnov)."""
    from scipy import stats
    n, L = 5000, 2.0
    dirs = workloads.normals(42, 9, 3 * n).reshape(n, 3)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    xs, ys, zs = workloads.rsa_positions(42, np.full(n, 0.01), (L, L, L))
    box = workloads.Box(xs, ys, zs, dirs[:, 0].copy(), dirs[:, 1].copy(), dirs[:, 2].copy(),
                        np.full(n, 0.01), np.ones(n), (L, L, L), 0.0764, 1.0)
    ke = lambda b: 0.5 * math.fsum(b.vx ** 2 + b.vy ** 2 + b.vz ** 2)
    ke0 = ke(box)
    p = pc.Particles.from_box(box)
    ctx = pc.Context(n)
    partner = torch.empty(n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(n, dtype=torch.float64, device="cuda")
    total = 0
    for step in range(1000):
        st = pc.pcol_step(ctx, p, box.L, box.dt, 1.0, partner, tcoll)
        torch.cuda.synchronize()
        ref = oracle.step(box)
        out = to_host(p)
        assert np.array_equal(partner.cpu().numpy().astype(np.int64), ref.partner), step
        assert np.array_equal(tcoll.cpu().numpy(), ref.tcoll, equal_nan=True), step
        for f in FIELDS:
            assert np.array_equal(out[f].view(np.uint64), getattr(ref, f).view(np.uint64)), (step, f)
        assert st["n_pairs"] == ref.n_pairs
        total += ref.n_pairs
        box = workloads.Box(ref.x, ref.y, ref.z, ref.vx, ref.vy, ref.vz, box.r, box.m, box.L,
                            box.dt, 1.0)
        if step % 250 == 249:
            _announce(f"kinetic-energy run: step {step + 1}, {total} collisions")
    assert abs(ke(box) - ke0) / ke0 < 1e-13
    comps = np.concatenate([box.vx, box.vy, box.vz])
    assert stats.kstest(comps, "norm", args=(0, math.sqrt(1 / 3))).pvalue > 1e-3
    assert 1e5 < total < 4e5
