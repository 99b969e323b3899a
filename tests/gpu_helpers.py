"""Helpers shared by the GPU tests: run the HIP library on a workloads.Box and
compare its results with the oracle's element by element."""
from __future__ import annotations

import numpy as np
import torch

import paper_2501_05340_amd as pc

FIELDS = ("x", "y", "z", "vx", "vy", "vz")


def to_host(p: "pc.Particles") -> dict:
    return {f: getattr(p, f).cpu().numpy() for f in FIELDS}


def gpu_step(box, ctx=None, **opts):
    """One pcol_step of box on cuda:0; returns (state dict, partner, tcoll, stats)."""
    p = pc.Particles.from_box(box)
    if ctx is None:
        ctx = pc.Context(max(box.n, 1), pc.pcol_default_opts(**opts) if opts else None)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll)
    torch.cuda.synchronize()
    out = to_host(p)
    return out, partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st


def compare_step(box, gpu, orc, rel=1e-12):
    """Pair set bit-exact; contact times bitwise; states within rel (relative to the
    magnitude scale of each field).  Returns the count of non-bitwise state values."""
    out, partner, tcoll, _ = gpu
    assert np.array_equal(partner, orc.partner), (
        f"pair set differs at {np.count_nonzero(partner != orc.partner)} spheres")
    assert np.array_equal(tcoll, orc.tcoll, equal_nan=True), "contact times differ"
    nonbit = 0
    for f in FIELDS:
        a, b = out[f], getattr(orc, f)
        scale = max(1.0, float(np.max(np.abs(b)))) if b.size else 1.0
        err = np.max(np.abs(a - b)) / scale if a.size else 0.0
        assert err <= rel, f"{f}: max relative error {err:.3e}"
        nonbit += int(np.count_nonzero(a.view(np.uint64) != b.view(np.uint64)))
    return nonbit


def box_slice(box, n):
    """First n spheres of a box (a valid box: spheres never overlap)."""
    from workloads import Box
    return Box(*[a[:n].copy() for a in box.arrays()], box.L, box.dt, box.e, box.name + f"[:{n}]")
