"""Constructed inputs at the edges of the contact rule (Sec. "Particle Collisions",
eq. (detect1/detect2): two positive roots, the lower one within the step, the spheres
approaching), embedded in a dense polydisperse box so that they go through the same
grid, filters, split and sweeps as any other sphere.

The box side is 96 and the step dt = 0.5, so the designed coordinates (integers plus
a few binary fractions) and contact times are exact in binary64.  A slab around
z = 48 is cleared of the random spheres and the designed groups sit in the plane
z = 48 on a lattice of 12 x 12 sites, each group within 2.5 of its site in x (the
groups across the periodic face within 4.25), so no sphere of one group can reach a
sphere of another group or a random sphere within the step.  This module only builds
inputs and names the designed outcomes; the oracle decides every result.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

import workloads

L_SIDE = 96.0
DT = 0.5
Z0 = 48.0
SLAB = 9.0     # random spheres with |z - Z0| < SLAB are removed


@dataclass
class Sphere:
    x: float
    y: float
    z: float
    vx: float
    vy: float
    vz: float
    r: float


@dataclass
class Group:
    name: str
    spheres: list
    first: int = -1                  # index of the group's first sphere in the box
    expect: dict = field(default_factory=dict)


def _pair(name, xi, vi, ri, xj, vj, rj, **expect):
    return Group(name, [Sphere(*xi, *vi, ri), Sphere(*xj, *vj, rj)], expect=expect)


def _interior_groups():
    """Groups placed around a site at the origin (shifted to their site later)."""
    g = []
    s2 = 0.625  # radius of the equal-sphere pairs (s = 1.25)
    # the contact time is exactly dt: d = (2, 0.75, 0), u = (-2, 0, 0), s = 1.25
    g.append(_pair("t_eq_dt", (-1, 0, 0), (1, 0, 0), s2, (1, 0.75, 0), (-1, 0, 0), s2,
                   t=0.5))
    # tangent contact, D = 0: d = (1, 1.25, 0), u = (-4, 0, 0): t = 1/4
    g.append(_pair("tangent", (-0.5, 0, 0), (2, 0, 0), s2, (0.5, 1.25, 0), (-2, 0, 0), s2,
                   t=0.25))
    # touching now (c = 0) and approaching: no collision
    g.append(_pair("touching", (-0.625, 0, 0), (1, 0, 0), s2, (0.625, 0, 0), (-1, 0, 0), s2,
                   t=None))
    # overlapping (c < 0) and approaching: no collision
    g.append(_pair("overlap", (-0.5, 0, 0), (1, 0, 0), s2, (0.5, 0, 0), (-1, 0, 0), s2, t=None))
    # b = 0: moving perpendicular to the separation
    g.append(_pair("b_zero", (-1, 0, 0), (0, 1, 0), s2, (1, 0, 0), (0, -1, 0), s2, t=None))
    # a = 0: equal velocities
    v = (0.75, -0.5, 0.25)
    g.append(_pair("a_zero", (-1, 0, 0), v, s2, (0.75, 0, 0), v, s2, t=None))
    # grazing: lateral offset rho = s (1 + eta), d = (1, rho, 0), u = (-2, 0, 0); the
    # contact, if any, is at (1 - sqrt(s^2 - rho^2)) / 2 <= dt
    s = 2 * s2
    for eta in (-1e-4, -1e-8, -1e-12, -1e-15, -2.0 ** -52, 0.0, 2.0 ** -52, 1e-15, 1e-12,
                1e-8, 5e-5, 1e-4, 1.34e-4, 2e-4, 1e-3):
        rho = s * (1.0 + eta)
        g.append(_pair(f"graze{eta:+.3g}", (-0.5, 0, 0), (1, 0, 0), s2, (0.5, rho, 0), (-1, 0, 0),
                       s2, t="graze"))
    # slow head-on approach from a gap s delta, closing speed w = s delta / (kappa dt)
    # (contact at about kappa dt), both spheres also carried by a common velocity
    frame = (1.3, -1.1, 0.7)
    for delta in (1e-9, 1e-7, 1e-5, 1e-3):
        for kappa in (1 - 1e-3, 1 - 1e-7, 1 - 1e-11, 1.0, 1 + 1e-11, 1 + 1e-7):
            gap = s * (1.0 + delta)
            w = s * delta / (kappa * DT)
            g.append(_pair(f"slow{delta:.0e}k{kappa:.12g}", (-gap / 2, 0, 0),
                           (frame[0] + w / 2, frame[1], frame[2]), s2, (gap / 2, 0, 0),
                           (frame[0] - w / 2, frame[1], frame[2]), s2, t="slow"))
    # exact tie: k at rest between two spheres closing at speed 2 from distance 2
    # (s = 0.5 + 0.75, t = (2.4375) / (4 + 2.5) = 0.375 for both), both index orders
    for order in ("ab", "ba"):
        k = Sphere(0, 0, 0, 0, 0, 0, 0.5)
        a = Sphere(-2, 0, 0, 2, 0, 0, 0.75)
        b = Sphere(2, 0, 0, -2, 0, 0, 0.75)
        sp = [k, a, b] if order == "ab" else [k, b, a]
        g.append(Group(f"tie_{order}", sp, expect={"t": 0.375, "tie": True}))
    return g


def _face_groups():
    """Groups across the periodic face x = 0 (site x = 0; coordinates below 0 wrap to
    L - ...)."""
    g = []
    for order in ("ab", "ba"):
        # both partners in the first layer: k at x = 1, a at x = 95 (separation -2 through
        # the face), b at x = 3
        k = Sphere(1, 0, 0, 0, 0, 0, 0.5)
        a = Sphere(-1, 0, 0, 2, 0, 0, 0.75)
        b = Sphere(3, 0, 0, -2, 0, 0, 0.75)
        sp = [k, a, b] if order == "ab" else [k, b, a]
        g.append(Group(f"face_tie_{order}", sp, expect={"t": 0.375, "tie": True}))
        # b large (radius 2, extent 3: above the split extent at quantile 0.9): the two
        # contacts come from the half-stencil search and the wide-sphere search; with
        # s = 2.5, d = 3.25, u = -2: t = 4.3125 / (6.5 + 5) = 0.375
        k, a = Sphere(1, 0, 0, 0, 0, 0, 0.5), Sphere(-1, 0, 0, 2, 0, 0, 0.75)
        b2 = Sphere(4.25, 0, 0, -2, 0, 0, 2.0)
        sp = [k, a, b2] if order == "ab" else [k, b2, a]
        g.append(Group(f"split_tie_{order}", sp, expect={"t": 0.375, "tie": True, "wide": 2.0}))
    # a sphere at x = 0 exactly and one just below L, each with a partner through the face
    g.append(_pair("at_zero", (0, 0, 0), (-1, 0, 0), 0.625, (-2, 0, 0), (1, 0, 0), 0.625,
                   t=0.375))
    below = -math.ulp(L_SIDE) / 2  # x = L - ulp/2 rounds to the largest double below L
    g.append(_pair("below_L", (below, 0, 0), (1, 0, 0), 0.625, (1.75, 0, 0), (-1, 0, 0), 0.625,
                   t="wrap"))
    # lone spheres crossing the face in free flight
    g.append(Group("lone_zero", [Sphere(0, 0, 0, -1.5, 0.5, 0, 0.8)], expect={"t": None}))
    g.append(Group("lone_below_L", [Sphere(below, 0, 0, 1.5, 0, -0.5, 0.8)], expect={"t": None}))
    return g


def _wrap(v):
    v = float(v)
    if v < 0.0:
        v = v + L_SIDE
        if v >= L_SIDE:
            v = math.nextafter(L_SIDE, 0.0)
    return v


def edge_box(seed: int = 31, e: float = 0.8, dt: float = DT):
    """The edge-case box and its designed groups (with each group's first index)."""
    base = workloads.make_box(48_000, seed=seed, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=e,
                              dt=dt, L=L_SIDE)
    keep = np.abs(base.z - Z0) >= SLAB
    arrs = [a[keep] for a in base.arrays()]
    groups = []
    interior = _interior_groups()
    face = _face_groups()
    sites = []
    for m in range(8):
        for k in range(8):
            if m < len(face) and k in (0, 7):
                continue
            sites.append((6.0 + 12.0 * k, 6.0 + 12.0 * m))
    assert len(interior) <= len(sites)
    for grp, (sx, sy) in zip(interior, sites):
        for sp in grp.spheres:
            sp.x, sp.y, sp.z = sx + sp.x, sy + sp.y, Z0 + sp.z
        groups.append(grp)
    for m, grp in enumerate(face):
        for sp in grp.spheres:
            sp.x, sp.y, sp.z = _wrap(sp.x), 6.0 + 12.0 * m + sp.y, Z0 + sp.z
        groups.append(grp)
    des = [sp for grp in groups for sp in grp.spheres]
    half = arrs[0].shape[0] // 2
    cols = list(zip(*[(sp.x, sp.y, sp.z, sp.vx, sp.vy, sp.vz, sp.r) for sp in des]))
    dr = np.array(cols[6])
    dsgn = [np.array(c, dtype=np.float64) for c in cols[:6]] + [dr, dr ** 3]
    out = [np.concatenate([a[:half], d, a[half:]]) for a, d in zip(arrs, dsgn)]
    at = half
    for grp in groups:
        grp.first = at
        at += len(grp.spheres)
    box = workloads.Box(*out, (L_SIDE, L_SIDE, L_SIDE), float(dt), float(e), "edge96")
    for a in range(3):
        p = box.arrays()[a]
        assert np.all(p >= 0.0) and np.all(p < L_SIDE)
    return box, groups


def check_designed(groups, partner, tcoll, dt=DT):
    """The designed outcome of every group whose outcome the construction fixes."""
    for g in groups:
        idx = g.first + np.arange(len(g.spheres))
        t = g.expect.get("t")
        if g.expect.get("tie"):
            k, first, second = idx
            # exact tie: k takes the smaller index, the other is left without a partner
            assert partner[k] == first and partner[first] == k, g.name
            assert partner[second] == -1, g.name
            assert tcoll[k] == g.expect["t"], g.name
        elif t is None:
            assert np.all(partner[idx] == -1), g.name
        elif isinstance(t, float):
            i, j = idx
            if t <= dt:
                assert partner[i] == j and partner[j] == i, g.name
                assert tcoll[i] == t and tcoll[j] == t, g.name
            else:
                assert partner[i] == -1 and partner[j] == -1, g.name
    graze = [g for g in groups if g.expect.get("t") == "graze"]
    hit = [partner[g.first] == g.first + 1 for g in graze]
    assert any(hit) and not all(hit)  # the family straddles the contact distance
    slow = [g for g in groups if g.expect.get("t") == "slow"]
    hit = [partner[g.first] == g.first + 1 for g in slow]
    assert any(hit) and not all(hit)  # and the end of the step
