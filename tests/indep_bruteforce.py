"""An independent brute-force statement of one collision step for tiny inputs.

Pure Python, all pairs, and a different way of finding contact times from the
one the oracle uses: the spheres touch when the distance |d + tau u| first falls
to the sum of radii.  Here that is decided geometrically (closest approach
within the step) and the time is found by bisection on the squared distance,
not by the closed-form root.  It follows the same rule as the paper's operator
(Sec. "Collision Operator": one collision per sphere per step, collided spheres
leave the eligible set; the earliest partner wins, ties to the smaller index).

Used only to pin the oracle on small inputs; agreement is up to the rounding
of the two root finders (relative 1e-12 on times, exact on pair sets).
"""
from __future__ import annotations

import math


def _sep(a, b, L):
    d = b - a
    if d > 0.5 * L:
        d -= L
    elif d < -0.5 * L:
        d += L
    return d


def contact_time(xi, vi, ri, xj, vj, rj, L, dt):
    d = [_sep(xi[k], xj[k], L[k]) for k in range(3)]
    u = [vj[k] - vi[k] for k in range(3)]
    s = ri + rj
    dist2 = lambda tau: sum((d[k] + tau * u[k]) ** 2 for k in range(3))
    if dist2(0.0) <= s * s:
        return None                       # touching or overlapping now: no collision
    uu = sum(x * x for x in u)
    du = sum(d[k] * u[k] for k in range(3))
    if uu == 0.0 or du >= 0.0:
        return None                       # not approaching
    tstar = -du / uu                      # time of closest approach
    hi = min(tstar, dt)
    if dist2(hi) > s * s:
        return None                       # never within s during [0, dt]
    lo = 0.0                              # dist2(lo) > s^2 >= dist2(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if dist2(mid) > s * s:
            lo = mid
        else:
            hi = mid
    return hi


def step(x, v, r, m, L, dt, e):
    """Pair set {(i, j): t} of one step by the sweep rule, all pairs, tiny N only."""
    n = len(x)
    active = [True] * n
    pairs = {}
    while True:
        best = [None] * n
        for i in range(n):
            if not active[i]:
                continue
            for j in range(n):
                if j == i or not active[j]:
                    continue
                t = contact_time(x[i], v[i], r[i], x[j], v[j], r[j], L, dt)
                if t is None:
                    continue
                if best[i] is None or (t, j) < best[i]:
                    best[i] = (t, j)
        found = []
        for i in range(n):
            if best[i] is None:
                continue
            t, j = best[i]
            if j > i and best[j] is not None and best[j][1] == i:
                found.append((i, j, t))
        if not found:
            return pairs
        for i, j, t in found:
            pairs[(i, j)] = t
            active[i] = active[j] = False


def earliest(box, active=None):
    """Earliest partner (index or -1) and contact time (inf if none) of every active
    sphere of a workloads.Box over the active set, all pairs, tiny N only."""
    n = box.n
    x = [(float(box.x[i]), float(box.y[i]), float(box.z[i])) for i in range(n)]
    v = [(float(box.vx[i]), float(box.vy[i]), float(box.vz[i])) for i in range(n)]
    act = [True] * n if active is None else [bool(a) for a in active]
    partner, tmin = [-1] * n, [math.inf] * n
    for i in range(n):
        if not act[i]:
            continue
        best = None
        for j in range(n):
            if j == i or not act[j]:
                continue
            t = contact_time(x[i], v[i], box.r[i], x[j], v[j], box.r[j], box.L, box.dt)
            if t is not None and (best is None or (t, j) < best):
                best = (t, j)
        if best is not None:
            tmin[i], partner[i] = best
    import numpy as np
    return np.array(partner, dtype=np.int64), np.array(tmin)


def kinetic_energy(m, vx, vy, vz):
    return 0.5 * math.fsum(m[i] * (vx[i] ** 2 + vy[i] ** 2 + vz[i] ** 2) for i in range(len(m)))
