"""Pins of the oracle's step with reflective walls (oracle.step_walls), CPU only.

Sec. "Intersection of Particles with Solid Walls" treats a wall contact a
posteriori with a perfectly reflective (elastic) wall: the normal velocity
component changes sign.  Sec. "Particle Collisions" accepts a particle pair's
collision only if it happens before either particle's next boundary
intersection.  The particle is tracked by its centre.  Pins: with no wall the
periodic step bitwise; closed forms of a reflection, of a pair that would meet
through a periodic boundary, and of a collision rejected because one sphere
reaches the wall first; an independent pure-Python brute force (bisection
contact times); energy conservation at e = 1 between walls; momentum along the
periodic axes; storage-permutation invariance."""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import indep_bruteforce as bf

FIELDS = ("x", "y", "z", "vx", "vy", "vz")


def _box(pos, vel, r=0.5, L=(10.0, 10.0, 10.0), dt=0.5, e=1.0):
    pos, vel = np.asarray(pos, float), np.asarray(vel, float)
    n = len(pos)
    return workloads.Box(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), vel[:, 0].copy(),
                         vel[:, 1].copy(), vel[:, 2].copy(), np.full(n, r), np.ones(n), tuple(L),
                         dt, e)


@pytest.mark.parametrize("k", [1, 2])
def test_no_wall_is_the_periodic_step_bitwise(k):
    box = workloads.config(1) if k == 1 else workloads.config(2, n=20_000)
    a, b = oracle.step(box), oracle.step_walls(box, (0, 0, 0))
    assert a.n_pairs == b.n_pairs and np.array_equal(a.partner, b.partner)
    assert np.array_equal(a.tcoll, b.tcoll, equal_nan=True)
    for f in FIELDS:
        assert np.array_equal(getattr(a, f).view(np.uint64), getattr(b, f).view(np.uint64))


def test_reflection_closed_form():
    # x: 9.5 + 0.5 * 2 = 10.5 beyond the wall at 10 -> 9.5, vx -> -2; y periodic wraps
    box = _box([[9.5, 9.75, 5.0], [0.25, 5.0, 5.0]], [[2.0, 1.0, 0.0], [-1.0, 0.0, 0.0]],
               L=(10.0, 10.0, 10.0))
    res = oracle.step_walls(box, (1, 0, 0))
    assert res.n_pairs == 0
    assert (res.x[0], res.vx[0], res.y[0]) == (9.5, -2.0, 0.25)
    assert (res.x[1], res.vx[1]) == (0.25, 1.0)           # 0.25 - 0.5 -> |-0.25|
    per = oracle.step(box)
    assert (per.x[0], per.vx[0]) == (0.5, 2.0)             # the periodic step wraps instead


def test_no_collision_through_a_wall():
    # 1.6 apart through the periodic boundary, closing at 4: the periodic step pairs
    # them at t = 0.15; between walls they are 8.4 apart and each reflects
    box = _box([[0.8, 5.0, 5.0], [9.2, 5.0, 5.0]], [[-2.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    per = oracle.step(box)
    assert per.n_pairs == 1 and per.tcoll[0] == pytest.approx(0.15, rel=1e-15)
    res = oracle.step_walls(box, (1, 0, 0))
    assert res.n_pairs == 0
    assert res.x[0] == pytest.approx(0.2, abs=1e-15) and res.vx[0] == 2.0
    assert res.x[1] == pytest.approx(9.8, abs=1e-15) and res.vx[1] == -2.0


def test_collision_after_a_wall_intersection_is_rejected():
    # A reaches the wall at t = 0.3 / 4 = 0.075; B would touch A at t = 0.125
    box = _box([[0.3, 5.0, 5.0], [1.8, 5.0, 5.0]], [[-4.0, 0.0, 0.0], [-8.0, 0.0, 0.0]],
               L=(40.0, 40.0, 40.0))
    per = oracle.step(box)
    assert per.n_pairs == 1 and per.tcoll[0] == 0.125
    res = oracle.step_walls(box, (1, 0, 0))
    assert res.n_pairs == 0
    assert (res.x[0], res.vx[0]) == (1.7, 4.0) and (res.x[1], res.vx[1]) == (2.2, 8.0)
    # with A slower, so that it meets B before the wall, the pair is kept
    box.vx[0] = -1.0   # time of flight 0.3; contact at 0.5 / 7 < 0.3
    res = oracle.step_walls(box, (1, 0, 0))
    assert res.n_pairs == 1 and res.tcoll[0] == pytest.approx(0.5 / 7, rel=1e-15)


def _tof(x, v, L, walls):
    tw = math.inf
    for k in range(3):
        if walls[k] and v[k] != 0.0:
            tw = min(tw, (L[k] - x[k]) / v[k] if v[k] > 0 else -x[k] / v[k])
    return tw


def _bruteforce_walls(box, walls):
    """All-pairs sweeps with bisection contact times (no minimum image across a wall)
    and the time-of-flight condition; returns {(i, j): t}."""
    n = box.n
    Leff = [math.inf if walls[k] else box.L[k] for k in range(3)]
    x = list(zip(box.x, box.y, box.z))
    v = list(zip(box.vx, box.vy, box.vz))
    tof = [_tof(x[i], v[i], box.L, walls) for i in range(n)]
    active, pairs = [True] * n, {}
    while True:
        best = [None] * n
        for i in range(n):
            if not active[i]:
                continue
            for j in range(n):
                if j == i or not active[j]:
                    continue
                t = bf.contact_time(x[i], v[i], box.r[i], x[j], v[j], box.r[j], Leff, box.dt)
                if t is None or t > tof[i] or t > tof[j]:
                    continue
                if best[i] is None or (t, j) < best[i]:
                    best[i] = (t, j)
        found = [(i, best[i][1], best[i][0]) for i in range(n) if best[i] is not None
                 and best[i][1] > i and best[best[i][1]] is not None and best[best[i][1]][1] == i]
        if not found:
            return pairs
        for i, j, t in found:
            pairs[(i, j)] = t
            active[i] = active[j] = False


@pytest.mark.parametrize("seed,walls", [(1, (1, 1, 1)), (2, (1, 0, 0)), (3, (0, 1, 1)),
                                         (4, (1, 1, 1))])
def test_matches_independent_bruteforce(seed, walls):
    box = workloads.make_box(300, seed=seed, phi=0.25, radius=0.5, e=0.85, dt=0.25)
    res = oracle.step_walls(box, walls)
    ref = _bruteforce_walls(box, walls)
    got = {(i, int(res.partner[i])): res.tcoll[i] for i in range(box.n) if res.partner[i] > i}
    assert set(got) == set(ref) and len(ref) > 20
    for key in ref:
        assert got[key] == pytest.approx(ref[key], rel=1e-9)
    # the walls change the pair set of this box
    per = oracle.step(box)
    assert {(i, int(per.partner[i])) for i in range(box.n) if per.partner[i] > i} != set(ref)


def test_energy_between_elastic_walls_and_momentum_along_periodic_axes():
    box = workloads.make_box(3000, seed=9, phi=0.2, radius=0.5, e=1.0, dt=0.25)
    m = box.m
    ke = lambda b: 0.5 * math.fsum(m * (b.vx ** 2 + b.vy ** 2 + b.vz ** 2))
    py = lambda b: math.fsum(m * b.vy)
    k0, p0 = ke(box), py(box)
    b = box.copy()
    reflected = 0
    for _ in range(40):
        r = oracle.step_walls(b, (1, 0, 1))
        free = r.partner < 0
        reflected += int(np.count_nonzero(r.vx[free] == -b.vx[free]))
        b.x, b.y, b.z, b.vx, b.vy, b.vz = r.x, r.y, r.z, r.vx, r.vy, r.vz
        for f, a in (("x", 0), ("y", 1), ("z", 2)):
            c = getattr(b, f)
            assert np.all(c >= 0.0) and np.all(c < box.L[a])
    assert reflected > 100
    assert ke(b) == pytest.approx(k0, rel=1e-12)
    assert py(b) == pytest.approx(p0, abs=1e-9 * math.fsum(m * np.abs(box.vy)))


def test_storage_permutation_invariance():
    box = workloads.make_box(2000, seed=5, phi=0.3, radius=0.5, e=0.8, dt=0.25)
    res = oracle.step_walls(box, (1, 1, 0))
    perm = np.random.default_rng(3).permutation(box.n)
    inv = np.argsort(perm)
    pb = workloads.Box(*[a[perm].copy() for a in box.arrays()], box.L, box.dt, box.e)
    rp = oracle.step_walls(pb, (1, 1, 0))
    assert np.array_equal(np.where(rp.partner[inv] >= 0, perm[rp.partner[inv]], -1), res.partner)
    for f in FIELDS:
        assert np.array_equal(getattr(rp, f)[inv], getattr(res, f))


def _spins(n, seed, scale=3.0):
    return np.random.default_rng(seed).normal(size=(3, n)) * scale


def test_walls_with_spin_reduce_to_each_part_bitwise():
    box = workloads.make_box(3000, seed=6, phi=0.25, radius=0.5, e=0.8, dt=0.25)
    w = _spins(box.n, 2)
    # no wall: the periodic friction step
    a, b = oracle.step_spin(box, w, 0.4), oracle.step_walls_spin(box, (0, 0, 0), w, 0.4)
    assert np.array_equal(a.partner, b.partner)
    for f in FIELDS + ("wx", "wy", "wz"):
        assert np.array_equal(getattr(a, f).view(np.uint64), getattr(b, f).view(np.uint64)), f
    # no friction: the frictionless walls step, spins unchanged
    c, d = oracle.step_walls(box, (1, 0, 1)), oracle.step_walls_spin(box, (1, 0, 1), w, 0.0)
    assert np.array_equal(c.partner, d.partner) and c.n_pairs > 50
    for f in FIELDS:
        assert np.array_equal(getattr(c, f).view(np.uint64), getattr(d, f).view(np.uint64)), f
    for k, f in enumerate(("wx", "wy", "wz")):
        assert np.array_equal(getattr(d, f), w[k])


def test_walls_with_friction_pairs_and_reflections():
    box = workloads.make_box(3000, seed=7, phi=0.25, radius=0.5, e=0.8, dt=0.25)
    w = _spins(box.n, 3)
    walls = (1, 1, 0)
    res = oracle.step_walls_spin(box, walls, w, 0.5)
    plain = oracle.step_walls(box, walls)
    assert np.array_equal(res.partner, plain.partner)           # spins do not move contacts
    free = res.partner < 0
    for k, f in enumerate(("wx", "wy", "wz")):                    # walls leave spins alone
        assert np.array_equal(getattr(res, f)[free], w[k][free])
    # free spheres between walls move exactly as without friction (reflections included)
    for f in FIELDS:
        assert np.array_equal(getattr(res, f)[free], getattr(plain, f)[free])
    hit = ~free
    assert np.count_nonzero(res.wx[hit] != w[0][hit]) > 0.9 * hit.sum()
