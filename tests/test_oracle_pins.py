"""Pins of the FP64 oracle against the paper and the mathematics (CPU only).

Each test fixes the oracle against something other than itself: closed-form
contact times and textbook restitution results, the paper's two-sphere case
(Sec. "Validation", "Simple Particle Collision"), an independent brute force
on tiny inputs (tests/indep_bruteforce.py), conservation laws, the kinetic
energy analogy run (Sec. "Kinetic Energy Analogy and Preservation"), and the
geometric closest-approach test for collision existence.
"""
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
import workloads
from tests import indep_bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def two_box(xi, vi, ri, xj, vj, rj, L=(10.0, 10.0, 10.0), dt=1.0, e=1.0, mi=1.0, mj=1.0):
    a = lambda *v: np.array(v, dtype=np.float64)
    return workloads.Box(a(xi[0], xj[0]), a(xi[1], xj[1]), a(xi[2], xj[2]), a(vi[0], vj[0]),
                         a(vi[1], vj[1]), a(vi[2], vj[2]), a(ri, rj), a(mi, mj), tuple(L), dt, e)


# ---------------------------------------------------------------- pair time


def test_head_on_closed_form():
    # separation 3, radii 0.5 + 0.5, closing speed 1: contact at (3 - 1) / 1 = 2 exactly
    t = oracle.pair_time([1, 2, 2], [0.5, 0, 0], 0.5, [4, 2, 2], [-0.5, 0, 0], 0.5, [10] * 3, 3.0)
    assert t == 2.0


def test_oblique_pythagorean_exact():
    # s = 1.25, lateral offset 0.75 -> along-line gap at contact sqrt(s^2 - b^2) = 1;
    # closing 3 -> 1 at relative speed 2 takes exactly 1.0
    t = oracle.pair_time([1, 1, 1], [1, 0, 0], 0.625, [4, 1.75, 1], [-1, 0, 0], 0.625, [10] * 3, 2.0)
    assert t == 1.0


def test_tangent_contact_counts():
    # lateral offset equal to s: the quadratic has a double root (D = 0) at t = 1.5
    t = oracle.pair_time([1, 1, 1], [1, 0, 0], 0.625, [4, 2.25, 1], [-1, 0, 0], 0.625, [10] * 3, 2.0)
    assert t == 1.5


def test_contact_exactly_at_dt_counts_and_later_does_not():
    args = ([1, 1, 1], [1, 0, 0], 0.625, [4, 1.75, 1], [-1, 0, 0], 0.625, [10] * 3)
    assert oracle.pair_time(*args, 1.0) == 1.0
    assert oracle.pair_time(*args, np.nextafter(1.0, 0.0)) is None


@pytest.mark.parametrize("case", ["same_velocity", "receding", "perpendicular", "overlap",
                                  "touching", "miss"])
def test_no_collision_cases(case):
    xi, vi, xj, vj, r = [1, 1, 1], [1, 0, 0], [4, 1, 1], [-1, 0, 0], 0.5
    if case == "same_velocity":        # a = 0
        vj = [1, 0, 0]
    elif case == "receding":           # b > 0
        vi, vj = [-1, 0, 0], [1, 0, 0]
    elif case == "perpendicular":      # b = 0
        vi, vj = [0, 1, 0], [0, -1, 0]
    elif case == "overlap":            # c < 0
        xj = [1.5, 1, 1]
    elif case == "touching":           # c = 0: already in contact, no new collision
        xj = [2.0, 1, 1]
    elif case == "miss":               # D < 0
        xj = [4, 2.5, 1]
    assert oracle.pair_time(xi, vi, r, xj, vj, r, [10] * 3, 100.0) is None


def test_pair_time_is_symmetric_bitwise():
    rng = np.random.default_rng(7)
    L = np.array([7.0, 8.0, 9.0])
    hits = 0
    for _ in range(4000):
        xi, xj = rng.uniform(0, 1, 3) * L, rng.uniform(0, 1, 3) * L
        xj = xi + rng.normal(0, 0.8, 3)
        xj = np.mod(xj, L)
        vi, vj = rng.normal(0, 1, 3), rng.normal(0, 1, 3)
        ri, rj = rng.uniform(0.1, 0.4, 2)
        t1 = oracle.pair_time(xi, vi, ri, xj, vj, rj, L, 2.0)
        t2 = oracle.pair_time(xj, vj, rj, xi, vi, ri, L, 2.0)
        assert (t1 is None) == (t2 is None)
        if t1 is not None:
            hits += 1
            assert t1 == t2
    assert hits > 100


def test_periodic_minimum_image_across_faces():
    # spheres on opposite faces of the box meet through the periodic boundary
    L = [10.0, 10.0, 10.0]
    t = oracle.pair_time([0.2, 5, 5], [-1, 0, 0], 0.25, [9.6, 5, 5], [1, 0, 0], 0.25, L, 1.0)
    # gap through the boundary 0.6 - 0.5 = 0.1 at closing speed 2
    assert t == pytest.approx(0.05, rel=1e-14)


def test_existence_matches_closest_approach_geometry():
    """Collision exists iff the closest approach within [0, dt] reaches s (spheres apart and
    approaching) -- an independent geometric criterion, vectorised in numpy."""
    rng = np.random.default_rng(11)
    n = 20000
    L = np.array([50.0, 50.0, 50.0])
    d = rng.normal(0, 1.2, (n, 3))
    u = rng.normal(0, 1.0, (n, 3))
    s = rng.uniform(0.5, 1.5, n)
    dt = 0.7
    tt = np.full(n, np.nan)
    for k in range(n):
        xi = np.array([25.0, 25.0, 25.0])
        t = oracle.pair_time(xi, [0, 0, 0], 0.5 * s[k], xi + d[k], u[k], 0.5 * s[k], L, dt)
        if t is not None:
            tt[k] = t
    c0 = (d * d).sum(1) - s * s
    du = (d * u).sum(1)
    uu = (u * u).sum(1)
    tau = np.clip(-du / uu, 0.0, dt)
    dmin2 = ((d + tau[:, None] * u) ** 2).sum(1)
    geo = (c0 > 0) & (du < 0) & (dmin2 <= s * s)
    margin = np.abs(dmin2 - s * s) > 1e-9 * s * s
    got = ~np.isnan(tt)
    assert np.array_equal(got[margin], geo[margin])
    assert got.sum() > 500
    # the returned time is a root: |d + t u| = s to rounding
    k = np.where(got)[0]
    res = np.sqrt(((d[k] + tt[k, None] * u[k]) ** 2).sum(1)) / s[k] - 1.0
    assert np.max(np.abs(res)) < 1e-9


# ---------------------------------------------------------------- the paper's two-sphere case


def test_two_sphere_periodic_case_from_paper():
    g = json.load(open(os.path.join(GOLDEN, "two_sphere_periodic.json")))
    lo = np.array(g["box_lo"])
    L = tuple(np.array(g["box_hi"]) - lo)
    r = 0.5 * g["diameter"]
    dt = 1e-3
    box = two_box(np.array(g["x1"]) - lo, g["v1"], r, np.array(g["x2"]) - lo, g["v2"], r, L=L,
                  dt=dt, e=g["restitution"])
    getcontext().prec = 50
    t_exact = (Decimal("1.2") - (Decimal("0.04") ** 2 - Decimal("0.037") ** 2).sqrt()) / 30
    hit_step = None
    for k in range(60):
        res = oracle.step(box)
        if res.n_pairs:
            hit_step = k
            t_num = k * dt + res.tcoll[0]
            break
        box = workloads.Box(res.x, res.y, res.z, res.vx, res.vy, res.vz, box.r, box.m, L, dt, 1.0)
    assert hit_step == 39            # the 40th step, after the y-wrap
    assert abs(t_num - float(t_exact)) / float(t_exact) < 1e-13
    # elastic, equal masses: the normal velocity components are exchanged; momentum is zero
    assert res.vy[0] + res.vy[1] == pytest.approx(0.0, abs=1e-13)
    ke0 = 0.5 * (15.0 ** 2) * 2
    ke1 = 0.5 * sum(v ** 2 for v in (res.vx[0], res.vy[0], res.vz[0], res.vx[1], res.vy[1], res.vz[1]))
    assert ke1 == pytest.approx(ke0, rel=1e-14)
    assert g["printed_t_coll"] != pytest.approx(float(t_exact), rel=1e-3)


# ---------------------------------------------------------------- resolve


@pytest.mark.parametrize("e", [0.0, 0.5, 0.9, 1.0])
@pytest.mark.parametrize("masses", [(1.0, 1.0), (1.0, 3.0), (2.5, 0.4)])
def test_head_on_textbook_restitution(e, masses):
    m1, m2 = masses
    box = two_box([1, 2, 2], [0.5, 0, 0], 0.5, [4, 2, 2], [-0.5, 0, 0], 0.5, dt=3.0, e=e, mi=m1, mj=m2)
    res = oracle.step(box)
    assert res.n_pairs == 1 and res.tcoll[0] == 2.0
    v1, v2 = 0.5, -0.5
    v1p = (m1 * v1 + m2 * v2 + m2 * e * (v2 - v1)) / (m1 + m2)
    v2p = (m1 * v1 + m2 * v2 + m1 * e * (v1 - v2)) / (m1 + m2)
    assert res.vx[0] == pytest.approx(v1p, abs=1e-15)
    assert res.vx[1] == pytest.approx(v2p, abs=1e-15)
    # moved to contact (t = 2), then the remaining 1.0 at the new velocity
    assert res.x[0] == pytest.approx(1 + 2 * v1 + 1.0 * v1p, abs=1e-15)
    assert res.x[1] == pytest.approx(4 + 2 * v2 + 1.0 * v2p, abs=1e-15)


@pytest.mark.parametrize("e", [0.3, 1.0])
def test_oblique_tangential_unchanged_normal_scaled(e):
    box = two_box([1, 1, 1], [1, 0, 0], 0.625, [4, 1.75, 1], [-1, 0, 0], 0.625, L=(20.0,) * 3, dt=2.0, e=e,
                  mi=1.0, mj=2.0)
    res = oracle.step(box)
    n = np.array([0.8, 0.6, 0.0])          # (d + t u) / s at t = 1
    u0 = np.array([-2.0, 0.0, 0.0])
    u1 = np.array([res.vx[1] - res.vx[0], res.vy[1] - res.vy[0], res.vz[1] - res.vz[0]])
    assert np.dot(u1, n) == pytest.approx(-e * np.dot(u0, n), abs=1e-14)
    tan0 = u0 - np.dot(u0, n) * n
    tan1 = u1 - np.dot(u1, n) * n
    assert np.allclose(tan1, tan0, atol=1e-14)
    p0 = np.array([1.0 * 1 + 2.0 * -1, 0, 0])
    p1 = np.array([res.vx[0] + 2 * res.vx[1], res.vy[0] + 2 * res.vy[1], res.vz[0] + 2 * res.vz[1]])
    assert np.allclose(p0, p1, atol=1e-14)


def _pair_state(box, i, j):
    x = np.array([box.x, box.y, box.z]).T
    v = np.array([box.vx, box.vy, box.vz]).T
    L = np.array(box.L)
    d = x[j] - x[i]
    d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
    return d, v[j] - v[i]


@pytest.mark.parametrize("e", [0.8, 1.0])
def test_config1_conservation_and_energy_loss_per_pair(e):
    box = workloads.config(1)
    res = oracle.step(box, e=e)
    m = box.m
    p0 = np.array([np.sum(m * box.vx), np.sum(m * box.vy), np.sum(m * box.vz)])
    p1 = np.array([np.sum(m * res.vx), np.sum(m * res.vy), np.sum(m * res.vz)])
    scale = np.sum(m * np.sqrt(box.vx ** 2 + box.vy ** 2 + box.vz ** 2))
    assert np.max(np.abs(p1 - p0)) < 1e-14 * scale
    ke = lambda vx, vy, vz: 0.5 * math.fsum(m * (vx ** 2 + vy ** 2 + vz ** 2))
    ke0, ke1 = ke(box.vx, box.vy, box.vz), ke(res.vx, res.vy, res.vz)
    # closed-form loss of each pair: (1 - e^2) / 2 * m_r * g^2, g the normal closing speed
    loss = 0.0
    for i in np.where(res.partner >= 0)[0]:
        j = res.partner[i]
        if j < i:
            continue
        d, u = _pair_state(box, i, j)
        w = d + res.tcoll[i] * u
        s = box.r[i] + box.r[j]
        g = np.dot(u, w) / s
        mr = m[i] * m[j] / (m[i] + m[j])
        loss += 0.5 * (1 - e * e) * mr * g * g
    assert res.n_pairs > 50
    assert (ke0 - ke1) == pytest.approx(loss, rel=1e-10, abs=1e-13 * ke0)


# ---------------------------------------------------------------- the sweep rule


def _tiny_box(seed, n=250, phi=0.3, mono=False):
    # dense enough for 3-4 sweeps, with dt small enough that 2 * reach < L
    if mono:
        return workloads.make_box(n, seed=seed, phi=phi, radius=0.5, e=0.85, dt=0.25)
    return workloads.make_box(n, seed=seed, phi=phi, lognormal=(0.5, 0.3, 0.25, 1.0), e=0.85,
                              dt=0.2)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_oracle_matches_independent_bruteforce(seed):
    box = _tiny_box(seed, mono=seed % 2 == 0)
    L = box.L
    res = oracle.step(box, grid=False)
    x = list(zip(box.x, box.y, box.z))
    v = list(zip(box.vx, box.vy, box.vz))
    ref = bf.step(x, v, list(box.r), list(box.m), L, box.dt, box.e)
    got = {(i, int(res.partner[i])): res.tcoll[i] for i in range(box.n)
           if res.partner[i] > i}
    assert set(got) == set(ref)
    for key in ref:
        assert got[key] == pytest.approx(ref[key], rel=1e-9)
    assert res.n_pairs == len(ref) and res.n_pairs > 50 and res.n_sweeps >= 3


@pytest.mark.parametrize("order", [(0, 1, 2), (1, 0, 2), (2, 1, 0), (0, 2, 1)])
def test_exact_tie_goes_to_smaller_index(order):
    """A sphere approached from both sides by mirror-image spheres has two contacts at
    bitwise-equal times; the earlier index wins, the loser flies on freely."""
    xs = {"c": [5.0, 5.0, 5.0], "l": [2.0, 5.0, 5.0], "r": [8.0, 5.0, 5.0]}
    vs = {"c": [0.0, 0.0, 0.0], "l": [1.0, 0.0, 0.0], "r": [-1.0, 0.0, 0.0]}
    names = ["c", "l", "r"]
    idx = {names[k]: order[k] for k in range(3)}
    arr = lambda src, k: np.array([src[nm][k] for nm in sorted(names, key=lambda q: idx[q])])
    box = workloads.Box(arr(xs, 0), arr(xs, 1), arr(xs, 2), arr(vs, 0), arr(vs, 1), arr(vs, 2),
                        np.full(3, 0.5), np.ones(3), (20.0, 20.0, 20.0), 3.0, 1.0)
    res = oracle.step(box)
    winner = min(idx["l"], idx["r"])
    loser = max(idx["l"], idx["r"])
    assert res.n_pairs == 1
    assert res.partner[idx["c"]] == winner and res.partner[loser] == -1
    assert res.tcoll[idx["c"]] == 2.0


def test_grid_equals_brute_force_and_is_cell_size_invariant():
    box = workloads.config(1)
    pb, tb, _ = oracle.earliest(box, grid=False)
    for mult in (1.0, 1.37, 2.0, 3.1):
        pg, tg, _ = oracle.earliest(box, grid=True, cell_mult=mult)
        assert np.array_equal(pb, pg) and np.array_equal(tb, tg)
    sb = oracle.step(box, grid=False)
    for mult in (1.0, 2.5):
        sg = oracle.step(box, grid=True, cell_mult=mult)
        for a, b in zip(sb.__dict__.values(), sg.__dict__.values()):
            if isinstance(a, np.ndarray):
                assert np.array_equal(a, b, equal_nan=True)


def test_sweep_invariants_config1():
    box = workloads.config(1)
    res = oracle.step(box)
    p = res.partner
    hit = p >= 0
    assert np.all(p[p[hit]] == np.where(hit)[0])          # symmetric, each sphere in <= 1 pair
    assert np.all(res.tcoll[hit] == res.tcoll[p[hit]])
    # the globally earliest contact (ties to smaller index) is resolved in the first sweep
    pj, tj, _ = oracle.earliest(box, grid=False)
    i0 = min((t, i) for i, t in enumerate(tj) if pj[i] >= 0)[1]
    assert res.partner[i0] == pj[i0] and res.sweep[i0] == 0
    # termination: among the spheres left eligible no contact remains
    pr, _, _ = oracle.earliest(box, active=~hit, grid=False)
    assert np.all(pr[~hit] < 0)
    assert res.n_sweeps == int(res.sweep.max()) + 2      # the last sweep finds nothing


def test_storage_permutation_invariance():
    box = workloads.config(1)
    res = oracle.step(box)
    perm = np.random.default_rng(5).permutation(box.n)
    pbox = box.copy()
    for name in ("x", "y", "z", "vx", "vy", "vz", "r", "m"):
        setattr(pbox, name, getattr(box, name)[perm].copy())
    pres = oracle.step(pbox)
    inv = np.argsort(perm)
    for name in ("x", "y", "z", "vx", "vy", "vz", "tcoll"):
        assert np.array_equal(getattr(pres, name)[inv], getattr(res, name), equal_nan=True)
    mapped = np.where(pres.partner >= 0, perm[np.maximum(pres.partner, 0)], -1)[inv]
    assert np.array_equal(mapped, res.partner)


def test_free_flight_and_wrap():
    box = two_box([0.1, 5, 9.95], [-1, 0, 0.5], 0.1, [5, 5, 5], [0, 0, 0], 0.1, dt=0.2)
    res = oracle.step(box)
    assert res.n_pairs == 0
    assert res.x[0] == pytest.approx(0.1 - 0.2 + 10.0, abs=1e-14)
    assert res.z[0] == pytest.approx(9.95 + 0.1 - 10.0, abs=1e-14)
    assert 0.0 <= res.x[0] < 10.0 and 0.0 <= res.z[0] < 10.0


def test_empty_and_single():
    for n in (0, 1):
        box = workloads.Box(*[np.full(n, 0.5) for _ in range(6)], np.full(n, 0.1), np.ones(n),
                            (2.0, 2.0, 2.0), 0.1, 0.9)
        res = oracle.step(box)
        assert res.n_pairs == 0 and res.x.shape == (n,)


# ---------------------------------------------------------------- error paths


def test_error_codes():
    box = workloads.config(1)
    bad = box.copy()
    bad.r[3] = 0.0
    with pytest.raises(oracle.OracleError) as ei:
        oracle.step(bad)
    assert ei.value.code == oracle.E_INVALID
    bad = box.copy()
    bad.x[5] = box.L[0]
    with pytest.raises(oracle.OracleError) as ei:
        oracle.step(bad)
    assert ei.value.code == oracle.E_INVALID
    bad = box.copy()
    bad.vz[7] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.step(bad)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.step(box, e=1.5)
    assert ei.value.code == oracle.E_INVALID
    big = box.copy()
    big.dt = 0.2          # reach = 2 r + 2 v_max dt exceeds L / 2
    with pytest.raises(oracle.OracleError) as ei:
        oracle.step(big)
    assert ei.value.code == oracle.E_BOX
    with pytest.raises(oracle.OracleError) as ei:
        oracle.step(box, max_sweeps=1)
    assert ei.value.code == oracle.E_SWEEPS


# ---------------------------------------------------------------- kinetic energy analogy


@pytest.mark.slow
def test_kinetic_energy_preservation_and_maxwell_boltzmann():
    """Sec. "Kinetic Energy Analogy and Preservation": 5000 spheres of diameter 0.02 in the
    periodic cube [-1, 1]^3, speed 1 in random directions, e = 1.  Kinetic energy is preserved
    to rounding and the velocity components relax to the Maxwell-Boltzmann normal law with
    variance <|v|^2>/3 = 1/3.  The paper gives no dt; dt = 0.0764 gives about 2e5 collisions
    per 1000 steps at this density (the paper's count); 150 steps are run here."""
    from scipy import stats
    n = 5000
    L = 2.0
    dirs = workloads.normals(42, 9, 3 * n).reshape(n, 3)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    xs, ys, zs = workloads.rsa_positions(42, np.full(n, 0.01), (L, L, L))
    box = workloads.Box(xs, ys, zs, dirs[:, 0].copy(), dirs[:, 1].copy(), dirs[:, 2].copy(),
                        np.full(n, 0.01), np.ones(n), (L, L, L), 0.0764, 1.0)
    ke = lambda b: 0.5 * math.fsum(b.vx ** 2 + b.vy ** 2 + b.vz ** 2)
    ke0 = ke(box)
    comps0 = np.concatenate([box.vx, box.vy, box.vz])
    assert stats.kstest(comps0, "norm", args=(0, math.sqrt(1 / 3))).pvalue < 1e-6
    total = 0
    for _ in range(150):
        res = oracle.step(box)
        total += res.n_pairs
        box = workloads.Box(res.x, res.y, res.z, res.vx, res.vy, res.vz, box.r, box.m, box.L,
                            box.dt, 1.0)
    assert abs(ke(box) - ke0) / ke0 < 1e-13
    comps = np.concatenate([box.vx, box.vy, box.vz])
    assert stats.kstest(comps, "norm", args=(0, math.sqrt(1 / 3))).pvalue > 1e-3
    assert 150 * 2e5 / 1000 * 0.5 < total < 150 * 2e5 / 1000 * 2.0
