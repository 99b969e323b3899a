"""Pins of the oracle's forward-mode derivative (step_jvp), CPU only.

The derivative is checked against the textbook head-on restitution result
differentiated by hand, and against central finite differences of the oracle's
primal step (a computation independent of the tangent code) over one and
several steps, with the pair set held fixed.
"""
import numpy as np
import pytest

import oracle
import workloads


def _perturbed(box, q, h):
    b = box.copy()
    for k, f in enumerate(("x", "y", "z")):
        setattr(b, f, np.mod(getattr(b, f) + h * q["dx"][k], box.L[k]))
    for k, f in enumerate(("vx", "vy", "vz")):
        setattr(b, f, getattr(b, f) + h * q["dv"][k])
    b.e = box.e + h * q["de"]
    return b


def _state(res):
    return np.array([res.x, res.y, res.z]), np.array([res.vx, res.vy, res.vz])


def _min_image(dx, L):
    L = np.asarray(L)[:, None]
    return dx - L * np.round(dx / L)


def test_head_on_closed_form_derivatives():
    m1, m2, e = 1.0, 3.0, 0.6
    v1, v2 = 0.5, -0.5
    box = workloads.Box(np.array([1.0, 4.0]), np.array([2.0, 2.0]), np.array([2.0, 2.0]),
                        np.array([v1, v2]), np.zeros(2), np.zeros(2), np.array([0.5, 0.5]),
                        np.array([m1, m2]), (10.0, 10.0, 10.0), 3.0, e)
    z = np.zeros((3, 2))
    # d/de
    _, _, tx, tv, partner = oracle.step_jvp(box, z, z, 1.0)
    assert partner.tolist() == [1, 0]
    assert tv[0, 0] == pytest.approx(m2 * (v2 - v1) / (m1 + m2), abs=1e-15)
    assert tv[0, 1] == pytest.approx(m1 * (v1 - v2) / (m1 + m2), abs=1e-15)
    # d/dv1: v1' = ((m1 - e m2) v1 + (1 + e) m2 v2) / (m1 + m2); contact at t = (D - s) / (v1 - v2)
    dv = np.zeros((3, 2))
    dv[0, 0] = 1.0
    _, _, tx, tv, _ = oracle.step_jvp(box, z, dv, 0.0)
    assert tv[0, 0] == pytest.approx((m1 - e * m2) / (m1 + m2), abs=1e-15)
    t = (3.0 - 1.0) / (v1 - v2)
    v1p = ((m1 - e * m2) * v1 + (1 + e) * m2 * v2) / (m1 + m2)
    dt_dv1 = -t / (v1 - v2)
    expect = dt_dv1 * (v1 - v1p) + t + (box.dt - t) * (m1 - e * m2) / (m1 + m2)
    assert tx[0, 0] == pytest.approx(expect, abs=1e-14)


def _fd_check(box, steps, seed, h=1e-7, rel=2e-6):
    rng = np.random.default_rng(seed)
    n = box.n
    q = {"dx": rng.normal(size=(3, n)), "dv": rng.normal(size=(3, n)), "de": rng.normal()}
    # tangent through `steps` steps
    b = box.copy()
    tx, tv, te = q["dx"], q["dv"], q["de"]
    partners = []
    for _ in range(steps):
        xo, vo, tx, tv, partner = oracle.step_jvp(b, tx, tv, te)
        partners.append(partner)
        b = workloads.Box(*xo, *vo, b.r, b.m, b.L, b.dt, b.e)
    # finite differences of the primal
    outs = []
    for sgn in (1, -1):
        bb = _perturbed(box, q, sgn * h)
        for k in range(steps):
            res = oracle.step(bb)
            if not np.array_equal(res.partner, partners[k]):
                pytest.skip("pair set changed under the perturbation")
            bb = workloads.Box(res.x, res.y, res.z, res.vx, res.vy, res.vz, bb.r, bb.m, bb.L,
                               bb.dt, bb.e)
        outs.append((np.array([bb.x, bb.y, bb.z]), np.array([bb.vx, bb.vy, bb.vz])))
    fdx = _min_image(outs[0][0] - outs[1][0], box.L) / (2 * h)
    fdv = (outs[0][1] - outs[1][1]) / (2 * h)
    scale_x = np.max(np.abs(tx)) + 1.0
    scale_v = np.max(np.abs(tv)) + 1.0
    assert np.max(np.abs(fdx - tx)) <= rel * scale_x * 10
    assert np.max(np.abs(fdv - tv)) <= rel * scale_v * 10
    return sum(int((p >= 0).sum()) for p in partners)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_jvp_matches_central_differences_one_step(seed):
    box = workloads.make_box(300, seed=seed, phi=0.25, lognormal=(0.5, 0.3, 0.25, 1.0), e=0.7,
                             dt=0.2)
    assert _fd_check(box, 1, seed) > 40


def test_jvp_matches_central_differences_three_steps():
    box = workloads.make_box(300, seed=7, phi=0.2, radius=0.5, e=0.85, dt=0.15)
    assert _fd_check(box, 3, 7) > 60


def test_jvp_linearity_and_zero_tangent():
    box = workloads.make_box(200, seed=4, phi=0.2, radius=0.5, e=0.9, dt=0.2)
    rng = np.random.default_rng(0)
    a = (rng.normal(size=(3, box.n)), rng.normal(size=(3, box.n)), 0.3)
    b = (rng.normal(size=(3, box.n)), rng.normal(size=(3, box.n)), -1.1)
    ra = oracle.step_jvp(box, *a)
    rb = oracle.step_jvp(box, *b)
    rab = oracle.step_jvp(box, a[0] + 2 * b[0], a[1] + 2 * b[1], a[2] + 2 * b[2])
    assert np.allclose(rab[2], ra[2] + 2 * rb[2], rtol=1e-12, atol=1e-12)
    assert np.allclose(rab[3], ra[3] + 2 * rb[3], rtol=1e-12, atol=1e-12)
    z = np.zeros((3, box.n))
    r0 = oracle.step_jvp(box, z, z, 0.0)
    assert np.all(r0[2] == 0) and np.all(r0[3] == 0)
