"""Pins of the oracle's collision with Coulomb friction and spin (CPU only).

The resolve follows Sec. "Inter-Particle Collisions" (impulse J = J_n n_p + J_t t_p,
J_t = max(mu J_n, -(2/7)(1+e) m_r |v_rt|), jump relations of momentum and angular
momentum) with the solid-sphere moment of inertia of Sec. "Dispersed Phase"
(I = pi rho d^5 / 60 = m d^2 / 10).  It is pinned against the frictionless
oracle (mu = 0), conservation of linear and angular momentum per pair, the
energy balance, and closed forms of a sliding and a sticking impact."""
import numpy as np
import pytest

import oracle
import workloads


def _cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def _spins(n, seed, scale=3.0):
    return np.random.default_rng(seed).normal(size=(3, n)) * scale


def test_zero_friction_is_the_frictionless_step_bitwise():
    box = workloads.config(1)
    w = _spins(box.n, 5, 30.0)
    a = oracle.step(box)
    b = oracle.step_spin(box, w, 0.0)
    assert a.n_pairs > 100 and b.n_pairs == a.n_pairs
    for f in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(getattr(a, f).view(np.uint64), getattr(b, f).view(np.uint64)), f
    assert np.array_equal(a.partner, b.partner) and np.array_equal(a.tcoll, b.tcoll, equal_nan=True)
    for k, f in enumerate(("wx", "wy", "wz")):
        assert np.array_equal(getattr(b, f), w[k])


def _pairs(res):
    return [(i, int(j)) for i, j in enumerate(res.partner) if j > i]


def _unwrap(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("mu", [0.1, 0.4, 5.0])
@pytest.mark.parametrize("e", [0.0, 0.8, 1.0])
def test_momentum_angular_momentum_and_energy_per_pair(mu, e):
    """Per collided pair: linear momentum and angular momentum (about the origin,
    the two spheres at their contact positions, unwrapped) are conserved to rounding,
    and the kinetic energy (translation + rotation) does not grow."""
    box = workloads.config(1)
    w = _spins(box.n, 11, 40.0)
    res = oracle.step_spin(box, w, mu, e=e)
    L = np.array(box.L)
    pairs = _pairs(res)
    assert len(pairs) > 100
    x0 = np.array([box.x, box.y, box.z])
    v0 = np.array([box.vx, box.vy, box.vz])
    v1 = np.array([res.vx, res.vy, res.vz])
    w1 = np.array([res.wx, res.wy, res.wz])
    m, r = box.m, box.r
    inertia = m * (2 * r) ** 2 / 10.0
    worst_p = worst_l = 0.0
    for i, j in pairs:
        t = res.tcoll[i]
        xi = x0[:, i] + t * v0[:, i]
        xj = xi + _unwrap((x0[:, j] + t * v0[:, j]) - xi, L)
        dp = m[i] * (v1[:, i] - v0[:, i]) + m[j] * (v1[:, j] - v0[:, j])
        pscale = m[i] * np.abs(v0[:, i]).max() + m[j] * np.abs(v0[:, j]).max()
        worst_p = max(worst_p, np.abs(dp).max() / pscale)
        dl = (m[i] * _cross(xi, v1[:, i] - v0[:, i]) + inertia[i] * (w1[:, i] - w[:, i]) +
              m[j] * _cross(xj, v1[:, j] - v0[:, j]) + inertia[j] * (w1[:, j] - w[:, j]))
        lscale = sum(m[k] * np.abs(xx).max() * np.abs(v0[:, k]).max() + inertia[k] *
                     np.abs(w[:, k]).max() for k, xx in ((i, xi), (j, xj)))
        worst_l = max(worst_l, np.abs(dl).max() / lscale)
        ke0 = sum(0.5 * m[k] * v0[:, k] @ v0[:, k] + 0.5 * inertia[k] * w[:, k] @ w[:, k]
                  for k in (i, j))
        ke1 = sum(0.5 * m[k] * v1[:, k] @ v1[:, k] + 0.5 * inertia[k] * w1[:, k] @ w1[:, k]
                  for k in (i, j))
        assert ke1 <= ke0 * (1 + 1e-13), (i, j, ke0, ke1)
    assert worst_p < 1e-14 and worst_l < 1e-13, (worst_p, worst_l)


def _impact(vy, spin_z, mu, e, r=0.5, m=(1.0, 1.0)):
    """Sphere 0 at rest-frame contact along +x with sphere 1 at t = 0.25: sphere 0
    moves (1, vy, 0) and spins spin_z about z, sphere 1 is at rest without spin."""
    s = 2 * r
    # separation at the start chosen so that d + 0.25 u = (s, 0, 0): n = x at contact
    d = np.array([s + 0.25, 0.25 * vy, 0.0])
    x0 = np.array([3.0, 3.0, 3.0])
    box = workloads.Box(np.array([x0[0], x0[0] + d[0]]), np.array([x0[1], x0[1] + d[1]]),
                        np.array([x0[2], x0[2]]), np.array([1.0, 0.0]), np.array([vy, 0.0]),
                        np.zeros(2), np.full(2, r), np.array(m), (20.0, 20.0, 20.0), 1.0, e)
    w = np.zeros((3, 2))
    w[2, 0] = spin_z
    xs, vs, ws = oracle.resolve_pair_spin(box, w, mu, 0, 1, 0.25)
    return box, w, vs, ws


@pytest.mark.parametrize("e", [0.5, 0.9])
def test_sliding_impact_closed_form(e):
    """Small friction: the tangential impulse is mu J_n (sliding)."""
    mu, vy = 0.05, 2.0
    box, w, vs, ws = _impact(vy, 0.0, mu, e)
    mr = 0.5
    jn = -mr * (1 + e) * 1.0          # J_n = -m_r (1+e) (v_r . n), v_r . n = 1
    jt = mu * jn                      # sliding: |mu J_n| below (2/7)(1+e) m_r |v_rt|
    assert abs(jt) < (2 / 7) * (1 + e) * mr * vy
    inertia = 1.0 * 1.0 ** 2 / 10
    exp_v0 = np.array([1.0 + jn, vy + jt, 0.0])      # t_p = +y
    exp_v1 = np.array([-jn, -jt, 0.0])
    exp_w = 0.5 * jt / inertia                       # (n x J)_z = J_t, r = 0.5
    assert np.allclose(vs[0], exp_v0, rtol=0, atol=1e-12)
    assert np.allclose(vs[1], exp_v1, rtol=0, atol=1e-12)
    assert np.allclose(ws[0], [0, 0, exp_w], rtol=0, atol=1e-11)
    assert np.allclose(ws[1], [0, 0, exp_w], rtol=0, atol=1e-11)


@pytest.mark.parametrize("e", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("spin_z", [0.0, 3.0])
def test_sticking_impact_reverses_contact_slip_by_e(e, spin_z):
    """Large friction: J_t = -(2/7)(1+e) m_r |v_rt| (sticking), which for solid spheres
    turns the tangential contact-point velocity v_rt into -e v_rt."""
    box, w, vs, ws = _impact(2.0, spin_z, 50.0, e)
    n = np.array([1.0, 0.0, 0.0])
    r = box.r

    def slip(v, om):
        vc = (v[0] - v[1]) + _cross(r[0] * om[0] + r[1] * om[1], n)
        return vc - (vc @ n) * n

    before = slip(np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 0.0]]), w.T)
    after = slip(vs, ws)
    assert np.linalg.norm(before) > 0.5
    assert np.allclose(after, -e * before, rtol=0, atol=1e-12), (before, after)


def test_perspective_and_storage_order_independent_bitwise():
    """The two sides of a pair evaluate exact negations of each other, so the result
    does not depend on which sphere is stored first."""
    box = workloads.make_box(300, seed=3, phi=0.3, radius=1.0, dt=0.4, e=0.9)
    w = _spins(box.n, 8, 5.0)
    a = oracle.step_spin(box, w, 0.3)
    perm = np.random.default_rng(2).permutation(box.n)
    pbox = workloads.Box(*[arr[perm] for arr in box.arrays()], box.L, box.dt, box.e)
    b = oracle.step_spin(pbox, w[:, perm], 0.3)
    assert a.n_pairs > 10
    for f in ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz"):
        assert np.array_equal(getattr(a, f)[perm].view(np.uint64), getattr(b, f).view(np.uint64)), f


def test_spin_errors():
    box = workloads.config(1)
    w = _spins(box.n, 1)
    with pytest.raises(oracle.OracleError):
        oracle.step_spin(box, w, -0.1)
    w[1, 7] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.step_spin(box, w, 0.2)
