"""Pins of the oracle's deposition onto cell-corner nodes (CPU only).

Sec. "Dispersed Phase" projects a per-particle source linearly onto the eight
corner nodes of the host element (a C0 version of inverse distance weighting);
Sec. "Deposition" takes the deposition radius equal to the cell size, numbers the
corner nodes with periodic identification and sums the contributions of all
particles node by node (conservative).  On a Cartesian grid of equal cells these
linear corner weights are the trilinear hat functions.  The pins: closed forms
(a sphere at a node, at a cell centre), the reference-space form of the weights,
the tent-function form by brute force, the adjoint of scipy's trilinear
interpolation, conservation, reproduction of linear fields, periodic wrap,
translation by one cell, linearity, and the error cases."""
import itertools

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import workloads


def _dep(x, y, z, a, nc, L):
    return oracle.deposit(np.atleast_1d(np.asarray(x, float)), np.atleast_1d(np.asarray(y, float)),
                          np.atleast_1d(np.asarray(z, float)), a, nc, L)


def test_sphere_on_a_node_gives_it_everything():
    nc, L = (4, 5, 6), (2.0, 2.5, 3.0)          # h = 0.5 on every axis
    out = _dep(1.0, 1.5, 0.5, [[3.0]], nc, L)
    assert out[0, 1, 3, 2] == 3.0                # node (i, j, k) = (2, 3, 1), stored [k, j, i]
    assert np.count_nonzero(out) == 1


def test_sphere_at_cell_centre_splits_in_eight():
    nc, L = (4, 4, 4), (4.0, 4.0, 4.0)
    out = _dep(1.5, 2.5, 0.5, [[8.0], [-2.0]], nc, L)
    for q, val in ((0, 1.0), (1, -0.25)):
        nz = np.argwhere(out[q] != 0)
        assert len(nz) == 8 and np.all(out[q][out[q] != 0] == val)
        assert {tuple(v) for v in nz} == {(k, j, i) for i in (1, 2) for j in (2, 3) for k in (0, 1)}


def _cell(p, L, nc):
    h = L / nc
    c = min(int(np.floor(p / h)), nc - 1)
    return c, p / h - c


def test_weights_equal_the_reference_space_form():
    # In reference coordinates xi in [-1, 1]^3 the linear corner weight of corner
    # xi_n in {-1, 1}^3 is prod_d (1 + xi_n^d xi^d) / 2.
    rng = np.random.default_rng(3)
    nc, L = (7, 5, 3), np.array([1.3, 0.7, 2.9])
    for _ in range(40):
        p = rng.random(3) * L
        out = _dep(*p, [[1.0]], nc, L)[0]
        cf = [_cell(p[d], L[d], nc[d]) for d in range(3)]
        xi = np.array([2.0 * f - 1.0 for _, f in cf])
        for corner in itertools.product((-1, 1), repeat=3):
            w = np.prod([(1.0 + corner[d] * xi[d]) / 2.0 for d in range(3)])
            idx = [(cf[d][0] + (corner[d] + 1) // 2) % nc[d] for d in range(3)]
            assert out[idx[2], idx[1], idx[0]] == pytest.approx(w, abs=2e-16)
        assert out.sum() == pytest.approx(1.0, abs=4e-16)


def test_brute_force_tent_functions_on_a_tiny_grid():
    # Each node carries the tent function prod_d max(0, 1 - |x_d - X_d| / h_d)
    # with the periodic minimum-image distance; every node is visited.
    nc, L = (3, 4, 5), np.array([0.9, 1.6, 2.5])
    h = L / nc
    x, y, z, a = workloads.deposit_case(60, seed=11, L=L, comp=2)
    out = oracle.deposit(x, y, z, a, nc, L)
    ref = np.zeros_like(out)
    for i in range(len(x)):
        p = (x[i], y[i], z[i])
        for k in range(nc[2]):
            for j in range(nc[1]):
                for ii in range(nc[0]):
                    w = 1.0
                    for d, node in enumerate((ii, j, k)):
                        dist = abs(p[d] - node * h[d])
                        dist = min(dist, L[d] - dist)
                        w *= max(0.0, 1.0 - dist / h[d])
                    ref[:, k, j, ii] += w * a[:, i]
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13)


def test_adjoint_of_trilinear_interpolation():
    # Deposition is the transpose of trilinear interpolation of a node field:
    # sum_nodes out(node) g(node) = sum_i a_i g(x_i), with g interpolated by scipy
    # on the grid extended by one periodic layer.
    nc, L = (6, 9, 4), np.array([1.2, 2.7, 0.8])
    x, y, z, a = workloads.deposit_case(3000, seed=5, L=L, comp=3)
    out = oracle.deposit(x, y, z, a, nc, L)
    rng = np.random.default_rng(9)
    for q in range(3):
        g = rng.normal(size=(nc[2], nc[1], nc[0]))
        gp = np.pad(g, ((0, 1), (0, 1), (0, 1)), mode="wrap")
        axes = [np.arange(nc[d] + 1) * (L[d] / nc[d]) for d in (2, 1, 0)]
        gi = RegularGridInterpolator(axes, gp, method="linear")(np.stack([z, y, x], axis=1))
        lhs = float(np.sum(out[q] * g))
        rhs = float(np.sum(a[q] * gi))
        assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-11)


def test_conservation_and_linear_field_reproduction():
    nc, L = (8, 8, 8), np.array([1.0, 1.0, 1.0])
    x, y, z, a = workloads.deposit_case(5000, seed=7, L=L, comp=1)
    out = oracle.deposit(x, y, z, a, nc, L)
    assert out.sum() == pytest.approx(a.sum(), rel=1e-12, abs=1e-12)
    # Unit sources on spheres away from the last cell (no wrap): the first moments of
    # the node sums equal the sums of the positions.
    keep = (x < 7 / 8) & (y < 7 / 8) & (z < 7 / 8)
    ones = np.ones((1, int(keep.sum())))
    m = oracle.deposit(x[keep], y[keep], z[keep], ones, nc, L)[0]
    X = np.arange(8) / 8.0
    assert np.sum(m * X[None, None, :]) == pytest.approx(x[keep].sum(), rel=1e-12)
    assert np.sum(m * X[None, :, None]) == pytest.approx(y[keep].sum(), rel=1e-12)
    assert np.sum(m * X[:, None, None]) == pytest.approx(z[keep].sum(), rel=1e-12)


def test_periodic_wrap_of_the_last_cell():
    nc, L = (4, 4, 4), (1.0, 1.0, 1.0)
    out = _dep(0.875, 0.125, 0.125, [[1.0]], nc, L)[0]   # centre of cell (3, 0, 0)
    assert out[0, 0, 0] == 0.125 and out[0, 0, 3] == 0.125 and out[1, 1, 0] == 0.125
    assert np.count_nonzero(out) == 8


def test_translation_by_one_cell_rolls_the_nodes():
    nc, L = (8, 4, 16), (1.0, 0.5, 2.0)          # h = 0.125: shifts are exact
    x, y, z, a = workloads.deposit_case(400, seed=2, L=L, comp=2)
    out = oracle.deposit(x, y, z, a, nc, L)
    xs = np.mod(x + 0.125, 1.0)
    zs = np.mod(z + 3 * 0.125, 2.0)
    sh = oracle.deposit(xs, y, zs, a, nc, L)
    np.testing.assert_allclose(sh, np.roll(np.roll(out, 1, axis=3), 3, axis=1), rtol=0, atol=1e-13)


def test_components_are_independent_and_linear():
    nc, L = (5, 6, 7), (1.0, 1.2, 1.4)
    x, y, z, a = workloads.deposit_case(500, seed=4, L=L, comp=3)
    out = oracle.deposit(x, y, z, a, nc, L)
    for q in range(3):
        np.testing.assert_array_equal(out[q], oracle.deposit(x, y, z, a[q:q + 1], nc, L)[0])
    s = oracle.deposit(x, y, z, np.stack([a[0] + a[1]]), nc, L)[0]
    np.testing.assert_allclose(s, out[0] + out[1], rtol=0, atol=1e-13)


def test_empty_input_gives_zeros():
    out = oracle.deposit(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros((4, 0)), (3, 3, 3),
                         (1.0, 1.0, 1.0))
    assert out.shape == (4, 3, 3, 3) and not out.any()


@pytest.mark.parametrize("p", [(1.0, 0.5, 0.5), (-1e-300, 0.5, 0.5), (0.5, np.nan, 0.5),
                               (0.5, 0.5, np.inf)])
def test_positions_outside_the_box_are_rejected(p):
    with pytest.raises(oracle.OracleError):
        _dep(*p, [[1.0]], (2, 2, 2), (1.0, 1.0, 1.0))


def test_invalid_grid_is_rejected():
    with pytest.raises(oracle.OracleError):
        _dep(0.5, 0.5, 0.5, [[1.0]], (0, 2, 2), (1.0, 1.0, 1.0))
    with pytest.raises(oracle.OracleError):
        _dep(0.5, 0.5, 0.5, [[1.0]], (2, 2, 2), (1.0, 0.0, 1.0))
