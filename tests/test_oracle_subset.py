"""Pins of the oracle's per-sphere search ``orc_earliest_subset`` (the earliest
partner of listed spheres only), which the full-size GPU tests use to check a
sphere's partner and the termination of a step where a whole-step oracle run is
not needed.

It is a separate statement of the earliest-partner rule (its own grid walk), so it
is pinned against the two whole-set statements of the rule, each itself pinned in
``test_oracle_pins.py``: the all-pairs brute force (the definition) on tiny boxes and
the cell-grid search on larger ones, at every listed index, bitwise, with and
without an active mask; and on the independent pure-Python brute force that finds
contact times by bisection.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.indep_bruteforce import earliest as py_earliest


def _masks(n, seed):
    rng = np.random.default_rng(seed)
    return [None, (rng.random(n) < 0.7).astype(np.uint8), (rng.random(n) < 0.2).astype(np.uint8)]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_subset_equals_brute_force_on_tiny_boxes(seed):
    box = workloads.make_box(300, seed=seed, phi=0.3, radius=0.5, e=0.9, dt=0.25)
    idx = np.arange(box.n)
    for act in _masks(box.n, seed):
        bp, bt, _ = oracle.earliest(box, act, grid=False)
        sp, st = oracle.earliest_subset(box, idx, active=act)
        assert np.array_equal(sp, bp)
        assert np.array_equal(st, bt)
        if act is None:
            assert (bp >= 0).sum() > 20


def test_subset_equals_independent_bisection_brute_force():
    box = workloads.make_box(120, seed=9, phi=0.3, radius=0.5, e=0.9, dt=0.2)
    for act in _masks(box.n, 9)[:2]:
        pp, pt = py_earliest(box, act)
        sp, st = oracle.earliest_subset(box, np.arange(box.n), active=act)
        assert np.array_equal(sp, pp)
        has = pp >= 0
        assert np.allclose(st[has], pt[has], rtol=1e-9, atol=0)


def test_subset_equals_grid_search_polydisperse_20k():
    box = workloads.make_box(20_000, seed=11, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)
    rng = np.random.default_rng(5)
    idx = rng.permutation(box.n)  # every sphere, listed in a shuffled order
    for act in _masks(box.n, 5):
        gp, gt, _ = oracle.earliest(box, act)
        sp, st = oracle.earliest_subset(box, idx, active=act)
        assert np.array_equal(sp, gp[idx])
        assert np.array_equal(st, gt[idx])


def test_subset_equals_grid_search_config2_sampled():
    """10,000 listed spheres of config 2 (1M) against the whole-set grid search."""
    box = workloads.config(2)
    rng = np.random.default_rng(7)
    idx = rng.choice(box.n, 10_000, replace=False)
    for act in _masks(box.n, 7)[:2]:
        gp, gt, _ = oracle.earliest(box, act)
        sp, st = oracle.earliest_subset(box, idx, active=act)
        assert np.array_equal(sp, gp[idx])
        assert np.array_equal(st, gt[idx])
        if act is None:
            assert (sp >= 0).sum() > 2000


def test_subset_inactive_and_out_of_range_entries_have_no_partner():
    box = workloads.make_box(300, seed=4, phi=0.3, radius=0.5, e=0.9, dt=0.25)
    act = np.ones(box.n, dtype=np.uint8)
    bp, _, _ = oracle.earliest(box, act, grid=False)
    i = int(np.where(bp >= 0)[0][0])
    act[i] = 0
    sp, st = oracle.earliest_subset(box, np.array([i, -1, box.n, i]), active=act)
    assert np.all(sp == -1) and np.all(np.isinf(st))
    # the partner of a sphere whose partner is switched off is not that sphere any more
    j = int(bp[i])
    sp, _ = oracle.earliest_subset(box, np.array([j]), active=act)
    assert sp[0] != i
