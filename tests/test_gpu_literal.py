"""The paper's collision order taken literally, on the GPU (opts.order = 1), against
the oracle's sequential statement of it (``orc_step_sequential``: elements along the
Morton curve, each particle taking the first eligible partner with a contact in its
candidate elements in curve order, both then leaving the eligible set).

That sequential pass gives the greedy matching of the contact graph under the order
of an edge's lower-ranked end, then its higher-ranked end, a sphere's rank being
(Morton code of its cell, index).  The GPU reaches the same matching in parallel:
every sphere points at its eligible contact of smallest rank and every mutual pair
collides, sweep after sweep.  Pair sets, contact times and states must equal the
oracle's bitwise, on every search path (both filters, the extent split, one contact
slot, a grid with fewer than three cells per axis) and on the 1M workload.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.edge_cases import edge_box
from tests.gpu_helpers import compare_step, gpu_step

pytestmark = pytest.mark.gpu

import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def poly20k():
    return workloads.make_box(20_000, seed=11, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)


@pytest.fixture(scope="module")
def cfg2():
    return workloads.config(2)


@pytest.mark.parametrize("which", ["config1", "poly20k", "small", "edge", "config2"])
def test_literal_order_matches_oracle(which, poly20k, cfg2):
    if which == "config1":
        box = workloads.config(1)
    elif which == "poly20k":
        box = poly20k
    elif which == "small":
        box = workloads.make_box(250, seed=5, phi=0.3, radius=0.5, e=0.85, dt=0.25)
    elif which == "edge":
        box = edge_box()[0]
    else:
        box = cfg2
    _announce(f"literal order {which} n={box.n}")
    orc = oracle.step_sequential(box)
    gpu = gpu_step(box, order=1)
    assert compare_step(box, gpu, orc) == 0
    assert gpu[3]["n_pairs"] == orc.n_pairs and orc.n_pairs > 0
    # the mutual-earliest rule gives a different matching of the same contacts
    if box.n >= 20_000:
        early = oracle.step(box)
        assert not np.array_equal(early.partner, orc.partner)


@pytest.mark.parametrize("opts", [{"filter": 1}, {"split_quantile": 0.0}, {"split_quantile": 0.9},
                                  {"contact_slots": 1}, {"contact_slots": 2, "filter": 1},
                                  {"cell_mult": 1.7}],
                         ids=["fp32", "nosplit", "split0.9", "slots1", "slots2fp32", "cell1.7"])
def test_literal_order_every_search_path(poly20k, opts):
    """The order is the curve grid's (cell side the reach), whatever grid, filter or
    contact-slot count the search uses."""
    _announce(f"literal order poly20k {opts}")
    gpu = gpu_step(poly20k, order=1, **opts)
    assert compare_step(poly20k, gpu, oracle.step_sequential(poly20k)) == 0


def test_literal_order_refused_where_not_built(poly20k):
    p = pc.Particles.from_box(poly20k)
    ctx = pc.Context(poly20k.n, pc.pcol_default_opts(order=1))
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_step_walls(ctx, p, poly20k.L, (1, 0, 0), poly20k.dt, poly20k.e)
    assert ei.value.code == pc.PCOL_E_INVALID
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_step_batched(ctx, p, [0, poly20k.n], [poly20k.L], poly20k.dt, poly20k.e)
    assert ei.value.code == pc.PCOL_E_INVALID
    with pytest.raises(pc.PcolError):
        pc.Context(10, pc.pcol_default_opts(order=2))
