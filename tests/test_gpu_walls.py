"""pcol_step_walls (reflective walls on chosen axes) on the GPU against the oracle's
orc_step_walls, element by element: pair set and contact times bit-exact, positions
and velocities within 1e-12 relative (in practice bitwise)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_helpers import FIELDS, box_slice, compare_step, to_host
import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def poly20k():
    return workloads.make_box(20000, seed=13, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)


def gpu_step_walls(box, walls, ctx=None, **opts):
    p = pc.Particles.from_box(box)
    if ctx is None:
        ctx = pc.Context(max(box.n, 1), pc.pcol_default_opts(**opts) if opts else None)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step_walls(ctx, p, box.L, walls, box.dt, box.e, partner, tcoll)
    torch.cuda.synchronize()
    return to_host(p), partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st


def test_no_walls_equals_pcol_step_bitwise(poly20k):
    _announce("walls none poly20k")
    g = gpu_step_walls(poly20k, (0, 0, 0))
    assert compare_step(poly20k, g, oracle.step(poly20k)) == 0


@pytest.mark.parametrize("walls", [(1, 1, 1), (1, 0, 0), (0, 1, 1)])
@pytest.mark.parametrize("case", ["config1", "poly20k", "poly4097", "config2"])
def test_walls_match_oracle(poly20k, case, walls):
    box = {"config1": lambda: workloads.config(1), "poly20k": lambda: poly20k,
           "poly4097": lambda: box_slice(poly20k, 4097),
           "config2": lambda: workloads.config(2)}[case]()
    _announce(f"walls {walls} {case} n={box.n}")
    g = gpu_step_walls(box, walls)
    orc = oracle.step_walls(box, walls)
    assert orc.n_pairs > 0
    assert compare_step(box, g, orc) == 0


@pytest.mark.parametrize("opts", [{"filter": 1}, {"home_cells": 2}, {"contact_slots": 1},
                                  {"split_quantile": 0.9}, {"split_quantile": 0.0}])
def test_walls_every_filter_and_search_path(poly20k, opts):
    walls = (1, 0, 1)
    _announce(f"walls {walls} poly20k {opts}")
    g = gpu_step_walls(poly20k, walls, **opts)
    assert compare_step(poly20k, g, oracle.step_walls(poly20k, walls)) == 0


@pytest.mark.parametrize("seed", [1, 2])
def test_walls_small_box_fewer_than_three_cells(seed):
    box = workloads.make_box(250, seed=seed, phi=0.3, radius=0.5, e=0.85, dt=0.25)
    _announce(f"walls small box seed={seed}")
    g = gpu_step_walls(box, (1, 1, 1))
    assert min(g[3]["nc"]) < 3
    assert compare_step(box, g, oracle.step_walls(box, (1, 1, 1))) == 0


def test_walls_many_steps_in_lockstep_energy_conserved():
    box = workloads.make_box(3000, seed=9, phi=0.2, radius=0.5, e=1.0, dt=0.25)
    walls = (1, 0, 1)
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n)
    ref = box.copy()
    ke0 = 0.5 * np.sum(box.m * (box.vx ** 2 + box.vy ** 2 + box.vz ** 2))
    _announce("walls 30 steps lockstep")
    for step in range(30):
        pc.pcol_step_walls(ctx, p, box.L, walls, box.dt, box.e)
        r = oracle.step_walls(ref, walls)
        ref.x, ref.y, ref.z, ref.vx, ref.vy, ref.vz = r.x, r.y, r.z, r.vx, r.vy, r.vz
        got = to_host(p)
        for f in FIELDS:
            assert np.array_equal(got[f].view(np.uint64), getattr(ref, f).view(np.uint64)), \
                (step, f)
    ke = 0.5 * np.sum(box.m * (ref.vx ** 2 + ref.vy ** 2 + ref.vz ** 2))
    assert ke == pytest.approx(ke0, rel=1e-12)


def test_composed_api_refuses_a_walls_binning(poly20k):
    box = box_slice(poly20k, 2000)
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n)
    pc.pcol_step_walls(ctx, p, box.L, (1, 0, 0), box.dt, box.e)
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_detect(ctx, p, box.L, box.dt)
    assert ei.value.code == pc.PCOL_E_STATE
    pc.pcol_bin(ctx, p, box.L, box.dt)
    pc.pcol_detect(ctx, p, box.L, box.dt)   # a periodic binning works again
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [0, 1, 2])
def test_walls_degenerate_sizes(n):
    # two spheres colliding at t = 0.2, before the first reaches the x wall (t = 0.3), both
    # reflected afterwards; one sphere alone crosses the wall
    full = workloads.Box(np.array([0.6, 2.0]), np.array([5.0, 5.0]), np.array([5.0, 5.0]),
                         np.array([-2.0, -4.0]), np.zeros(2), np.zeros(2), np.full(2, 0.5),
                         np.ones(2), (20.0, 20.0, 20.0), 0.5, 0.9)
    box = box_slice(full, n)
    _announce(f"walls n={n}")
    g = gpu_step_walls(box, (1, 0, 0))
    assert compare_step(box, g, oracle.step_walls(box, (1, 0, 0))) == 0


def test_walls_restitution_zero_and_errors(poly20k):
    box = box_slice(poly20k, 6000)
    box.e = 0.0
    _announce("walls e=0")
    g = gpu_step_walls(box, (0, 1, 0))
    assert compare_step(box, g, oracle.step_walls(box, (0, 1, 0))) == 0
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n)
    with pytest.raises(pc.PcolError) as ei:   # e outside [0, 1]
        pc.pcol_step_walls(ctx, p, box.L, (1, 1, 1), box.dt, 1.5)
    assert ei.value.code == pc.PCOL_E_INVALID
    x0 = p.x.clone()
    p.x[3] = box.L[0]   # a position outside [0, L) is refused, inputs unchanged otherwise
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_step_walls(ctx, p, box.L, (1, 1, 1), box.dt, box.e)
    assert ei.value.code == pc.PCOL_E_INVALID
    torch.cuda.synchronize()
    assert torch.equal(p.x[4:], x0[4:]) and torch.equal(p.vx, pc.Particles.from_box(box).vx)


def _spin_step_walls(box, w, walls, mu):
    p = pc.Particles.from_box(box)
    wt = [torch.as_tensor(np.ascontiguousarray(w[k]), dtype=torch.float64).cuda() for k in range(3)]
    ctx = pc.Context(max(box.n, 1))
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step_spin_walls(ctx, p, wt, box.L, walls, box.dt, box.e, mu, partner, tcoll)
    torch.cuda.synchronize()
    ws = np.stack([t.cpu().numpy() for t in wt])
    return (to_host(p), partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st), ws


@pytest.mark.parametrize("case,walls,mu", [("config1", (1, 1, 1), 0.4), ("poly20k", (1, 0, 1), 0.1),
                                           ("poly20k", (1, 1, 1), 5.0), ("config2", (1, 1, 1), 0.4),
                                           ("poly20k", (0, 0, 0), 0.4)])
def test_friction_between_walls_matches_oracle(poly20k, case, walls, mu):
    box = {"config1": lambda: workloads.config(1), "poly20k": lambda: poly20k,
           "config2": lambda: workloads.config(2)}[case]()
    w = np.random.default_rng(box.n % 97).normal(size=(3, box.n)) / box.r
    _announce(f"friction between walls {walls} {case} n={box.n} mu={mu}")
    g, ws = _spin_step_walls(box, w, walls, mu)
    orc = oracle.step_walls_spin(box, walls, w, mu)
    assert orc.n_pairs > 0
    assert compare_step(box, g, orc) == 0
    ref = np.stack([orc.wx, orc.wy, orc.wz])
    assert np.array_equal(ws.view(np.uint64), ref.view(np.uint64))
