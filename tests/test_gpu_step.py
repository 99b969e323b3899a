"""GPU parity of the HIP collision step against the FP64 oracle (needs an MI355X).

Bar: pair sets (partner per sphere) bit-exact, contact times bitwise equal, and
post-collision positions and velocities within 1e-12 relative; the rule fixes
every binary64 operation, so the states are expected to agree bitwise as well
and a dedicated test asserts that.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_helpers import FIELDS, box_slice, compare_step, gpu_step, to_host

pytestmark = pytest.mark.gpu

import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def cfg2():
    return workloads.config(2)


@pytest.fixture(scope="module")
def poly20k():
    # the 16M recipe (lognormal radii, phi 0.3, e 0.8) at 20k spheres: 8^3 cells
    return workloads.make_box(20000, seed=13, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)


def test_step_config1_bitwise():
    box = workloads.config(1)
    _announce(f"config1 n={box.n}")
    gpu = gpu_step(box)
    orc = oracle.step(box)
    assert orc.n_pairs > 50
    assert compare_step(box, gpu, orc) == 0
    st = gpu[3]
    assert st["n_pairs"] == orc.n_pairs and st["n_sweeps"] == orc.n_sweeps


def test_step_config2_1M(cfg2):
    _announce(f"config2 n={cfg2.n}")
    gpu = gpu_step(cfg2)
    orc = oracle.step(cfg2)
    nonbit = compare_step(cfg2, gpu, orc)
    assert nonbit == 0
    st = gpu[3]
    assert st["n_pairs"] == orc.n_pairs and st["n_sweeps"] == orc.n_sweeps
    assert st["pair_tests"] > 0 and st["contacts"] >= orc.n_pairs


@pytest.mark.parametrize("n", [20000, 19963, 4097, 65])
def test_step_polydisperse_tiles_and_ragged(poly20k, n):
    box = box_slice(poly20k, n)
    _announce(f"poly n={n}")
    gpu = gpu_step(box)
    orc = oracle.step(box)
    assert compare_step(box, gpu, orc) == 0


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
@pytest.mark.parametrize("mono", [True, False])
def test_step_small_box_fewer_than_three_cells(seed, mono):
    if mono:
        box = workloads.make_box(250, seed=seed, phi=0.3, radius=0.5, e=0.85, dt=0.25)
    else:
        box = workloads.make_box(250, seed=seed, phi=0.3, lognormal=(0.5, 0.3, 0.25, 1.0), e=0.85,
                                 dt=0.2)
    _announce(f"small box seed={seed} mono={mono}")
    gpu = gpu_step(box)
    assert min(gpu[3]["nc"]) < 3
    orc = oracle.step(box)
    assert orc.n_sweeps >= 3
    assert compare_step(box, gpu, orc) == 0


@pytest.mark.parametrize("e", [0.0, 1.0])
def test_step_restitution_limits(poly20k, e):
    box = box_slice(poly20k, 8000)
    box.e = e
    gpu = gpu_step(box)
    orc = oracle.step(box)
    assert compare_step(box, gpu, orc) == 0


@pytest.mark.parametrize("n", [0, 1, 2])
def test_step_degenerate_sizes(n):
    base = workloads.Box(np.array([1.0, 4.0]), np.array([2.0, 2.0]), np.array([2.0, 2.0]),
                         np.array([0.5, -0.5]), np.zeros(2), np.zeros(2), np.array([0.5, 0.5]),
                         np.ones(2), (10.0, 10.0, 10.0), 3.0, 0.7)
    box = box_slice(base, n)
    gpu = gpu_step(box)
    orc = oracle.step(box)
    assert compare_step(box, gpu, orc) == 0
    if n == 2:
        assert gpu[1].tolist() == [1, 0] and gpu[2][0] == 2.0


def test_two_sphere_periodic_case_multistep():
    """The paper's two-sphere validation inputs, stepped on the GPU and the oracle in
    lockstep; the contact happens through the periodic y boundary in step 40."""
    L = (2.2, 2.2, 2.2)
    box = workloads.Box(np.array([1.08, 1.117]), np.array([0.6, 1.6]), np.array([1.1, 1.1]),
                        np.array([0.0, 0.0]), np.array([-15.0, 15.0]), np.zeros(2),
                        np.array([0.02, 0.02]), np.ones(2), L, 1e-3, 1.0)
    hit = None
    for k in range(45):
        gpu = gpu_step(box)
        orc = oracle.step(box)
        assert compare_step(box, gpu, orc) == 0
        if orc.n_pairs and hit is None:
            hit = k
        out = gpu[0]
        box = workloads.Box(out["x"], out["y"], out["z"], out["vx"], out["vy"], out["vz"], box.r,
                            box.m, L, box.dt, 1.0)
    assert hit == 39


def test_detect_keys_all_active_and_masked(poly20k):
    box = poly20k
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n)
    pc.pcol_bin(ctx, p, box.L, box.dt)
    key, tmin = pc.pcol_detect(ctx, p, box.L, box.dt)
    torch.cuda.synchronize()
    key = key.cpu().numpy().view(np.uint64)
    tmin = tmin.cpu().numpy()
    op, ot, _ = oracle.earliest(box)
    has = op >= 0
    assert np.array_equal(key == np.uint64(2 ** 64 - 1), ~has)
    assert np.array_equal((key[has] & np.uint64(0xFFFFFFFF)).astype(np.int64), op[has])
    f32 = ot[has].astype(np.float32).view(np.uint32).astype(np.uint64)
    assert np.array_equal(key[has] >> np.uint64(32), f32)
    assert np.array_equal(tmin, ot)
    # a random active mask (exact neighbourhood search path)
    act = (np.random.default_rng(3).random(box.n) < 0.6).astype(np.uint8)
    key2, tmin2 = pc.pcol_detect(ctx, p, box.L, box.dt, active=torch.from_numpy(act).cuda())
    torch.cuda.synchronize()
    op2, ot2, _ = oracle.earliest(box, active=act)
    key2 = key2.cpu().numpy().view(np.uint64)
    has2 = op2 >= 0
    assert np.array_equal((key2[has2] & np.uint64(0xFFFFFFFF)).astype(np.int64), op2[has2])
    assert np.all(key2[~has2] == np.uint64(2 ** 64 - 1))
    assert np.array_equal(tmin2.cpu().numpy(), ot2)


def test_composed_entry_points_equal_step(poly20k):
    """pcol_bin, then pcol_detect + pcol_resolve per sweep, then pcol_advance, gives the
    same result as pcol_step."""
    box = box_slice(poly20k, 12000)
    ref = gpu_step(box)
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n)
    n = box.n
    pc.pcol_bin(ctx, p, box.L, box.dt)
    active = torch.ones(n, dtype=torch.uint8, device="cuda")
    partner = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    tcoll = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    sweeps = 0
    while True:
        key, _ = pc.pcol_detect(ctx, p, box.L, box.dt, active=active)
        before = int(npairs.item())
        pc.pcol_resolve(ctx, p, box.L, box.dt, box.e, key, active, partner, tcoll, npairs)
        sweeps += 1
        if int(npairs.item()) == before:
            break
    pc.pcol_advance(ctx, p, box.L, box.dt, partner)
    torch.cuda.synchronize()
    out = {f: getattr(p, f).cpu().numpy() for f in FIELDS}
    for f in FIELDS:
        assert np.array_equal(out[f], ref[0][f])
    assert np.array_equal(partner.cpu().numpy(), ref[1])
    assert np.array_equal(tcoll.cpu().numpy(), ref[2], equal_nan=True)
    assert sweeps == ref[3]["n_sweeps"]


def test_invariance_cell_size_slots_and_permutation(poly20k):
    box = box_slice(poly20k, 15000)
    ref = gpu_step(box)
    for opts in ({"cell_mult": 1.7}, {"cell_mult": 2.5}, {"contact_slots": 1},
                 {"contact_slots": 2}):
        got = gpu_step(box, **opts)
        for f in FIELDS:
            assert np.array_equal(got[0][f], ref[0][f]), opts
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2], equal_nan=True)
    perm = np.random.default_rng(9).permutation(box.n)
    pbox = workloads.Box(*[a[perm].copy() for a in box.arrays()], box.L, box.dt, box.e)
    got = gpu_step(pbox)
    inv = np.argsort(perm)
    for f in FIELDS:
        assert np.array_equal(got[0][f][inv], ref[0][f])
    mapped = np.where(got[1] >= 0, perm[np.maximum(got[1], 0)], -1)[inv]
    assert np.array_equal(mapped, ref[1])


def test_determinism_rerun(cfg2):
    a = gpu_step(cfg2)
    b = gpu_step(cfg2)
    for f in FIELDS:
        assert np.array_equal(a[0][f].view(np.uint64), b[0][f].view(np.uint64))
    assert np.array_equal(a[1], b[1])


def test_grid_of_the_last_call_reused_and_replaced(poly20k):
    """A context tries the grid of its last binning first (its reach pass then bins on
    it too) and keeps it only when this call's reach leads to the same grid and split
    extent: repeated, changed and invalid inputs on one context all give the oracle's
    step, and the grid follows the reach of each call."""
    ctx = pc.Context(poly20k.n)
    fast = poly20k.copy()
    for f in ("vx", "vy", "vz"):
        getattr(fast, f)[:] *= 2.0  # a larger reach: another grid
    bad = poly20k.copy()
    bad.x[5] = np.nan
    grids = []
    for k, b in enumerate([poly20k, poly20k, fast, fast, poly20k]):
        _announce(f"grid reuse call {k} n={b.n}")
        gpu = gpu_step(b, ctx)
        compare_step(b, gpu, oracle.step(b))
        grids.append((tuple(gpu[3]["nc"]), gpu[3]["rho_c"]))
        if k == 1:  # an invalid input on the same context fails and leaves no plan behind
            p = pc.Particles.from_box(bad)
            with pytest.raises(pc.PcolError) as ei:
                pc.pcol_step(ctx, p, bad.L, bad.dt, bad.e)
            assert ei.value.code == pc.PCOL_E_INVALID
    assert grids[0] == grids[1] == grids[4] and grids[2] == grids[3] and grids[0] != grids[2]


@pytest.mark.parametrize("opts", [{"filter": 1}, {"order": 1}], ids=["fp32", "literal"])
def test_steps_in_lockstep_on_one_context(poly20k, opts):
    """Six steps of the polydisperse box on one context (each call's binning tries the
    last call's grid) through the binary32 filter and through the literal order, every
    step against the oracle's step from the oracle's previous state, bitwise."""
    ctx = pc.Context(poly20k.n, pc.pcol_default_opts(**opts))
    p = pc.Particles.from_box(poly20k)
    partner = torch.empty(poly20k.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(poly20k.n, dtype=torch.float64, device="cuda")
    b = poly20k
    for k in range(6):
        _announce(f"lockstep {opts} step {k} n={b.n}")
        st = pc.pcol_step(ctx, p, b.L, b.dt, b.e, partner, tcoll)
        torch.cuda.synchronize()
        orc = oracle.step_sequential(b) if opts.get("order") else oracle.step(b)
        gpu = (to_host(p), partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st)
        assert orc.n_pairs > 0 and st["n_pairs"] == orc.n_pairs
        assert compare_step(b, gpu, orc) == 0
        b = workloads.Box(orc.x, orc.y, orc.z, orc.vx, orc.vy, orc.vz, b.r, b.m, b.L, b.dt, b.e)


def test_error_codes_leave_inputs_unchanged():
    box = workloads.config(1)
    ctx = pc.Context(box.n)

    def expect(code, mutate=None, dt=None, e=None, **kw):
        b = box.copy()
        if mutate:
            mutate(b)
        p = pc.Particles.from_box(b)
        before = [t.clone() for t in p.tensors()]
        with pytest.raises(pc.PcolError) as ei:
            pc.pcol_step(ctx, p, b.L, b.dt if dt is None else dt, b.e if e is None else e)
        assert ei.value.code == code
        if code != pc.PCOL_E_SWEEPS:
            for t0, t1 in zip(before, p.tensors()):
                assert torch.equal(t0.view(torch.int64), t1.view(torch.int64))

    expect(pc.PCOL_E_INVALID, lambda b: b.vx.__setitem__(3, np.nan))
    expect(pc.PCOL_E_INVALID, lambda b: b.r.__setitem__(4, 0.0))
    expect(pc.PCOL_E_INVALID, lambda b: b.m.__setitem__(5, -1.0))
    expect(pc.PCOL_E_INVALID, lambda b: b.x.__setitem__(6, b.L[0]))
    expect(pc.PCOL_E_INVALID, lambda b: b.z.__setitem__(7, -1e-300))
    expect(pc.PCOL_E_INVALID, e=1.5)
    expect(pc.PCOL_E_INVALID, dt=-1.0)
    expect(pc.PCOL_E_BOX, dt=0.2)
    ctx2 = pc.Context(box.n, pc.pcol_default_opts(max_sweeps=1))
    p = pc.Particles.from_box(box)
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_step(ctx2, p, box.L, box.dt, box.e)
    assert ei.value.code == pc.PCOL_E_SWEEPS
    # detect before any bin, and n above n_max
    ctx3 = pc.Context(box.n)
    p = pc.Particles.from_box(box)
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_detect(ctx3, p, box.L, box.dt)
    assert ei.value.code == pc.PCOL_E_STATE
    small = pc.Context(10)
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_step(small, p, box.L, box.dt, box.e)
    assert ei.value.code == pc.PCOL_E_INVALID


# ---------------------------------------------------------------- FP32 filter + FP64 recheck form


@pytest.mark.parametrize("flt", [1])
@pytest.mark.parametrize("which", ["config1", "config2", "poly20k", "small"])
def test_filter_forms_match_oracle(which, flt, cfg2, poly20k):
    """The binary32 filter (1) passes every pair the binary64 rule can keep and
    its survivors are decided in binary64, so pair sets, times and states equal
    the oracle's exactly."""
    if which == "config1":
        box = workloads.config(1)
    elif which == "config2":
        box = cfg2
    elif which == "poly20k":
        box = poly20k
    else:
        box = workloads.make_box(250, seed=5, phi=0.3, radius=0.5, e=0.85, dt=0.25)
    _announce(f"filter {flt} form {which}")
    gpu = gpu_step(box, filter=flt)
    orc = oracle.step(box)
    assert compare_step(box, gpu, orc) == 0
    st = gpu[3]
    if min(st["nc"]) >= 3:
        assert st["n_recheck"] >= orc.n_pairs
        if flt == 1:
            assert st["band"] >= 1e-4


@pytest.mark.parametrize("flt", [1])
@pytest.mark.parametrize("q", [0.0, 0.99])
def test_filter_forms_equal_plain_form_bitwise(poly20k, flt, q):
    a = gpu_step(poly20k, split_quantile=q)
    b = gpu_step(poly20k, filter=flt, split_quantile=q)
    for f in FIELDS:
        assert np.array_equal(a[0][f].view(np.uint64), b[0][f].view(np.uint64))
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2], equal_nan=True)
    assert a[3]["contacts"] == b[3]["contacts"]


@pytest.mark.parametrize("flt", [0, 1])
def test_home_cells_per_workgroup_invariance(poly20k, flt):
    """opts.home_cells (consecutive home cells per workgroup of the pair test) does
    not change any result bit, and pcol_stats reports the value used."""
    a = gpu_step(poly20k, filter=flt)
    ncell = a[3]["nc"][0] * a[3]["nc"][1] * a[3]["nc"][2]
    assert a[3]["home_cells"] == (4 if poly20k.n < 24 * ncell else 1)  # automatic choice
    for hc in (1, 2, 3, 8, 16):
        b = gpu_step(poly20k, filter=flt, home_cells=hc)
        assert b[3]["home_cells"] == hc
        for f in FIELDS:
            assert np.array_equal(a[0][f].view(np.uint64), b[0][f].view(np.uint64))
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2], equal_nan=True)
        assert a[3]["pair_tests"] == b[3]["pair_tests"]


def _chain(n=40, lines=1):
    """Spheres on a line, each closing on its right neighbour at the same speed with
    gaps shrinking to the right: every sphere's earliest partner is its right
    neighbour, so only the last pair is mutual, and each sweep resolves one pair
    from the right end: n/2 pairs in n/2 sweeps plus one that finds none.  lines
    copies of the chain sit on a square grid of (y, z), 8 apart (beyond the reach)."""
    gap = 0.05 - 0.001 * np.arange(n - 1)
    x1 = 10.0 + np.concatenate([[0.0], np.cumsum(1.0 + gap)])
    side = int(np.ceil(np.sqrt(lines)))
    k = np.arange(lines)
    y = np.repeat(4.0 + 8.0 * (k % side), n)
    z = np.repeat(4.0 + 8.0 * (k // side), n)
    x = np.tile(x1, lines)
    vx = np.tile(-0.01 * np.arange(n), lines)
    m = n * lines
    return workloads.Box(x, y, z, vx, np.zeros(m), np.zeros(m), np.full(m, 0.5), np.ones(m),
                         (400.0, 400.0, 400.0), 6.0, 0.9)


@pytest.mark.parametrize("lines", [1, 2500])
def test_sweeps_beyond_one_device_group(lines):
    """21 sweeps against the oracle.  One chain: a short list, one sweep per host
    round trip.  2,500 chains (95,000 spheres listed after sweep 1): the later sweeps
    run on the device in several groups (the first group's last check leaves the
    step unfinished, the host re-arms and queues more).  Then the sweep cap at and
    before the last pairing sweep."""
    box = _chain(lines=lines)
    _announce(f"sweep chains n={box.n}")
    gpu = gpu_step(box)
    orc = oracle.step(box)
    assert compare_step(box, gpu, orc) == 0
    st = gpu[3]
    assert st["nc"][0] >= 3 and st["n_pairs"] == 20 * lines and st["n_sweeps"] == 21
    assert orc.n_pairs == 20 * lines and orc.n_sweeps == 21
    # a cap that the last sweep (no pairs) meets is fine; one that the last pairing
    # sweep meets is an error, and the caller's arrays are left as they were
    gpu2 = gpu_step(box, max_sweeps=21)
    assert compare_step(box, gpu2, orc) == 0
    for cap in (20, 6, 2):
        ctx = pc.Context(box.n, pc.pcol_default_opts(max_sweeps=cap))
        p = pc.Particles.from_box(box)
        before = [t.clone() for t in p.tensors()]
        with pytest.raises(pc.PcolError) as ei:
            pc.pcol_step(ctx, p, box.L, box.dt, box.e)
        assert ei.value.code == pc.PCOL_E_SWEEPS, cap
        for t0, t1 in zip(before, p.tensors()):
            assert torch.equal(t0.view(torch.int64), t1.view(torch.int64)), cap


def test_step_cell_ordered_input(poly20k):
    """Spheres stored in cell order (consecutive spheres share a cell, so the binning takes
    one slot atomic per run of a wave): the step equals the oracle's."""
    box = poly20k
    L = np.array(box.L)
    key = [np.minimum(np.floor(getattr(box, f) / (L[a] / 8)), 7) for a, f in enumerate("xyz")]
    order = np.lexsort((box.x, key[0], key[1], key[2]))
    sb = workloads.Box(*[a[order].copy() for a in box.arrays()], box.L, box.dt, box.e,
                       box.name + " cell-ordered")
    _announce("cell-ordered poly20k")
    gpu = gpu_step(sb)
    assert compare_step(sb, gpu, oracle.step(sb)) == 0
