"""GPU parity at the benchmark's full size: 16,000,000 polydisperse spheres at
volume fraction 0.3 (lognormal radii, e = 0.8, dt = 0.4), in the launch
configuration bench.py times.

The plain step is compared with the oracle's whole step (about a minute on
the host's cores, run as a test of its own) element by element, in both filter forms: pair set and contact
times bitwise, states within 1e-12 relative (in fact bitwise), the pair and
sweep counts equal; pcol_detect's keys with the oracle's earliest partners of
all 16M spheres.  Properties that hold at any size are checked beside them
(momentum conservation, the closed-form energy loss per pair).  The friction and
walls steps at this size are checked on sampled pairs and by properties; both
are compared whole with the oracle at 1M in their own tests.  Each test keeps
one oracle computation, so no test runs silent for minutes.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_helpers import compare_step

pytestmark = pytest.mark.gpu

import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)

FIELDS = ("x", "y", "z", "vx", "vy", "vz")


@pytest.fixture(scope="module")
def big(box16m):
    return box16m, pc.Particles.from_box(box16m)


@pytest.fixture(scope="module")
def big_oracle(big):
    box, _ = big
    print("[gpu-test] oracle step at 16M", flush=True)
    return oracle.step(box)


@pytest.mark.timeout(900)
def test_16M_oracle_step(big_oracle):
    """The oracle's whole 16M step (its own test: about a minute on the host's cores),
    which the comparisons below use."""
    orc = big_oracle
    hit = orc.partner >= 0
    assert orc.n_pairs * 2 == int(hit.sum()) and orc.n_pairs > 1_000_000
    assert np.array_equal(orc.partner[orc.partner[hit]], np.where(hit)[0])
    assert np.array_equal(orc.tcoll[hit], orc.tcoll[orc.partner[hit]])


def _step(box, p0, flt):
    p = p0.clone()
    ctx = pc.Context(box.n, pc.pcol_default_opts(filter=flt))
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step(ctx, p, box.L, box.dt, box.e, partner, tcoll)
    torch.cuda.synchronize()
    out = {f: getattr(p, f).cpu().numpy() for f in FIELDS}
    ctx.close()
    del p
    return out, partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st


@pytest.mark.timeout(900)
def test_16M_workload(big):
    """The generated input: 16M spheres inside the box, no two overlapping (sampled
    against the oracle's neighbour search: a pair that overlaps has no contact time,
    so overlap is checked directly on the nearest neighbours of sampled spheres)."""
    box, p0 = big
    L = np.array(box.L)
    for f, a in (("x", 0), ("y", 1), ("z", 2)):
        v = getattr(box, f)
        assert np.all(v >= 0.0) and np.all(v < L[a])
    assert np.all(box.r >= 0.5) and np.all(box.r <= 2.0)
    assert np.allclose(box.m, box.r ** 3, rtol=0, atol=0)
    phi = math.fsum(4.0 / 3.0 * math.pi * box.r ** 3) / float(np.prod(L))
    assert phi == pytest.approx(0.3, rel=1e-9)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("flt", [0, 1])
def test_16M_step_equals_oracle(big, big_oracle, flt):
    """The whole 16M step against the oracle's: every partner, every contact time
    bitwise, every state within 1e-12 relative and in fact bitwise; pair and sweep
    counts equal.  Filter 1 (binary32 with the binary64 recheck) is the precision
    form: its pair-set mismatch against the binary64 oracle must be zero."""
    box, p0 = big
    orc = big_oracle
    print(f"[gpu-test] 16M step, filter {flt}", flush=True)
    gpu = _step(box, p0, flt)
    out, partner, tcoll, st = gpu
    assert compare_step(box, gpu, orc) == 0
    assert st["n_pairs"] == orc.n_pairs and st["n_pairs"] > 1_000_000
    assert st["n_sweeps"] == orc.n_sweeps
    if flt == 1:
        assert st["n_recheck"] > 0 and st["band"] >= 1e-4

    if flt == 0:
        # properties beside the comparison: momentum conserved; kinetic energy lost
        # exactly as the closed form per pair
        hit = partner >= 0
        m = box.m
        for f in ("vx", "vy", "vz"):
            p_in = math.fsum(m * getattr(box, f))
            p_out = math.fsum(m * out[f])
            assert abs(p_out - p_in) <= 1e-10 * math.fsum(m * np.abs(getattr(box, f)))
        ke = lambda vx, vy, vz: 0.5 * math.fsum(m * (vx * vx + vy * vy + vz * vz))
        loss = ke(box.vx, box.vy, box.vz) - ke(out["vx"], out["vy"], out["vz"])
        L = np.array(box.L)
        pairs = np.where(hit & (np.arange(box.n) < partner))[0]
        i, j = pairs, partner[pairs]
        d = np.stack([getattr(box, f)[j] - getattr(box, f)[i] for f in ("x", "y", "z")], 1)
        d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
        u = np.stack([getattr(box, f)[j] - getattr(box, f)[i] for f in ("vx", "vy", "vz")], 1)
        w = d + tcoll[i][:, None] * u
        g = np.sum(u * w, 1) / (box.r[i] + box.r[j])
        mr = m[i] * m[j] / (m[i] + m[j])
        expect = math.fsum(0.5 * (1 - box.e ** 2) * mr * g * g)
        assert loss == pytest.approx(expect, rel=1e-9)


@pytest.mark.timeout(900)
def test_16M_detect_keys_equal_oracle(big):
    """pcol_detect over all 16M spheres (all active) against the oracle's earliest
    partner of every sphere: partner index and exact contact time bitwise, and the
    key's packed binary32 time."""
    box, p0 = big
    n = box.n
    print("[gpu-test] 16M detect keys", flush=True)
    ctx = pc.Context(n)
    pc.pcol_bin(ctx, p0, box.L, box.dt)
    key, tmin = pc.pcol_detect(ctx, p0, box.L, box.dt)
    torch.cuda.synchronize()
    key = key.cpu().numpy().view(np.uint64)
    tmin = tmin.cpu().numpy()
    ctx.close()
    print("[gpu-test] oracle earliest partners at 16M", flush=True)
    op, ot, _ = oracle.earliest(box)
    none = np.uint64(2 ** 64 - 1)
    kj = np.where(key == none, -1, (key & np.uint64(0xFFFFFFFF)).astype(np.int64))
    assert np.array_equal(kj, op)
    assert np.array_equal(tmin, ot)
    has = op >= 0
    assert has.sum() > 4_000_000
    tf = (key[has] >> np.uint64(32)).astype(np.uint32).view(np.float32)
    assert np.array_equal(tf, ot[has].astype(np.float32))


@pytest.mark.timeout(900)
def test_16M_friction_and_spin_sampled(big):
    """pcol_step_spin at 16M (mu 0.3, spins N(0, 1) / r, as bench.py times it): the
    pair set and contact times equal the plain step's; spheres without a collision
    keep their spins; 300 sampled pairs equal the oracle's friction resolve bitwise;
    linear momentum is conserved."""
    box, p0 = big
    n, mu = box.n, 0.3
    rng = np.random.default_rng(17)
    w0 = np.stack([rng.normal(size=n) / box.r for _ in range(3)])
    print("[gpu-test] 16M step with friction and spin", flush=True)
    p = p0.clone()
    w = [torch.as_tensor(w0[k]).cuda() for k in range(3)]
    ctx = pc.Context(n)
    partner = torch.empty(n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step_spin(ctx, p, w, box.L, box.dt, box.e, mu, partner, tcoll)
    torch.cuda.synchronize()
    ctx.close()
    out = {f: getattr(p, f).cpu().numpy() for f in FIELDS}
    ws = np.stack([t.cpu().numpy() for t in w])
    partner, tcoll = partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy()
    del p, w
    _, partner0, tcoll0, st0 = _step(box, p0, 0)
    assert np.array_equal(partner, partner0) and st["n_pairs"] == st0["n_pairs"]
    assert np.array_equal(tcoll, tcoll0, equal_nan=True)
    hit = partner >= 0
    assert np.array_equal(ws[:, ~hit], w0[:, ~hit])
    assert np.count_nonzero(ws[:, hit] != w0[:, hit]) > st["n_pairs"]
    pairs = np.where(hit & (np.arange(n) < partner))[0]
    for i in rng.choice(pairs, 300, replace=False):
        j = partner[i]
        xs, vs, wsr = oracle.resolve_pair_spin(box, w0, mu, i, j, tcoll[i])
        for got, ref, names in ((out, xs, ("x", "y", "z")), (out, vs, ("vx", "vy", "vz"))):
            g = np.array([[got[f][i] for f in names], [got[f][j] for f in names]])
            assert np.array_equal(g, ref)
        assert np.array_equal(np.array([ws[:, i], ws[:, j]]), wsr)
    m = box.m
    for f in ("vx", "vy", "vz"):
        p_in = math.fsum(m * getattr(box, f))
        assert abs(math.fsum(m * out[f]) - p_in) <= 1e-10 * math.fsum(m * np.abs(getattr(box, f)))


def _reflect(p, L):
    """Free-flight end coordinate between walls at 0 and L (at most one plane crossed)."""
    flip = (p >= L) | (p < 0)
    q = np.where(p >= L, L - (p - L), np.where(p < 0, -p, p))
    q = np.where(q >= L, np.nextafter(L, 0.0), q)
    return q, flip


@pytest.mark.timeout(900)
def test_16M_walls_properties(big):
    """pcol_step_walls at 16M with walls on x and z (the oracle's walls step is too slow at
    this size): mutual pairs with bitwise-symmetric times, every contact no later than both
    centres' times of flight to a wall, the reflected free flight of every sphere without
    a collision exactly, y periodic, momentum along y conserved, positions inside."""
    box, p0 = big
    n, walls = box.n, (1, 0, 1)
    print("[gpu-test] 16M step between walls", flush=True)
    p = p0.clone()
    ctx = pc.Context(n)
    partner = torch.empty(n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step_walls(ctx, p, box.L, walls, box.dt, box.e, partner, tcoll)
    torch.cuda.synchronize()
    ctx.close()
    out = {f: getattr(p, f).cpu().numpy() for f in FIELDS}
    partner, tcoll = partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy()
    del p
    hit = partner >= 0
    assert st["n_pairs"] * 2 == int(hit.sum()) and st["n_pairs"] > 1_000_000
    assert np.array_equal(partner[partner[hit]], np.where(hit)[0])
    assert np.array_equal(tcoll[hit], tcoll[partner[hit]])
    L = np.array(box.L)
    tof = np.full(n, np.inf)
    for a, (f, v) in enumerate((("x", box.vx), ("y", box.vy), ("z", box.vz))):
        if not walls[a]:
            continue
        x = getattr(box, f)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(v > 0, (L[a] - x) / v, np.where(v < 0, -x / v, np.inf))
        tof = np.minimum(tof, t)
    i = np.where(hit)[0]
    assert np.all(tcoll[i] <= tof[i]) and np.all(tcoll[i] <= tof[partner[i]])
    for a, (f, vf) in enumerate((("x", "vx"), ("y", "vy"), ("z", "vz"))):
        x0, v0 = getattr(box, f)[~hit], getattr(box, vf)[~hit]
        x1 = x0 + box.dt * v0
        if walls[a]:
            x1, flip = _reflect(x1, L[a])
            v1 = np.where(flip, -v0, v0)
            assert flip.sum() > 1000
        else:
            x1 = np.where(x1 >= L[a], x1 - L[a], np.where(x1 < 0, x1 + L[a], x1))
            x1 = np.where(x1 >= L[a], 0.0, x1)
            v1 = v0
        assert np.array_equal(out[f][~hit], x1) and np.array_equal(out[vf][~hit], v1)
        assert np.all(out[f] >= 0.0) and np.all(out[f] < L[a])
    m = box.m
    p_in = math.fsum(m * box.vy)
    assert abs(math.fsum(m * out["vy"]) - p_in) <= 1e-10 * math.fsum(m * np.abs(box.vy))
