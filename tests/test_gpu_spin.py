"""pcol_step_spin (Coulomb friction and spin) on the GPU against the oracle's
orc_step_spin, element by element: pair set and contact times bit-exact, positions,
velocities and spins within 1e-12 relative (in practice bitwise)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_helpers import FIELDS, to_host
import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _spins(n, seed, scale):
    return np.random.default_rng(seed).normal(size=(3, n)) * scale


def gpu_step_spin(box, w, mu, ctx=None, **opts):
    p = pc.Particles.from_box(box)
    wt = [torch.as_tensor(np.ascontiguousarray(w[k]), dtype=torch.float64).cuda() for k in range(3)]
    if ctx is None:
        ctx = pc.Context(max(box.n, 1), pc.pcol_default_opts(**opts) if opts else None)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    st = pc.pcol_step_spin(ctx, p, wt, box.L, box.dt, box.e, mu, partner, tcoll)
    torch.cuda.synchronize()
    return (to_host(p), np.array([t.cpu().numpy() for t in wt]),
            partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st)


def compare_spin(gpu, orc, rel=1e-12):
    out, w, partner, tcoll, _ = gpu
    assert np.array_equal(partner, orc.partner), np.count_nonzero(partner != orc.partner)
    assert np.array_equal(tcoll, orc.tcoll, equal_nan=True)
    nonbit = 0
    pairs = list(zip(FIELDS, [out[f] for f in FIELDS])) + [("wx", w[0]), ("wy", w[1]), ("wz", w[2])]
    for f, a in pairs:
        b = getattr(orc, f)
        scale = max(1.0, float(np.max(np.abs(b)))) if b.size else 1.0
        err = np.max(np.abs(a - b)) / scale if a.size else 0.0
        assert err <= rel, f"{f}: max relative error {err:.3e}"
        nonbit += int(np.count_nonzero(a.view(np.uint64) != b.view(np.uint64)))
    return nonbit


@pytest.fixture(scope="module")
def poly20k():
    return workloads.make_box(20000, seed=13, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)


@pytest.mark.parametrize("which", ["config1", "poly20k"])
def test_zero_friction_equals_plain_step_bitwise(which, poly20k):
    box = workloads.config(1) if which == "config1" else poly20k
    _announce(f"spin mu=0 {which} n={box.n}")
    w = _spins(box.n, 3, 5.0)
    g = gpu_step_spin(box, w, 0.0)
    p = pc.Particles.from_box(box)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    pc.pcol_step(pc.Context(box.n), p, box.L, box.dt, box.e, partner)
    ref = to_host(p)
    for f in FIELDS:
        assert np.array_equal(g[0][f].view(np.uint64), ref[f].view(np.uint64)), f
    assert np.array_equal(g[1], w)
    assert np.array_equal(g[2], partner.cpu().numpy().astype(np.int64))


@pytest.mark.parametrize("which,mu", [("config1", 0.1), ("config1", 0.4), ("config1", 5.0),
                                      ("poly20k", 0.1), ("poly20k", 0.4), ("poly20k", 5.0),
                                      ("config2", 0.4)])
def test_spin_matches_oracle(which, mu, poly20k):
    box = poly20k if which == "poly20k" else workloads.config(1 if which == "config1" else 2)
    _announce(f"spin {which} n={box.n} mu={mu}")
    w = _spins(box.n, 7, 2.0 / float(np.min(box.r)))
    g = gpu_step_spin(box, w, mu)
    orc = oracle.step_spin(box, w, mu)
    assert orc.n_pairs > 0 and g[4]["n_pairs"] == orc.n_pairs
    assert compare_spin(g, orc) == 0


@pytest.mark.parametrize("lines", [1, 2500])
def test_spin_over_many_sweeps(lines):
    """The sweep chains of test_gpu_step with spins: one sweep per round trip for one
    chain, device sweep groups for 2,500 chains; against the oracle."""
    from tests.test_gpu_step import _chain
    box = _chain(lines=lines)
    w = _spins(box.n, 9, 0.05)
    _announce(f"spin chains n={box.n}")
    g = gpu_step_spin(box, w, 0.3)
    orc = oracle.step_spin(box, w, 0.3)
    assert g[4]["n_sweeps"] == 21 and orc.n_sweeps == 21
    assert compare_spin(g, orc) == 0


@pytest.mark.parametrize("walls", [None, (1, 1, 1)], ids=["periodic", "walls"])
def test_spin_steps_in_lockstep_on_one_context(walls, poly20k):
    """Eight friction steps of the polydisperse box on one context (each call's
    binning tries the last call's grid), every step against the oracle's step from
    the oracle's previous state, positions, velocities and spins bitwise."""
    box, mu = poly20k, 0.4
    w = _spins(box.n, 11, 1.0 / float(np.min(box.r)))
    p = pc.Particles.from_box(box)
    wt = [torch.as_tensor(np.ascontiguousarray(w[k]), dtype=torch.float64).cuda() for k in range(3)]
    ctx = pc.Context(box.n)
    partner = torch.empty(box.n, dtype=torch.int32, device="cuda")
    tcoll = torch.empty(box.n, dtype=torch.float64, device="cuda")
    b, wo = box, w
    for k in range(8):
        _announce(f"spin lockstep {walls} step {k} n={box.n}")
        if walls is None:
            st = pc.pcol_step_spin(ctx, p, wt, b.L, b.dt, b.e, mu, partner, tcoll)
            orc = oracle.step_spin(b, wo, mu)
        else:
            st = pc.pcol_step_spin_walls(ctx, p, wt, b.L, walls, b.dt, b.e, mu, partner, tcoll)
            orc = oracle.step_walls_spin(b, walls, wo, mu)
        torch.cuda.synchronize()
        g = (to_host(p), np.array([t.cpu().numpy() for t in wt]),
             partner.cpu().numpy().astype(np.int64), tcoll.cpu().numpy(), st)
        assert orc.n_pairs > 0 and st["n_pairs"] == orc.n_pairs
        assert compare_spin(g, orc) == 0
        b = workloads.Box(orc.x, orc.y, orc.z, orc.vx, orc.vy, orc.vz, b.r, b.m, b.L, b.dt, b.e)
        wo = np.array([orc.wx, orc.wy, orc.wz])


def test_spin_errors_leave_inputs_unchanged():
    box = workloads.config(1)
    ctx = pc.Context(box.n)
    for mu, bad in ((-0.1, None), (float("nan"), None), (0.3, (1, 17))):
        w = _spins(box.n, 1, 1.0)
        if bad:
            w[bad] = np.inf
        p = pc.Particles.from_box(box)
        wt = [torch.as_tensor(np.ascontiguousarray(w[k])).cuda() for k in range(3)]
        before = [t.clone() for t in p.tensors()] + [t.clone() for t in wt]
        with pytest.raises(pc.PcolError) as ei:
            pc.pcol_step_spin(ctx, p, wt, box.L, box.dt, box.e, mu)
        assert ei.value.code == pc.PCOL_E_INVALID
        for t0, t1 in zip(before, list(p.tensors()) + wt):
            assert torch.equal(t0.view(torch.int64), t1.view(torch.int64))
