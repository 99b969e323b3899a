"""GPU tests of the extent split: spheres whose extent r + |v| dt lies above a
quantile are binned into a second cell layer and searched separately, so the
first layer's cells need only twice the quantile extent.  The step must equal
the oracle's (which has no split) bitwise, for any quantile, on boxes with few
and with many wide spheres, through the slot-overflow and masked-detect paths
(which search both layers) and in the FP32 filter form."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_helpers import FIELDS, compare_step, gpu_step

pytestmark = pytest.mark.gpu

import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def poly():
    return workloads.make_box(30000, seed=17, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)


@pytest.fixture(scope="module")
def fast_tail():
    """Monodisperse box where 4% of the spheres move 5x faster: a heavy wide tail."""
    box = workloads.make_box(40000, seed=19, phi=0.2, radius=1.0, e=0.9, dt=0.2)
    pick = np.random.default_rng(19).random(box.n) < 0.04
    for f in ("vx", "vy", "vz"):
        v = getattr(box, f)
        v[pick] *= 5.0
    return box


def test_split_matches_oracle_and_is_used(poly):
    _announce(f"split poly n={poly.n}")
    gpu = gpu_step(poly)
    st = gpu[3]
    assert st["n_wide"] > 0 and st["rho_c"] > 0
    assert 2 * st["rho_c"] < 0.85 * st["reach"]
    orc = oracle.step(poly)
    assert compare_step(poly, gpu, orc) == 0
    assert st["n_pairs"] == orc.n_pairs and st["n_sweeps"] == orc.n_sweeps


def test_split_quantile_invariance(poly):
    """Every quantile (and no split) gives the same step bitwise; with one contact
    slot most spheres overflow into the exact search of both layers."""
    ref = gpu_step(poly, split_quantile=0.0)
    assert ref[3]["n_wide"] == 0
    for q in (0.5, 0.9, 0.99, 0.999):
        for slots in (12, 1):
            got = gpu_step(poly, split_quantile=q, contact_slots=slots)
            for f in FIELDS:
                assert np.array_equal(got[0][f].view(np.uint64), ref[0][f].view(np.uint64)), (q, f)
            assert np.array_equal(got[1], ref[1]), q
            assert np.array_equal(got[2], ref[2], equal_nan=True), q
            if q <= 0.99:
                assert got[3]["n_wide"] > 0


def test_split_heavy_fast_tail(fast_tail):
    box = fast_tail
    _announce(f"split fast tail n={box.n}")
    gpu = gpu_step(box)
    st = gpu[3]
    assert st["n_wide"] > 0
    orc = oracle.step(box)
    assert compare_step(box, gpu, orc) == 0
    # the same tail at a quantile that puts all fast spheres in the second layer
    gpu2 = gpu_step(box, split_quantile=0.9)
    assert gpu2[3]["n_wide"] >= 0.04 * box.n * 0.9
    assert compare_step(box, gpu2, orc) == 0
    # and in the binary32 filter form
    for flt in (1,):
        gpu3 = gpu_step(box, filter=flt, split_quantile=0.9)
        assert compare_step(box, gpu3, orc) == 0


def test_split_detect_keys_all_active_and_masked(fast_tail):
    box = fast_tail
    p = pc.Particles.from_box(box)
    ctx = pc.Context(box.n, pc.pcol_default_opts(split_quantile=0.9))
    pc.pcol_bin(ctx, p, box.L, box.dt)
    key, tmin = pc.pcol_detect(ctx, p, box.L, box.dt)
    torch.cuda.synchronize()
    key = key.cpu().numpy().view(np.uint64)
    op, ot, _ = oracle.earliest(box)
    has = op >= 0
    assert np.array_equal((key[has] & np.uint64(0xFFFFFFFF)).astype(np.int64), op[has])
    assert np.all(key[~has] == np.uint64(2 ** 64 - 1))
    assert np.array_equal(tmin.cpu().numpy(), ot)
    act = (np.random.default_rng(4).random(box.n) < 0.5).astype(np.uint8)
    key2, tmin2 = pc.pcol_detect(ctx, p, box.L, box.dt, active=torch.from_numpy(act).cuda())
    torch.cuda.synchronize()
    op2, ot2, _ = oracle.earliest(box, active=act)
    key2 = key2.cpu().numpy().view(np.uint64)
    has2 = op2 >= 0
    assert np.array_equal((key2[has2] & np.uint64(0xFFFFFFFF)).astype(np.int64), op2[has2])
    assert np.all(key2[~has2] == np.uint64(2 ** 64 - 1))
    assert np.array_equal(tmin2.cpu().numpy(), ot2)
    # pcol_detect with another dt than the binning is refused
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_detect(ctx, p, box.L, box.dt * 2)
    assert ei.value.code == pc.PCOL_E_STATE
