"""bench.py's command line on a machine without a GPU: more than one GPU is refused
with a message before anything is imported or measured."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_help_lists_every_leg_switch():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0
    for flag in ("--no-batched", "--no-adjoint", "--no-friction", "--no-walls", "--no-deposition",
                 "--no-cell-order", "--no-literal",
                 "--no-cpu-baseline", "--steps", "--warmup", "--gpus"):
        assert flag in res.stdout, flag


def test_reference_grid_pair_count_equals_the_oracles():
    """bench.py's pair-test count on the reference grid (cells of the reach, the 27
    around each sphere, unordered pairs of active spheres) equals the number of
    candidate pairs the oracle's grid search visits, with and without a mask."""
    import numpy as np
    import oracle
    import workloads
    sys.path.insert(0, ROOT)
    from bench import ref_grid_pair_tests
    box = workloads.make_box(20_000, seed=11, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8)
    reach = oracle.step(box).reach
    for act in (None, (np.arange(box.n) % 3 != 0).astype(np.uint8)):
        _, _, tests = oracle.earliest(box, act)
        assert ref_grid_pair_tests(box.x, box.y, box.z, box.L, reach, act) == tests
