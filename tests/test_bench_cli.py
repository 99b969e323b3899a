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
    for flag in ("--no-batched", "--no-adjoint", "--no-friction", "--no-walls", "--no-deposition", "--no-cell-order",
                 "--no-cpu-baseline", "--steps", "--warmup", "--gpus"):
        assert flag in res.stdout, flag
