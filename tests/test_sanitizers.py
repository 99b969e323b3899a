"""Host AddressSanitizer and UndefinedBehaviorSanitizer over the oracle and the input
generator: both C libraries are rebuilt with -fsanitize=address,undefined (every
error fatal) and the oracle's pins run against those builds in a child process
with the AddressSanitizer runtime preloaded.  Any out-of-bounds access, use after
free or undefined behaviour in the oracle's step, its friction, walls, deposition,
literal-order and derivative functions, or in the generator's placement, fails the
test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
         "-fPIC", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


@pytest.mark.slow
def test_oracle_and_generator_pins_under_asan_and_ubsan(tmp_path):
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    orc = tmp_path / "liboracle_san.so"
    gen = tmp_path / "libwlgen_san.so"
    subprocess.check_call(["gcc", *FLAGS, os.path.join(ROOT, "oracle", "pcol_oracle.c"), "-o",
                           str(orc), "-lm"])
    subprocess.check_call(["gcc", *FLAGS, os.path.join(ROOT, "workloads", "gen.c"), "-o", str(gen),
                           "-lm"])
    env = dict(os.environ, PCOL_ORACLE_LIB=str(orc), PCOL_WLGEN_LIB=str(gen), LD_PRELOAD=libasan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    files = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          "-m", "not gpu", *files], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=1500)
    tail = (res.stdout[-4000:] + res.stderr[-4000:])
    assert res.returncode == 0, tail
    assert "passed" in res.stdout and "AddressSanitizer" not in tail and "runtime error" not in tail
