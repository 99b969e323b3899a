"""pcol oracle -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU statement of the deterministic hard-sphere collision step
(``pcol_oracle.c``; every function there cites the paper passage it follows).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library neither calls nor links
it, and the two share no code.

Pins of this oracle against the paper and the mathematics are in
``tests/test_oracle_pins.py``; the forward-mode derivative ``step_jvp`` is
pinned in ``tests/test_oracle_jvp.py``, the per-sphere search
``earliest_subset`` in ``tests/test_oracle_subset.py``, and the friction,
walls, deposition and literal-order functions in their own
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "pcol_oracle.c")]
# PCOL_ORACLE_LIB: another build of pcol_oracle.c to load (the sanitizer test
# loads an AddressSanitizer / UndefinedBehaviorSanitizer build this way)
_LIB = os.environ.get("PCOL_ORACLE_LIB") or os.path.join(_HERE, "libpcol_oracle.so")
_lib = None

OK, E_INVALID, E_BOX, E_NOMEM, E_SWEEPS = 0, 1, 2, 3, 5

_FLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FMA contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_FLAGS, *_SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_sweeps", ctypes.c_int64),
                ("pair_tests", ctypes.c_int64), ("reach", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.orc_pair_time.argtypes = [_D, _D, ctypes.c_double, _D, _D, ctypes.c_double, _D,
                                      ctypes.c_double, _D]
        lib.orc_pair_time.restype = ctypes.c_int
        lib.orc_earliest.argtypes = [ctypes.c_int64] + [_D] * 7 + [_D, ctypes.c_double, _U8,
                                                                  ctypes.c_int, ctypes.c_double,
                                                                  _I64, _D, _I64]
        lib.orc_earliest.restype = ctypes.c_int
        lib.orc_earliest_subset.argtypes = [ctypes.c_int64] + [_D] * 7 + [_D, ctypes.c_double, _U8,
                                                                         ctypes.c_int64, _I64, _I64, _D]
        lib.orc_earliest_subset.restype = ctypes.c_int
        lib.orc_step_jvp.argtypes = [ctypes.c_int64] + [_D] * 8 + [_D, ctypes.c_double,
                                                                  ctypes.c_double] + [_D] * 6 + \
            [ctypes.c_double] + [_D] * 12 + [_I64]
        lib.orc_step_jvp.restype = ctypes.c_int
        lib.orc_resolve_pair.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double] + [_D] * 8 + \
            [_D, ctypes.c_double, ctypes.c_double] + [_D] * 6
        lib.orc_resolve_pair.restype = None
        lib.orc_step.argtypes = [ctypes.c_int64] + [_D] * 8 + [_D, ctypes.c_double, ctypes.c_double,
                                                              ctypes.c_int, ctypes.c_double,
                                                              ctypes.c_int] + [_D] * 6 + \
            [_I64, _D, _I32, ctypes.POINTER(_Stats)]
        lib.orc_step.restype = ctypes.c_int
        lib.orc_step_spin.argtypes = [ctypes.c_int64] + [_D] * 11 + [
            _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
            ctypes.c_int] + [_D] * 9 + [_I64, _D, _I32, ctypes.POINTER(_Stats)]
        lib.orc_step_spin.restype = ctypes.c_int
        lib.orc_resolve_pair_spin.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double] + \
            [_D] * 11 + [_D, ctypes.c_double, ctypes.c_double, ctypes.c_double] + [_D] * 9
        lib.orc_resolve_pair_spin.restype = None
        lib.orc_step_sequential.argtypes = [ctypes.c_int64] + [_D] * 8 + [
            _D, ctypes.c_double, ctypes.c_double, ctypes.c_double] + [_D] * 6 + [
            _I64, _D, ctypes.POINTER(_Stats)]
        lib.orc_step_sequential.restype = ctypes.c_int
        lib.orc_step_walls.argtypes = [ctypes.c_int64] + [_D] * 8 + [
            _D, _I32, ctypes.c_double, ctypes.c_double] + [_D] * 6 + [
            _I64, _D, ctypes.POINTER(_Stats)]
        lib.orc_step_walls.restype = ctypes.c_int
        lib.orc_step_walls_spin.argtypes = [ctypes.c_int64] + [_D] * 11 + [
            _D, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_double] + [_D] * 9 + [
            _I64, _D, ctypes.POINTER(_Stats)]
        lib.orc_step_walls_spin.restype = ctypes.c_int
        lib.orc_deposit.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), _D, _D]
        lib.orc_deposit.restype = ctypes.c_int
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}")
        self.code = code


def max_threads() -> int:
    """Threads the oracle's parallel loops run on (OpenMP)."""
    return int(_load().orc_max_threads())


def pair_time(xi, vi, ri, xj, vj, rj, L, dt):
    """Contact time of one pair within [0, dt] or None (eq. detect1/detect2)."""
    a = [_c64(v) for v in (xi, vi, xj, vj, L)]
    t = ctypes.c_double(0.0)
    hit = _load().orc_pair_time(_d(a[0]), _d(a[1]), float(ri), _d(a[2]), _d(a[3]), float(rj),
                                _d(a[4]), float(dt), ctypes.byref(t))
    return t.value if hit else None


def earliest(box, active=None, *, grid: bool = True, cell_mult: float = 1.0):
    """Earliest partner (index or -1) and its contact time for every active sphere."""
    n = box.n
    partner = np.empty(n, dtype=np.int64)
    tmin = np.empty(n, dtype=np.float64)
    tests = ctypes.c_int64(0)
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r)]
    act = None
    if active is not None:
        act = np.ascontiguousarray(active, dtype=np.uint8)
    L = _c64(box.L)
    rc = _load().orc_earliest(n, *[_d(a) for a in arrs], _d(L), float(box.dt),
                              act.ctypes.data_as(_U8) if act is not None else None, int(grid),
                              float(cell_mult), partner.ctypes.data_as(_I64), _d(tmin),
                              ctypes.byref(tests))
    if rc:
        raise OracleError(rc)
    return partner, tmin, tests.value


def earliest_subset(box, idx, active=None):
    """Earliest partner and time of the spheres idx only (same rule as earliest)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    partner = np.empty(idx.shape[0], dtype=np.int64)
    tmin = np.empty(idx.shape[0], dtype=np.float64)
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r)]
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    L = _c64(box.L)
    rc = _load().orc_earliest_subset(box.n, *[_d(a) for a in arrs], _d(L), float(box.dt),
                                     act.ctypes.data_as(_U8) if act is not None else None,
                                     idx.shape[0], idx.ctypes.data_as(_I64),
                                     partner.ctypes.data_as(_I64), _d(tmin))
    if rc:
        raise OracleError(rc)
    return partner, tmin


@dataclass
class StepResult:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    partner: np.ndarray   # int64, -1 = no collision
    tcoll: np.ndarray     # contact time within the step, NaN = none
    sweep: np.ndarray     # int32 sweep index of the collision, -1 = none
    n_pairs: int
    n_sweeps: int
    pair_tests: int
    reach: float


def step(box, *, e: float | None = None, grid: bool = True, cell_mult: float = 1.0,
         max_sweeps: int = 0) -> StepResult:
    """One collision step of ``box`` (a workloads.Box); inputs are not modified."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r, box.m)]
    outs = [np.empty(n) for _ in range(6)]
    partner = np.empty(n, dtype=np.int64)
    tcoll = np.empty(n)
    sweep = np.empty(n, dtype=np.int32)
    st = _Stats()
    L = _c64(box.L)
    rc = _load().orc_step(n, *[_d(a) for a in arrs], _d(L), float(box.dt),
                          float(box.e if e is None else e), int(grid), float(cell_mult),
                          int(max_sweeps), *[_d(o) for o in outs], partner.ctypes.data_as(_I64),
                          _d(tcoll), sweep.ctypes.data_as(_I32), ctypes.byref(st))
    if rc:
        raise OracleError(rc)
    return StepResult(*outs, partner, tcoll, sweep, st.n_pairs, st.n_sweeps, st.pair_tests,
                      st.reach)


@dataclass
class SpinStepResult(StepResult):
    wx: np.ndarray = None
    wy: np.ndarray = None
    wz: np.ndarray = None


def step_spin(box, w, mu: float, *, e: float | None = None, grid: bool = True,
              cell_mult: float = 1.0, max_sweeps: int = 0) -> SpinStepResult:
    """One collision step of ``box`` with angular velocities ``w`` (shape (3, n))
    and Coulomb friction ``mu``; inputs are not modified."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, w[0], w[1], w[2],
                              box.r, box.m)]
    outs = [np.empty(n) for _ in range(9)]
    partner = np.empty(n, dtype=np.int64)
    tcoll = np.empty(n)
    sweep = np.empty(n, dtype=np.int32)
    st = _Stats()
    L = _c64(box.L)
    rc = _load().orc_step_spin(n, *[_d(a) for a in arrs], _d(L), float(box.dt),
                               float(box.e if e is None else e), float(mu), int(grid),
                               float(cell_mult), int(max_sweeps), *[_d(o) for o in outs],
                               partner.ctypes.data_as(_I64), _d(tcoll), sweep.ctypes.data_as(_I32),
                               ctypes.byref(st))
    if rc:
        raise OracleError(rc)
    return SpinStepResult(*outs[:6], partner, tcoll, sweep, st.n_pairs, st.n_sweeps,
                          st.pair_tests, st.reach, *outs[6:9])


def resolve_pair_spin(box, w, mu: float, i: int, j: int, t: float, *, e: float | None = None):
    """New (x, v, w) of spheres i and j after their collision at time t, with friction
    mu (arrays of shape (2, 3))."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, w[0], w[1], w[2],
                              box.r, box.m)]
    outs = [np.zeros(n) for _ in range(9)]
    L = _c64(box.L)
    _load().orc_resolve_pair_spin(int(i), int(j), float(t), *[_d(a) for a in arrs], _d(L),
                                  float(box.dt), float(box.e if e is None else e), float(mu),
                                  *[_d(o) for o in outs])
    pick = lambda ks: np.array([[outs[k][i] for k in ks], [outs[k][j] for k in ks]])
    return pick(range(3)), pick(range(3, 6)), pick(range(6, 9))


def step_jvp(box, dx, dv, de: float, *, e: float | None = None):
    """One step and its forward-mode derivative along (dx, dv, de), pair set fixed.

    dx, dv: arrays of shape (3, n).  Returns (StateTuple x, v as (3, n) arrays,
    tangent tx, tv as (3, n) arrays, partner)."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r, box.m)]
    tin = [_c64(a) for a in (dx[0], dx[1], dx[2], dv[0], dv[1], dv[2])]
    outs = [np.empty(n) for _ in range(12)]
    partner = np.empty(n, dtype=np.int64)
    L = _c64(box.L)
    rc = _load().orc_step_jvp(n, *[_d(a) for a in arrs], _d(L), float(box.dt),
                              float(box.e if e is None else e), *[_d(a) for a in tin], float(de),
                              *[_d(o) for o in outs], partner.ctypes.data_as(_I64))
    if rc:
        raise OracleError(rc)
    return (np.array(outs[0:3]), np.array(outs[3:6]), np.array(outs[6:9]), np.array(outs[9:12]),
            partner)


def resolve_pair(box, i: int, j: int, t: float, *, e: float | None = None):
    """New (x, v) of spheres i and j after their collision at time t (arrays of shape (2, 3))."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r, box.m)]
    outs = [np.zeros(n) for _ in range(6)]
    L = _c64(box.L)
    _load().orc_resolve_pair(int(i), int(j), float(t), *[_d(a) for a in arrs], _d(L),
                             float(box.dt), float(box.e if e is None else e),
                             *[_d(o) for o in outs])
    xs = np.array([[outs[k][i] for k in range(3)], [outs[k][j] for k in range(3)]])
    vs = np.array([[outs[k][i] for k in range(3, 6)], [outs[k][j] for k in range(3, 6)]])
    return xs, vs


def deposit(x, y, z, a, nc, L):
    """Node sums of the linear corner deposition of a (shape (comp, n)) onto the periodic
    grid of nc cells per axis over the box L; returns shape (comp, nc2, nc1, nc0)."""
    a = np.ascontiguousarray(np.atleast_2d(np.asarray(a, dtype=np.float64)))
    comp, n = a.shape
    ncv = (ctypes.c_int * 3)(*[int(v) for v in nc])
    out = np.empty(comp * int(nc[0]) * int(nc[1]) * int(nc[2]))
    rc = _load().orc_deposit(n, _d(_c64(x)), _d(_c64(y)), _d(_c64(z)), _d(a), comp, ncv,
                             _d(_c64(L)), _d(out))
    if rc:
        raise OracleError(rc)
    return out.reshape(comp, int(nc[2]), int(nc[1]), int(nc[0]))


def step_sequential(box, *, e: float | None = None, cell_mult: float = 1.0) -> StepResult:
    """One step of ``box`` with the paper's collision order taken literally (elements
    along a Morton curve, first valid collision found, one pass); inputs unchanged."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r, box.m)]
    outs = [np.empty(n) for _ in range(6)]
    partner = np.empty(n, dtype=np.int64)
    tcoll = np.empty(n)
    st = _Stats()
    rc = _load().orc_step_sequential(n, *[_d(a) for a in arrs], _d(_c64(box.L)), float(box.dt),
                                     float(box.e if e is None else e), float(cell_mult),
                                     *[_d(o) for o in outs], partner.ctypes.data_as(_I64),
                                     _d(tcoll), ctypes.byref(st))
    if rc:
        raise OracleError(rc)
    sweep = np.where(partner >= 0, 0, -1).astype(np.int32)
    return StepResult(*outs, partner, tcoll, sweep, st.n_pairs, st.n_sweeps, st.pair_tests,
                      st.reach)


def step_walls(box, walls, *, e: float | None = None) -> StepResult:
    """One step of ``box`` with reflective walls on the axes where walls[k] is true (the
    others periodic); inputs unchanged."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, box.r, box.m)]
    outs = [np.empty(n) for _ in range(6)]
    partner = np.empty(n, dtype=np.int64)
    tcoll = np.empty(n)
    st = _Stats()
    wl = np.ascontiguousarray([1 if w else 0 for w in walls], dtype=np.int32)
    rc = _load().orc_step_walls(n, *[_d(a) for a in arrs], _d(_c64(box.L)),
                                wl.ctypes.data_as(_I32), float(box.dt),
                                float(box.e if e is None else e), *[_d(o) for o in outs],
                                partner.ctypes.data_as(_I64), _d(tcoll), ctypes.byref(st))
    if rc:
        raise OracleError(rc)
    sweep = np.where(partner >= 0, 0, -1).astype(np.int32)
    return StepResult(*outs, partner, tcoll, sweep, st.n_pairs, st.n_sweeps, st.pair_tests,
                      st.reach)


def step_walls_spin(box, walls, w, mu: float, *, e: float | None = None) -> SpinStepResult:
    """One step of ``box`` between walls (walls[k] true: walls on axis k) with angular
    velocities ``w`` (shape (3, n)) and Coulomb friction ``mu``; inputs unchanged."""
    n = box.n
    arrs = [_c64(a) for a in (box.x, box.y, box.z, box.vx, box.vy, box.vz, w[0], w[1], w[2],
                              box.r, box.m)]
    outs = [np.empty(n) for _ in range(9)]
    partner = np.empty(n, dtype=np.int64)
    tcoll = np.empty(n)
    st = _Stats()
    wl = np.ascontiguousarray([1 if v else 0 for v in walls], dtype=np.int32)
    rc = _load().orc_step_walls_spin(n, *[_d(a) for a in arrs], _d(_c64(box.L)),
                                     wl.ctypes.data_as(_I32), float(box.dt),
                                     float(box.e if e is None else e), float(mu),
                                     *[_d(o) for o in outs], partner.ctypes.data_as(_I64),
                                     _d(tcoll), ctypes.byref(st))
    if rc:
        raise OracleError(rc)
    sweep = np.where(partner >= 0, 0, -1).astype(np.int32)
    return SpinStepResult(*outs[:6], partner, tcoll, sweep, st.n_pairs, st.n_sweeps,
                          st.pair_tests, st.reach, outs[6], outs[7], outs[8])
