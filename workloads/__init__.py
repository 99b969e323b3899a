"""Seeded synthetic particle boxes shared by the oracle, the GPU path, the tests
and the benchmark.

This module only *makes inputs*: radii, random-sequential-placement (RSA)
positions, Gaussian velocities and masses.  It contains none of the collision
method's arithmetic.  All random numbers come from ``gen.c`` (xoshiro256**
seeded by splitmix64, Box-Muller normals), so a given (recipe, seed) yields the
same bytes on every machine.

Recipes (the dense periodic particle boxes of the paper's collision tests,
Sec. "Parallel Performance" sets 1.6e7 particles; the validation section sets the
two-sphere and kinetic-energy cases):

* ``config(1)``  2,000 monodisperse spheres, r = 0.01, volume fraction 0.05.
  The box side follows from N, r and phi (L = 0.551293); e = 0.9,
  dt = 0.2 * diameter / sigma_v = 0.004.
* ``config(2)``  1,000,000 spheres, r = 1, phi = 0.2 (L = 275.65); e = 0.9,
  dt = 0.4.
* ``config(3)``  16,000,000 spheres, radii lognormal (median 1, log-sd 0.25)
  clamped to [0.5, 2], m = r^3, phi = 0.3; e = 0.8, dt = 0.4.
* ``config(4)``  512 independent boxes, N_b = round(exp(U(ln 1e3, ln 6.4e4))),
  r = 1, phi_b ~ U(0.05, 0.35); e = 0.9, dt = 0.4.
* ``config(5)``  the config-2 input, stepped 10 times with a learnable e.

Velocities are i.i.d. N(0, 1) per component (no mean removal); masses are 1
for monodisperse sets and r^3 otherwise.  Seed = config number unless given.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
# PCOL_WLGEN_LIB: another build of gen.c to load (used by the sanitizer test)
_LIB = os.environ.get("PCOL_WLGEN_LIB") or os.path.join(_HERE, "libwlgen.so")
_lib = None

# RNG stream ids (one independent xoshiro stream per purpose)
_S_RADII, _S_VEL, _S_PERM, _S_BATCH = 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile gen.c into libwlgen.so (gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.wl_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_double)]
        lib.wl_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_double)]
        lib.wl_permutation.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_int64)]
        lib.wl_rsa.argtypes = [ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_double), ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int,
                               P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double)]
        lib.wl_rsa.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def normals(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().wl_normals(seed, stream, n, _dp(out))
    return out


def uniforms(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().wl_uniforms(seed, stream, n, _dp(out))
    return out


def permutation(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _load().wl_permutation(seed, stream, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def rsa_positions(seed: int, r: np.ndarray, L, max_trials: int = 50_000_000):
    """Random sequential placement of spheres r (placed in array order)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    x = np.empty(n); y = np.empty(n); z = np.empty(n)
    cap = 16
    while True:
        rc = _load().wl_rsa(seed, n, _dp(r), float(L[0]), float(L[1]), float(L[2]),
                            max_trials, cap, _dp(x), _dp(y), _dp(z))
        if rc == -3 and cap < 1024:
            cap *= 2
            continue
        if rc < 0:
            raise RuntimeError(f"RSA placement failed (code {rc}) for n={n}, L={L}")
        return x, y, z


@dataclass
class Box:
    """One periodic box [0, L0) x [0, L1) x [0, L2) of spheres (SoA, float64)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    r: np.ndarray
    m: np.ndarray
    L: tuple
    dt: float
    e: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "Box":
        return Box(self.x.copy(), self.y.copy(), self.z.copy(), self.vx.copy(), self.vy.copy(),
                   self.vz.copy(), self.r.copy(), self.m.copy(), tuple(self.L), self.dt, self.e,
                   self.name, dict(self.meta))

    def arrays(self):
        return [self.x, self.y, self.z, self.vx, self.vy, self.vz, self.r, self.m]


def box_side(r: np.ndarray, phi: float) -> float:
    """Cube side for spheres r at volume fraction phi."""
    vol = float(np.sum((4.0 / 3.0) * math.pi * r.astype(np.float64) ** 3))
    return (vol / phi) ** (1.0 / 3.0)


def lognormal_radii(seed: int, n: int, median=1.0, logsd=0.25, lo=0.5, hi=2.0) -> np.ndarray:
    g = normals(seed, _S_RADII, n)
    return np.clip(median * np.exp(logsd * g), lo, hi)


def make_box(n: int, *, seed: int, phi: float, radius: float | None = None,
             lognormal: tuple | None = None, sigma_v: float = 1.0, e: float = 0.9,
             dt: float | None = None, L: float | None = None, name: str = "") -> Box:
    """A periodic cube of n non-overlapping spheres (RSA) with N(0, sigma_v^2) velocities.

    Either ``radius`` (monodisperse, m = 1) or ``lognormal=(median, logsd, lo, hi)``
    (m = r^3).  The side is chosen from phi unless ``L`` is given.  ``dt`` defaults
    to 0.2 * (median) diameter / sigma_v.
    """
    if lognormal is not None:
        med, lsd, lo, hi = lognormal
        r = lognormal_radii(seed, n, med, lsd, lo, hi)
        m = r ** 3
        dref = 2.0 * med
    else:
        r = np.full(n, float(radius))
        m = np.ones(n)
        dref = 2.0 * float(radius)
    side = float(L) if L is not None else box_side(r, phi)
    Lb = (side, side, side)
    order = np.argsort(-r, kind="stable")          # place large spheres first
    xs, ys, zs = rsa_positions(seed, r[order], Lb)
    x = np.empty(n); y = np.empty(n); z = np.empty(n)
    x[order] = xs; y[order] = ys; z[order] = zs
    perm = permutation(seed, _S_PERM, n)           # storage order uncorrelated with radius
    v = normals(seed, _S_VEL, 3 * n) * sigma_v
    if dt is None:
        dt = 0.2 * dref / sigma_v
    return Box(x[perm].copy(), y[perm].copy(), z[perm].copy(), v[0::3].copy(), v[1::3].copy(),
               v[2::3].copy(), r[perm].copy(), m[perm].copy(), Lb, float(dt), float(e), name,
               {"phi": phi, "seed": seed})


def config(k: int, seed: int | None = None, n: int | None = None) -> Box | list:
    """The benchmark configurations (see module docstring).  ``n`` overrides N."""
    s = k if seed is None else seed
    if k == 1:
        return make_box(n or 2000, seed=s, phi=0.05, radius=0.01, e=0.9, name="mono2k_phi0.05")
    if k in (2, 5):
        return make_box(n or 1_000_000, seed=s, phi=0.2, radius=1.0, e=0.9,
                        name="mono1M_phi0.2" if k == 2 else "mono1M_phi0.2_10steps")
    if k == 3:
        return make_box(n or 16_000_000, seed=s, phi=0.3, lognormal=(1.0, 0.25, 0.5, 2.0), e=0.8,
                        name="poly16M_phi0.3")
    if k == 4:
        return batch_boxes(512 if n is None else n, seed=s)
    raise ValueError(f"unknown config {k}")


def batch_boxes(nbox: int, *, seed: int, nmin: float = 1e3, nmax: float = 6.4e4,
                phi_lo: float = 0.05, phi_hi: float = 0.35, e: float = 0.9) -> list:
    """Uneven independent periodic boxes: N_b log-uniform in [nmin, nmax], phi_b uniform."""
    u = uniforms(seed, _S_BATCH, 2 * nbox)
    boxes = []
    for b in range(nbox):
        nb = int(round(math.exp(math.log(nmin) + u[2 * b] * (math.log(nmax) - math.log(nmin)))))
        phib = phi_lo + u[2 * b + 1] * (phi_hi - phi_lo)
        boxes.append(make_box(nb, seed=seed * 100003 + b + 1, phi=phib, radius=1.0, e=e,
                              name=f"box{b}"))
    return boxes


def deposit_case(n: int, *, seed: int, L=(1.0, 1.0, 1.0), comp: int = 4):
    """Positions uniform in the periodic box [0, L0) x [0, L1) x [0, L2) and comp
    standard-normal source components per sphere, shape (comp, n) (a momentum source of
    three components and an energy source, as carried by the deposition)."""
    L = tuple(float(v) for v in L)
    pos = []
    for d in range(3):
        u = uniforms(seed, 40 + d, n) * L[d]
        pos.append(np.where(u < L[d], u, np.nextafter(L[d], 0.0)))
    a = np.stack([normals(seed, 50 + q, n) for q in range(comp)]) if n else np.zeros((comp, 0))
    return pos[0], pos[1], pos[2], a
