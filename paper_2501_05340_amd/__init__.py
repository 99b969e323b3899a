"""pcol: a deterministic hard-sphere binary collision step on one AMD MI355X.

Thin Python binding of ``libpcol.so`` (C ABI declared in ``include/pcol.h``):
argument marshalling only.  Every step of the method runs in the library's HIP
kernels; PyTorch supplies device memory and the current stream.  There is no
CPU path: importing this package without the built library raises.

The entry points keep the C names (``pcol_create``, ``pcol_bin``,
``pcol_detect``, ``pcol_resolve``, ``pcol_advance``, ``pcol_step``).  Arrays are
torch tensors on the GPU: float64 for positions, velocities, radii, masses and
times, uint8 for active masks, int32 for partners, int64 for keys (the uint64
key bits reinterpreted).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcol.so")

(PCOL_OK, PCOL_E_INVALID, PCOL_E_BOX, PCOL_E_NOMEM, PCOL_E_HIP, PCOL_E_SWEEPS, PCOL_E_STATE,
 PCOL_E_SCRATCH) = range(8)
STATUS_NAMES = {0: "PCOL_OK", 1: "PCOL_E_INVALID", 2: "PCOL_E_BOX", 3: "PCOL_E_NOMEM",
                4: "PCOL_E_HIP", 5: "PCOL_E_SWEEPS", 6: "PCOL_E_STATE", 7: "PCOL_E_SCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 << 20  # PCOL_NOALLOC_SCRATCH_BYTES
NO_KEY = -1  # UINT64_MAX seen as int64


class pcol_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                                          ("x", "y", "z", "vx", "vy", "vz", "r", "m")]


class pcol_box(ctypes.Structure):
    _fields_ = [("len", ctypes.c_double * 3)]


class pcol_opts(ctypes.Structure):
    _fields_ = [("cell_mult", ctypes.c_double), ("max_sweeps", ctypes.c_int),
                ("home_cells", ctypes.c_int), ("contact_slots", ctypes.c_int),
                ("filter", ctypes.c_int), ("band_rel", ctypes.c_double),
                ("timing", ctypes.c_int), ("autotune", ctypes.c_int),
                ("split_quantile", ctypes.c_double), ("order", ctypes.c_int)]


class pcol_stats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_sweeps", ctypes.c_int64),
                ("pair_tests", ctypes.c_int64), ("contacts", ctypes.c_int64),
                ("n_overflow", ctypes.c_int64), ("n_recheck", ctypes.c_int64),
                ("nc", ctypes.c_int32 * 3), ("home_cells", ctypes.c_int32),
                ("max_cell", ctypes.c_int32), ("h", ctypes.c_double * 3),
                ("reach", ctypes.c_double), ("band", ctypes.c_double),
                ("ms_bin", ctypes.c_double),
                ("ms_detect", ctypes.c_double), ("ms_sweeps", ctypes.c_double),
                ("ms_advance", ctypes.c_double), ("n_wide", ctypes.c_int64),
                ("rho_c", ctypes.c_double)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class pcol_batch_stats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_sweeps", ctypes.c_int64),
                ("contacts", ctypes.c_int64), ("n_overflow", ctypes.c_int64),
                ("total_cells", ctypes.c_int64), ("replanned", ctypes.c_int32),
                ("finished_on_host", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("home_cells", ctypes.c_int32), ("cell_mult", ctypes.c_double)]

    as_dict = pcol_stats.as_dict


class pcol_state_grad(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc, gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.POINTER, ctypes.c_void_p
    ctx_p = ctypes.c_void_p
    lib.pcol_default_opts.argtypes = [P(pcol_opts)]
    lib.pcol_default_opts.restype = None
    lib.pcol_create.argtypes = [P(ctx_p), ctypes.c_int64, V, P(pcol_opts)]
    lib.pcol_create.restype = ctypes.c_int
    lib.pcol_destroy.argtypes = [ctx_p]
    lib.pcol_destroy.restype = None
    lib.pcol_last_error.argtypes = [ctx_p]
    lib.pcol_last_error.restype = ctypes.c_char_p
    lib.pcol_set_stream.argtypes = [ctx_p, V]
    lib.pcol_set_stream.restype = ctypes.c_int
    lib.pcol_bin.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), ctypes.c_double]
    lib.pcol_bin.restype = ctypes.c_int
    lib.pcol_detect.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), ctypes.c_double, V, V, V]
    lib.pcol_detect.restype = ctypes.c_int
    lib.pcol_resolve.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), ctypes.c_double,
                                 ctypes.c_double, V, V, V, V, V]
    lib.pcol_resolve.restype = ctypes.c_int
    lib.pcol_advance.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), ctypes.c_double, V]
    lib.pcol_advance.restype = ctypes.c_int
    lib.pcol_step.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), ctypes.c_double,
                              ctypes.c_double, V, V, P(pcol_stats)]
    lib.pcol_step.restype = ctypes.c_int
    lib.pcol_step_spin.argtypes = [ctx_p, P(pcol_particles), V, V, V, P(pcol_box),
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, V, V,
                                   P(pcol_stats)]
    lib.pcol_step_spin.restype = ctypes.c_int
    lib.pcol_step_backward.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), ctypes.c_double,
                                       ctypes.c_double, V, V, P(pcol_state_grad),
                                       P(pcol_state_grad), V]
    lib.pcol_step_backward.restype = ctypes.c_int
    lib.pcol_step_batched.argtypes = [ctx_p, ctypes.c_int32, V, P(pcol_box), P(pcol_particles),
                                      ctypes.c_double, ctypes.c_double, V, V,
                                      P(pcol_batch_stats)]
    lib.pcol_step_batched.restype = ctypes.c_int
    lib.pcol_step_walls.argtypes = [ctx_p, P(pcol_particles), P(pcol_box), P(ctypes.c_int32),
                                    ctypes.c_double, ctypes.c_double, V, V, P(pcol_stats)]
    lib.pcol_step_walls.restype = ctypes.c_int
    lib.pcol_step_spin_walls.argtypes = [ctx_p, P(pcol_particles), V, V, V, P(pcol_box),
                                         P(ctypes.c_int32), ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, V, V, P(pcol_stats)]
    lib.pcol_step_spin_walls.restype = ctypes.c_int
    lib.pcol_deposit.argtypes = [ctx_p, V, V, V, ctypes.c_int64, V, ctypes.c_int,
                                 P(ctypes.c_int32), P(ctypes.c_double), V]
    lib.pcol_deposit.restype = ctypes.c_int
    lib.pcol_deposit_noalloc.argtypes = [V, V, V, ctypes.c_int64, V, ctypes.c_int,
                                         P(ctypes.c_int32), P(ctypes.c_double), V, V]
    lib.pcol_deposit_noalloc.restype = ctypes.c_int
    return lib


lib = _load()

EXPORTED = ["pcol_default_opts", "pcol_create", "pcol_destroy", "pcol_last_error",
            "pcol_set_stream", "pcol_bin", "pcol_detect", "pcol_resolve", "pcol_advance",
            "pcol_step", "pcol_step_spin", "pcol_step_backward", "pcol_step_batched",
            "pcol_deposit", "pcol_step_walls", "pcol_step_spin_walls", "pcol_deposit_noalloc"]


class PcolError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


@dataclass
class Particles:
    """SoA sphere state on the GPU (float64, contiguous, length n)."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    vx: torch.Tensor
    vy: torch.Tensor
    vz: torch.Tensor
    r: torch.Tensor
    m: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @staticmethod
    def from_box(box, device="cuda") -> "Particles":
        f = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        return Particles(f(box.x), f(box.y), f(box.z), f(box.vx), f(box.vy), f(box.vz), f(box.r),
                         f(box.m))

    def clone(self) -> "Particles":
        return Particles(*[t.clone() for t in self.tensors()])

    def tensors(self):
        return [self.x, self.y, self.z, self.vx, self.vy, self.vz, self.r, self.m]

    def struct(self) -> pcol_particles:
        n = self.n
        for t in self.tensors():
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.shape != (n,):
                raise ValueError("particle arrays must be contiguous float64 CUDA tensors of equal length")
        return pcol_particles(n, *[t.data_ptr() for t in self.tensors()])


def _box(L) -> pcol_box:
    b = pcol_box()
    for a in range(3):
        b.len[a] = float(L[a])
    return b


def _ptr(t, dtype=None, n=None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or (dtype is not None and t.dtype != dtype):
        raise ValueError(f"expected a contiguous CUDA tensor of {dtype}")
    if n is not None and t.shape[0] != n:
        raise ValueError("array length differs from the particle count")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def pcol_default_opts(**kw) -> pcol_opts:
    o = pcol_opts()
    lib.pcol_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """Owns a pcol_ctx; destroyed with the object."""

    def __init__(self, n_max: int, opts: pcol_opts | None = None):
        self._h = ctypes.c_void_p()
        st = lib.pcol_create(ctypes.byref(self._h), int(n_max), ctypes.c_void_p(_stream()),
                             ctypes.byref(opts) if opts is not None else None)
        if st != PCOL_OK:
            raise PcolError(st, "pcol_create failed")
        self.n_max = int(n_max)

    @property
    def handle(self):
        return self._h

    def check(self, st: int):
        if st != PCOL_OK:
            raise PcolError(st, lib.pcol_last_error(self._h).decode())

    def sync_stream(self):
        lib.pcol_set_stream(self._h, ctypes.c_void_p(_stream()))

    def close(self):
        if self._h:
            lib.pcol_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcol_create(n_max: int, opts: pcol_opts | None = None) -> Context:
    return Context(n_max, opts)


def pcol_destroy(ctx: Context) -> None:
    ctx.close()


def pcol_last_error(ctx: Context) -> str:
    return lib.pcol_last_error(ctx.handle).decode()


def pcol_set_stream(ctx: Context, stream=None) -> None:
    """Point the context at a stream (default: torch's current stream)."""
    h = stream.cuda_stream if stream is not None else _stream()
    ctx.check(lib.pcol_set_stream(ctx.handle, ctypes.c_void_p(h)))


def pcol_bin(ctx: Context, p: Particles, L, dt: float) -> None:
    ctx.sync_stream()
    ps = p.struct()
    ctx.check(lib.pcol_bin(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)), float(dt)))


def pcol_detect(ctx: Context, p: Particles, L, dt: float, active=None, key_out=None,
                tmin_out=None):
    """Returns (key, tmin) tensors (allocated if not given)."""
    n = p.n
    if key_out is None:
        key_out = torch.empty(n, dtype=torch.int64, device=p.x.device)
    if tmin_out is None:
        tmin_out = torch.empty(n, dtype=torch.float64, device=p.x.device)
    ctx.sync_stream()
    ps = p.struct()
    ctx.check(lib.pcol_detect(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)), float(dt),
                              _ptr(active, torch.uint8, n), _ptr(key_out, torch.int64, n),
                              _ptr(tmin_out, torch.float64, n)))
    return key_out, tmin_out


def pcol_resolve(ctx: Context, p: Particles, L, dt: float, e: float, key, active, partner=None,
                 tcoll=None, n_pairs=None) -> None:
    n = p.n
    ctx.sync_stream()
    ps = p.struct()
    ctx.check(lib.pcol_resolve(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)), float(dt),
                               float(e), _ptr(key, torch.int64, n), _ptr(active, torch.uint8, n),
                               _ptr(partner, torch.int32, n), _ptr(tcoll, torch.float64, n),
                               _ptr(n_pairs, torch.int64)))


def pcol_advance(ctx: Context, p: Particles, L, dt: float, partner) -> None:
    ctx.sync_stream()
    ps = p.struct()
    ctx.check(lib.pcol_advance(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)), float(dt),
                               _ptr(partner, torch.int32, p.n)))


def pcol_step(ctx: Context, p: Particles, L, dt: float, e: float, partner=None, tcoll=None,
              stats: bool = True):
    """One full step in place; returns a dict of pcol_stats (or None)."""
    n = p.n
    st = pcol_stats() if stats else None
    ctx.sync_stream()
    ps = p.struct()
    ctx.check(lib.pcol_step(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)), float(dt),
                            float(e), _ptr(partner, torch.int32, n), _ptr(tcoll, torch.float64, n),
                            ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def pcol_step_spin(ctx: Context, p: Particles, w, L, dt: float, e: float, mu: float,
                   partner=None, tcoll=None, stats: bool = True):
    """One full step with angular velocities w = (wx, wy, wz) (float64 device tensors,
    updated in place) and Coulomb friction mu; returns a dict of pcol_stats (or None)."""
    n = p.n
    st = pcol_stats() if stats else None
    ctx.sync_stream()
    ps = p.struct()
    wp = [_ptr(t, torch.float64, n) for t in w]
    ctx.check(lib.pcol_step_spin(ctx.handle, ctypes.byref(ps), *wp, ctypes.byref(_box(L)),
                                 float(dt), float(e), float(mu), _ptr(partner, torch.int32, n),
                                 _ptr(tcoll, torch.float64, n),
                                 ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def pcol_step_batched(ctx: Context, p: Particles, box_off, Ls, dt: float, e: float, partner=None,
                      tcoll=None, stats: bool = True):
    """One step of many independent periodic boxes in place.  The spheres of box b
    are p[box_off[b]:box_off[b+1]] (positions within [0, Ls[b]) per axis);
    partner indices are global (into p).  Returns a dict of pcol_batch_stats."""
    n = p.n
    off = [int(v) for v in box_off]
    nbox = len(off) - 1
    if nbox < 1 or len(Ls) != nbox:
        raise ValueError("box_off needs nbox + 1 entries and Ls nbox boxes")
    off_arr = (ctypes.c_int64 * (nbox + 1))(*off)
    boxes = (pcol_box * nbox)()
    for b, L in enumerate(Ls):
        Lb = (L, L, L) if isinstance(L, (int, float)) else L
        for a in range(3):
            boxes[b].len[a] = float(Lb[a])
    st = pcol_batch_stats() if stats else None
    ctx.sync_stream()
    ps = p.struct()
    ctx.check(lib.pcol_step_batched(ctx.handle, nbox, ctypes.cast(off_arr, ctypes.c_void_p), boxes,
                                    ctypes.byref(ps), float(dt), float(e),
                                    _ptr(partner, torch.int32, n), _ptr(tcoll, torch.float64, n),
                                    ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def _grad_struct(ts, n):
    return pcol_state_grad(*[_ptr(t, torch.float64, n) for t in ts])


def pcol_step_backward(ctx: Context, start: Particles, L, dt: float, e: float, partner, tcoll,
                       g_out, g_in, ge) -> None:
    """Adjoint of one step (pair set fixed).  g_out, g_in: sequences of six float64
    tensors (x, y, z, vx, vy, vz); ge: float64 scalar tensor, accumulated."""
    n = start.n
    ctx.sync_stream()
    ps = start.struct()
    go = _grad_struct(g_out, n)
    gi = _grad_struct(g_in, n)
    ctx.check(lib.pcol_step_backward(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)),
                                     float(dt), float(e), _ptr(partner, torch.int32, n),
                                     _ptr(tcoll, torch.float64, n), ctypes.byref(go),
                                     ctypes.byref(gi), _ptr(ge, torch.float64)))


class Rollout(torch.autograd.Function):
    """``nsteps`` collision steps as a differentiable function of the initial
    positions, velocities and the restitution coefficient e (pair sets held fixed
    at those of the forward pass).  Every ``checkpoint_every``-th start state is
    kept together with every step's pair record (partner, contact time); the
    backward pass recomputes the other start states by stepping forward from the
    nearest checkpoint (the step is deterministic, so the pair sets repeat
    bitwise), then applies pcol_step_backward step by step in reverse."""

    @staticmethod
    def forward(fctx, x, y, z, vx, vy, vz, e, r, m, L, dt, nsteps, pctx, checkpoint_every=1):
        n = x.shape[0]
        p = Particles(x.detach().clone(), y.detach().clone(), z.detach().clone(),
                      vx.detach().clone(), vy.detach().clone(), vz.detach().clone(), r, m)
        ev = float(e)
        ckpt, records = {}, []
        for k in range(nsteps):
            if k % checkpoint_every == 0:
                ckpt[k] = [t.clone() for t in p.tensors()[:6]]
            partner = torch.empty(n, dtype=torch.int32, device=x.device)
            tcoll = torch.empty(n, dtype=torch.float64, device=x.device)
            pcol_step(pctx, p, L, dt, ev, partner, tcoll, stats=False)
            records.append((partner, tcoll))
        fctx.ckpt, fctx.records = ckpt, records
        fctx.meta = (L, dt, ev, nsteps, pctx, checkpoint_every, r, m)
        return p.x, p.y, p.z, p.vx, p.vy, p.vz

    @staticmethod
    def backward(fctx, *grads):
        L, dt, ev, nsteps, pctx, every, r, m = fctx.meta
        n = r.shape[0]
        g = [gr.contiguous() if gr is not None else torch.zeros(n, dtype=torch.float64, device=r.device)
             for gr in grads]
        ge = torch.zeros((), dtype=torch.float64, device=r.device)
        cache = {}
        for k in reversed(range(nsteps)):
            if k not in cache:  # recompute the start states of this checkpoint segment
                base = (k // every) * every
                s = [t.clone() for t in fctx.ckpt[base]]
                cache = {base: [t.clone() for t in s]}
                p = Particles(*s, r, m)
                for q in range(base, k):
                    partner = torch.empty(n, dtype=torch.int32, device=r.device)
                    tcoll = torch.empty(n, dtype=torch.float64, device=r.device)
                    pcol_step(pctx, p, L, dt, ev, partner, tcoll, stats=False)
                    cache[q + 1] = [t.clone() for t in p.tensors()[:6]]
            start = Particles(*cache[k], r, m)
            partner, tcoll = fctx.records[k]
            gin = [torch.empty_like(t) for t in g]
            pcol_step_backward(pctx, start, L, dt, ev, partner, tcoll, g, gin, ge)
            g = gin
        return (*g, ge, None, None, None, None, None, None, None)


def rollout(p: Particles, e, L, dt: float, nsteps: int, ctx: Context, checkpoint_every: int = 1):
    """Differentiable multi-step rollout; returns the final (x, y, z, vx, vy, vz).
    e: float64 0-d tensor (requires_grad for its gradient)."""
    return Rollout.apply(p.x, p.y, p.z, p.vx, p.vy, p.vz, e, p.r, p.m, L, dt, nsteps, ctx,
                         checkpoint_every)


def pcol_deposit(ctx: Context, x, y, z, a, nc, L, out=None):
    """Deposit the sources a (float64 device tensor, shape (comp, n)) of spheres at
    x, y, z onto the corner nodes of the periodic grid of nc cells per axis over the
    box L.  Returns out, shape (nc2, nc1, nc0, comp) (node-major), overwritten."""
    n = int(x.shape[0])
    comp = int(a.shape[0])
    if a.dim() != 2 or a.shape[1] != n:
        raise ValueError("a must have shape (comp, n)")
    ncs = [int(v) for v in nc]
    Lb = (L, L, L) if isinstance(L, (int, float)) else L
    if out is None:
        out = torch.empty((ncs[2], ncs[1], ncs[0], comp), dtype=torch.float64, device=x.device)
    if out.numel() != ncs[0] * ncs[1] * ncs[2] * comp:
        raise ValueError("out has the wrong size")
    ncv = (ctypes.c_int32 * 3)(*ncs)
    Lv = (ctypes.c_double * 3)(*[float(v) for v in Lb])
    ctx.sync_stream()
    ctx.check(lib.pcol_deposit(ctx.handle, _ptr(x, torch.float64, n), _ptr(y, torch.float64, n),
                               _ptr(z, torch.float64, n), n, _ptr(a, torch.float64), comp, ncv,
                               Lv, _ptr(out, torch.float64)))
    return out


def pcol_deposit_noalloc(x, y, z, a, nc, L, out):
    """pcol_deposit without a context or any allocation (the library's fixed device
    scratch; see include/pcol.h).  out: float64 device tensor of nc2 nc1 nc0 comp
    values, overwritten.  Raises PcolError (PCOL_E_SCRATCH when the input does not fit)."""
    n = int(x.shape[0])
    comp = int(a.shape[0])
    if a.dim() != 2 or a.shape[1] != n:
        raise ValueError("a must have shape (comp, n)")
    ncs = [int(v) for v in nc]
    Lb = (L, L, L) if isinstance(L, (int, float)) else L
    if out.numel() != ncs[0] * ncs[1] * ncs[2] * comp:
        raise ValueError("out has the wrong size")
    ncv = (ctypes.c_int32 * 3)(*ncs)
    Lv = (ctypes.c_double * 3)(*[float(v) for v in Lb])
    st = lib.pcol_deposit_noalloc(_ptr(x, torch.float64, n), _ptr(y, torch.float64, n),
                                  _ptr(z, torch.float64, n), n, _ptr(a, torch.float64), comp, ncv,
                                  Lv, _ptr(out, torch.float64), ctypes.c_void_p(_stream()))
    if st != PCOL_OK:
        raise PcolError(st, "pcol_deposit_noalloc failed")
    return out


def pcol_step_walls(ctx: Context, p: Particles, L, walls, dt: float, e: float, partner=None,
                    tcoll=None, stats: bool = True):
    """One full step in place with reflective walls on the axes where walls[k] is true
    (the others periodic); returns a dict of pcol_stats (or None)."""
    n = p.n
    st = pcol_stats() if stats else None
    ctx.sync_stream()
    ps = p.struct()
    wl = (ctypes.c_int32 * 3)(*[1 if w else 0 for w in walls])
    ctx.check(lib.pcol_step_walls(ctx.handle, ctypes.byref(ps), ctypes.byref(_box(L)), wl,
                                  float(dt), float(e), _ptr(partner, torch.int32, n),
                                  _ptr(tcoll, torch.float64, n),
                                  ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def pcol_step_spin_walls(ctx: Context, p: Particles, w, L, walls, dt: float, e: float, mu: float,
                         partner=None, tcoll=None, stats: bool = True):
    """pcol_step_spin between reflective walls on the axes where walls[k] is true; the
    spins w = (wx, wy, wz) are updated in place.  Returns a dict of pcol_stats (or None)."""
    n = p.n
    st = pcol_stats() if stats else None
    ctx.sync_stream()
    ps = p.struct()
    wp = [_ptr(t, torch.float64, n) for t in w]
    wl = (ctypes.c_int32 * 3)(*[1 if v else 0 for v in walls])
    ctx.check(lib.pcol_step_spin_walls(ctx.handle, ctypes.byref(ps), *wp, ctypes.byref(_box(L)),
                                       wl, float(dt), float(e), float(mu),
                                       _ptr(partner, torch.int32, n), _ptr(tcoll, torch.float64, n),
                                       ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None
