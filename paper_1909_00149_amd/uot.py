"""Python binding of libuot (torch tensors in, argument marshalling only).

Every step of the solve runs in the HIP kernels behind the C ABI of
include/uot.h; PyTorch supplies device memory and the stream.  There is no
CPU fallback: without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, fields

import torch

from . import _lib
from ._lib import (UOT_WARM_START, UOT_ALLOW_SIGNED, UOT_UNSAFE_STEPS, UOT_NO_GRAPH,  # noqa: F401
                   UOT_AUTOTUNE, UOT_ADAPTIVE_STEPS, UOT_RECORD_HISTORY, UOT_WARM_FALLBACK)

DIST, PROX, PROX_FIXED = 0, 1, 2
NORM_ISO, NORM_ANISO = 0, 1
PLANES = ("Mx", "My", "r", "a", "x0", "x1")


class UOTError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = int(code)
        msg = _lib.load().uot_status_string(self.code).decode()
        super().__init__(f"{where}: {msg} (status {self.code})")


@dataclass
class Params:
    """Fields of uot_params (include/uot.h)."""
    nx: int = 0
    ny: int = 0
    mode: int = DIST
    balanced: bool = False
    residual_p: int = 1
    bc: int = 0
    mu: float = 1.0
    rho: float = 1.0
    tau1: float = 0.0
    tau2: float = 0.0
    max_iter: int = 1000
    check_every: int = 20
    tol: float = 0.0
    flags: int = 0
    tile_rows: int = 0
    pitch: int = 0
    norm: int = 0          # NORM_ISO (the paper's l2,1) or NORM_ANISO (l1,1)
    max_groups: int = 0    # cap on the persistent grid (0 = fill the device)

    def to_c(self):
        return _lib.Params(**{f.name: (int(getattr(self, f.name)) if f.type in ("int", "bool")
                                       else getattr(self, f.name)) for f in fields(self)})


def check_params(p: Params) -> int:
    """uot_check_params: validates without touching the GPU (0 = OK)."""
    c = p.to_c()
    return int(_lib.load().uot_check_params(ctypes.byref(c)))


def knorm2(nx, ny, mode=DIST, balanced=False, bc=0) -> float:
    return float(_lib.load().uot_knorm2(nx, ny, mode, int(balanced), bc))


def required_planes(mode, balanced):
    req = ["Mx", "My", "a"] + ([] if balanced else ["r"])
    if mode == PROX:
        req += ["x0", "x1"]
    elif mode == PROX_FIXED:
        req += ["x1"]
    return req


def new_state(mode, balanced, numel_or_shape, device="cuda"):
    """Zeroed caller-owned state planes for a mode."""
    return {k: torch.zeros(numel_or_shape, dtype=torch.float32, device=device)
            for k in required_planes(mode, balanced)}


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("planes must be contiguous float32 device tensors")
    return t.data_ptr()


def _cstate(st):
    return _lib.State(*[_ptr(st.get(k)) for k in PLANES])


def _layout(nx, ny, pitch, offset):
    """Host arrays of a batch layout; pitch None -> NULL (rows back to back)."""
    B = len(nx)
    if not (len(ny) == len(offset) == B and (pitch is None or len(pitch) == B)):
        raise ValueError("nx, ny, offset (and pitch) must have one entry per pair")
    ax = (ctypes.c_int32 * B)(*[int(v) for v in nx])
    ay = (ctypes.c_int32 * B)(*[int(v) for v in ny])
    ap = None if pitch is None else (ctypes.c_int32 * B)(*[int(v) for v in pitch])
    ao = (ctypes.c_int64 * B)(*[int(v) for v in offset])
    return ax, ay, ap, ao


class Solver:
    """One handle of the C ABI bound to the current device and stream."""

    def __init__(self, params: Params, stream=None):
        self.lib = _lib.load()
        self.params = params
        self._c = params.to_c()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.uot_create(ctypes.byref(self._c), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise UOTError(rc, "uot_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.uot_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, src, dst, state=None):
        """uot_solve on images of shape (ny, nx); returns (state, report)."""
        p = self.params
        if state is None:
            state = new_state(p.mode, p.balanced, src.shape, src.device)
        cs = _cstate(state)
        rep = _lib.Report()
        rc = self.lib.uot_solve(self._h, _ptr(src), _ptr(dst), ctypes.byref(cs), ctypes.byref(rep))
        if rc != 0:
            raise UOTError(rc, "uot_solve")
        return state, rep.as_dict()

    def step(self, src, dst, state_in, iters, state_out=None):
        """uot_step: `iters` iterations from state_in into state_out (state_in
        is only read); returns state_out."""
        p = self.params
        if state_out is None:
            state_out = new_state(p.mode, p.balanced, src.shape, src.device)
        ci, co = _cstate(state_in), _cstate(state_out)
        rc = self.lib.uot_step(self._h, _ptr(src), _ptr(dst), ctypes.byref(ci), ctypes.byref(co), int(iters))
        if rc != 0:
            raise UOTError(rc, "uot_step")
        return state_out

    def solve_batched(self, src, dst, nx, ny, offset, state=None, pitch=None):
        """uot_solve_batched (uot_solve_batched_pitched when pitch is given) on
        packed 1-D planes; returns (state, [reports])."""
        p = self.params
        B = len(nx)
        if state is None:
            state = new_state(p.mode, p.balanced, src.numel(), src.device)
        ax, ay, ap, ao = _layout(nx, ny, pitch, offset)
        reps = (_lib.Report * B)()
        cs = _cstate(state)
        if pitch is None:
            rc = self.lib.uot_solve_batched(self._h, B, ax, ay, ao, _ptr(src), _ptr(dst), ctypes.byref(cs), reps)
        else:
            rc = self.lib.uot_solve_batched_pitched(self._h, B, ax, ay, ap, ao, _ptr(src), _ptr(dst),
                                                    ctypes.byref(cs), reps)
        if rc != 0:
            raise UOTError(rc, "uot_solve_batched")
        return state, [r.as_dict() for r in reps]

    def poisson(self, rhs, alpha=0.0, out=None):
        """uot_poisson: phi = (alpha I + D D*)^{-1} rhs (zero-flux boundary)."""
        ny, nx = rhs.shape
        phi = torch.empty_like(rhs) if out is None else out
        rc = self.lib.uot_poisson(self._h, nx, ny, float(alpha), _ptr(rhs), _ptr(phi))
        if rc != 0:
            raise UOTError(rc, "uot_poisson")
        return phi

    def init_poisson(self, src, dst, state=None, nx=None, ny=None, offset=None, pitch=None):
        """uot_init_poisson(_pitched): Poisson-flux start (single grid, or
        packed pairs when nx/ny/offset are given)."""
        p = self.params
        if nx is None:
            ny_, nx_ = src.shape
            nx, ny, offset = [nx_], [ny_], [0]
        B = len(nx)
        if state is None:
            state = new_state(p.mode, p.balanced, src.shape, src.device)
        ax, ay, ap, ao = _layout(nx, ny, pitch, offset)
        cs = _cstate(state)
        if pitch is None:
            rc = self.lib.uot_init_poisson(self._h, B, ax, ay, ao, _ptr(src), _ptr(dst), ctypes.byref(cs))
        else:
            rc = self.lib.uot_init_poisson_pitched(self._h, B, ax, ay, ap, ao, _ptr(src), _ptr(dst),
                                                   ctypes.byref(cs))
        if rc != 0:
            raise UOTError(rc, "uot_init_poisson")
        return state

    def time_iterations(self, src, dst, state, n):
        """uot_time_iterations: (average ms per fused-iteration launch, the
        kernel shape code that ran)."""
        cs = _cstate(state)
        ms = ctypes.c_double()
        shape = ctypes.c_int32()
        rc = self.lib.uot_time_iterations(self._h, _ptr(src), _ptr(dst), ctypes.byref(cs), int(n), ctypes.byref(ms),
                                          ctypes.byref(shape))
        if rc != 0:
            raise UOTError(rc, "uot_time_iterations")
        return ms.value, shape.value

    def time_iterations_batched(self, src, dst, nx, ny, offset, state, n, pitch=None):
        """uot_time_iterations_batched on packed planes: (average ms per
        launch with every pair live, the kernel shape code that ran)."""
        B = len(nx)
        ax, ay, ap, ao = _layout(nx, ny, pitch, offset)
        cs = _cstate(state)
        ms = ctypes.c_double()
        shape = ctypes.c_int32()
        rc = self.lib.uot_time_iterations_batched(self._h, B, ax, ay, ap, ao, _ptr(src), _ptr(dst),
                                                  ctypes.byref(cs), int(n), ctypes.byref(ms), ctypes.byref(shape))
        if rc != 0:
            raise UOTError(rc, "uot_time_iterations_batched")
        return ms.value, shape.value

    def history(self, pair=0):
        """uot_history: (iterations, rel_res) at every check of the last solve
        made with UOT_RECORD_HISTORY, for one pair; two numpy arrays."""
        import numpy as np
        n = ctypes.c_int32(0)
        rc = self.lib.uot_history(self._h, int(pair), None, None, 0, ctypes.byref(n))
        if rc != 0:
            raise UOTError(rc, "uot_history")
        it = np.zeros(n.value, np.int32)
        rr = np.zeros(n.value, np.float64)
        rc = self.lib.uot_history(self._h, int(pair), it.ctypes.data_as(ctypes.c_void_p),
                                  rr.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n))
        if rc != 0:
            raise UOTError(rc, "uot_history")
        return it, rr

    def dr_solve(self, src, dst, gamma=1.0, state=None):
        """uot_dr_solve: Douglas-Rachford splitting with the DCT projection on
        images of shape (ny, nx); returns (z state, report)."""
        p = self.params
        if state is None:
            state = new_state(p.mode, p.balanced, src.shape, src.device)
        cs = _cstate(state)
        rep = _lib.DrReport()
        rc = self.lib.uot_dr_solve(self._h, _ptr(src), _ptr(dst), ctypes.byref(cs), float(gamma), ctypes.byref(rep))
        if rc != 0:
            raise UOTError(rc, "uot_dr_solve")
        return state, rep.as_dict()

    def objective(self, src, dst, state, prev=None):
        cs = _cstate(state)
        cp = _cstate(prev) if prev is not None else None
        rep = _lib.Report()
        rc = self.lib.uot_objective(self._h, _ptr(src), _ptr(dst), ctypes.byref(cs),
                                    ctypes.byref(cp) if cp is not None else None, ctypes.byref(rep))
        if rc != 0:
            raise UOTError(rc, "uot_objective")
        return rep.as_dict()


def solve_noalloc(params: Params, src, dst, state=None, stream=None):
    """uot_solve_noalloc: one grid solved with the library's fixed device
    scratch instead of a handle's allocations (for callers that cannot
    allocate); returns (state, report)."""
    lib = _lib.load()
    if state is None:
        state = new_state(params.mode, params.balanced, src.shape, src.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    c = params.to_c()
    cs = _cstate(state)
    rep = _lib.Report()
    rc = lib.uot_solve_noalloc(ctypes.byref(c), ctypes.c_void_p(stream.cuda_stream), _ptr(src), _ptr(dst),
                               ctypes.byref(cs), ctypes.byref(rep))
    if rc != 0:
        raise UOTError(rc, "uot_solve_noalloc")
    return state, rep.as_dict()


def pack(images):
    """Packs a list of (ny, nx) tensors into one flat plane; returns
    (packed, nx list, ny list, offsets)."""
    nx = [int(t.shape[1]) for t in images]
    ny = [int(t.shape[0]) for t in images]
    offs, o = [], 0
    for a, b in zip(nx, ny):
        offs.append(o)
        o += a * b
    flat = torch.cat([t.reshape(-1) for t in images]) if images else torch.zeros(0)
    return flat.contiguous(), nx, ny, offs


def unpack(flat, nx, ny, offsets):
    return [flat[o:o + a * b].view(b, a) for a, b, o in zip(nx, ny, offsets)]


def pack_pitched(images, align=64):
    """Packs (ny, nx) tensors into one flat plane with every row starting on
    an `align`-element boundary; the padding is zero and is never touched by
    the solver.  The default, 64 elements (256 bytes, one row of a 64-pixel
    tile), keeps every L2 line and HBM burst of a tile row inside that row;
    on a ragged batch it is worth about a third more fused-kernel bandwidth
    than rows packed back to back.  Returns (packed, nx list, ny list, pitch
    list, offsets)."""
    if align < 1:
        raise ValueError("align must be >= 1")
    nx = [int(t.shape[1]) for t in images]
    ny = [int(t.shape[0]) for t in images]
    pitch = [-(-a // align) * align for a in nx]
    offs, o = [], 0
    for pt, b in zip(pitch, ny):
        offs.append(o)
        o += pt * b
    dev = images[0].device if images else "cpu"
    flat = torch.zeros(o, dtype=torch.float32, device=dev)
    for t, pt, b, off in zip(images, pitch, ny, offs):
        flat[off:off + pt * b].view(b, pt)[:, :t.shape[1]] = t
    return flat, nx, ny, pitch, offs


def unpack_pitched(flat, nx, ny, pitch, offsets):
    """Views (ny, nx) of each pair of a pitched plane (strided, not copied)."""
    return [flat[o:o + pt * b].view(b, pt)[:, :a] for a, b, pt, o in zip(nx, ny, pitch, offsets)]
