"""Python binding of the ADMM solvers of include/uot_admm.h (argument
marshalling only: every step runs in the library's HIP kernels).

UOT-DF (Sec. IV-A, Algorithm 2): ``UotDf(nx, ny, kappa=..., mu=..., rho=...)
.solve(y, s0, phi=None)`` returns the frame estimate s and the report.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .uot import UOTError, _ptr


class UotDf:
    """One UOT-DF handle for a grid of ny x nx pixels on the current device
    and stream."""

    def __init__(self, nx, ny, kappa, mu, rho, lam=0.0, balanced=False, residual_p=1, bc=0, prox_iters=1,
                 max_iter=5000, check_every=10, eps=1e-3, flags=0, prox_tau_ratio=0.0, stream=None):
        self.lib = _lib.load()
        self.shape = (int(ny), int(nx))
        self._c = _lib.DfParams(int(nx), int(ny), int(balanced), int(residual_p), int(bc), float(kappa), float(mu),
                                float(lam), float(rho), int(prox_iters), int(max_iter), int(check_every), float(eps),
                                int(flags), float(prox_tau_ratio))
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.uotdf_create(ctypes.byref(self._c), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise UOTError(rc, "uotdf_create")
        self._h = h

    @staticmethod
    def check(**kw) -> int:
        """uotdf_check_params on keyword parameters (0 = valid)."""
        d = dict(nx=1, ny=1, balanced=0, residual_p=1, bc=0, kappa=1.0, mu=1.0, lam=0.0, rho=1.0, prox_iters=1,
                 max_iter=10, check_every=1, eps=1e-3, flags=0, prox_tau_ratio=0.0)
        d.update(kw)
        c = _lib.DfParams(*[d[k] for k, _ in _lib.DfParams._fields_])
        return int(_lib.load().uotdf_check_params(ctypes.byref(c)))

    def solve(self, y, s0, phi=None, out=None):
        s = torch.empty_like(y) if out is None else out
        rep = _lib.DfReport()
        rc = self.lib.uotdf_solve(self._h, _ptr(y), _ptr(phi), _ptr(s0), _ptr(s), ctypes.byref(rep))
        if rc != 0:
            raise UOTError(rc, "uotdf_solve")
        return s, rep.as_dict()

    def planes(self, device="cuda"):
        """The ADMM planes x, z, a, b left by the last solve."""
        out = {k: torch.empty(self.shape, dtype=torch.float32, device=device) for k in ("x", "z", "a", "b")}
        rc = self.lib.uotdf_copy_planes(self._h, *[_ptr(out[k]) for k in ("x", "z", "a", "b")])
        if rc != 0:
            raise UOTError(rc, "uotdf_copy_planes")
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.lib.uotdf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Rpca:
    """One RPCA+UOT-DF handle (Algorithm 3) for T frames of ny x nx pixels;
    signed=True solves the signed variant S = S+ - S- (eq. RPCA_UOTDF_PN)."""

    PLANES = ("X", "Tn", "A", "D", "Z", "W", "B", "C")

    def __init__(self, nx, ny, frames, lam, gam, kappa, mu, rho, balanced=False, residual_p=1, bc=0, prox_iters=1,
                 max_iter=5000, check_every=10, eps=1e-4, flags=0, prox_tau_ratio=0.0, signed=False, stream=None):
        self.lib = _lib.load()
        self.shape = (int(frames), int(ny), int(nx))
        self.signed = bool(signed)
        self._c = _lib.RpParams(int(nx), int(ny), int(frames), int(balanced), int(residual_p), int(bc), float(lam),
                                float(gam), float(kappa), float(mu), float(rho), int(prox_iters), int(max_iter),
                                int(check_every), float(eps), int(flags), float(prox_tau_ratio), int(self.signed), 0)
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.rpca_create(ctypes.byref(self._c), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise UOTError(rc, "rpca_create")
        self._h = h

    @staticmethod
    def check(**kw) -> int:
        d = dict(nx=4, ny=4, frames=3, balanced=0, residual_p=1, bc=0, lam=0.1, gam=0.1, kappa=1.0, mu=1.0,
                 rho=1.0, prox_iters=1, max_iter=10, check_every=1, eps=1e-4, flags=0, prox_tau_ratio=0.0,
                 signed_sparse=0, reserved=0)
        d.update(kw)
        c = _lib.RpParams(*[d[k] for k, _ in _lib.RpParams._fields_])
        return int(_lib.load().rpca_check_params(ctypes.byref(c)))

    def solve(self, y, phi=None):
        """y (and phi): (T, ny, nx) device tensors; returns (S, L, report)."""
        S = torch.empty_like(y)
        L = torch.empty_like(y)
        rep = _lib.RpReport()
        rc = self.lib.rpca_solve(self._h, _ptr(y), _ptr(phi), _ptr(S), _ptr(L), ctypes.byref(rep))
        if rc != 0:
            raise UOTError(rc, "rpca_solve")
        return S, L, rep.as_dict()

    def planes(self, device="cuda"):
        """The split variables and multipliers; pair planes (Z, W, B, C) hold
        the T - 1 pairs, and with signed=True also Zm, Wm, Bm, Cm (the -
        pairs) and Sp, Sm."""
        T, ny, nx = self.shape
        npair = (2 if self.signed else 1) * (T - 1)
        out = {k: torch.empty((T if k in ("X", "Tn", "A", "D") else npair, ny, nx), dtype=torch.float32,
                              device=device) for k in self.PLANES}
        rc = self.lib.rpca_copy_planes(self._h, *[_ptr(out[k]) for k in self.PLANES])
        if rc != 0:
            raise UOTError(rc, "rpca_copy_planes")
        if self.signed:
            for k in ("Z", "W", "B", "C"):
                out[k + "m"] = out[k][T - 1:]
                out[k] = out[k][:T - 1]
            sp = torch.empty((T, ny, nx), dtype=torch.float32, device=device)
            sm = torch.empty_like(sp)
            rc = self.lib.rpca_copy_sparse(self._h, _ptr(sp), _ptr(sm))
            if rc != 0:
                raise UOTError(rc, "rpca_copy_sparse")
            out["Sp"], out["Sm"] = sp, sm
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.lib.rpca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
