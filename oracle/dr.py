"""An independent FP64 solver for the same convex programs (small grids).

TEST INFRASTRUCTURE ONLY.  Douglas-Rachford splitting of
    min_z  G(z) + indicator{ K z = b }
where G collects the separable terms (flux norm, residual penalty, the prox
quadratic and x >= 0) and the affine constraint is the divergence constraint
of eqs. ``Unbal_OT_beckman`` / ``Prox_UOT`` / ``Prox_UOT_specialcase``.  The
projection onto {K z = b} is a dense solve with the loop-assembled D, so this
route shares neither algorithm nor operator code with Algorithm 1 in
``oracle.uot``; the proximal maps of G are written out here on their own.

Variables z (vector layout of ``sparse_ops``):
  DIST        (m, r)           K z = D m - r,            b = p - q
  PROX        (m, x0, x1, r)   K z = D m - x0 + x1 - r,  b = 0
  PROX_FIXED  (m, x1, r)       K z = D m + x1 - r,       b = s
(balanced drops r).
"""
from __future__ import annotations

import numpy as np

from .sparse_ops import div_matrix, flux_index

DIST, PROX, PROX_FIXED = 0, 1, 2


class DRSolver:
    def __init__(self, src, dst, mode=DIST, balanced=False, residual_p=1, bc=0, mu=1.0, rho=1.0,
                 gamma=1.0):
        self.src = np.asarray(src, dtype=np.float64)
        self.dst = np.asarray(dst, dtype=np.float64)
        ny, nx = self.src.shape
        self.nx, self.ny = nx, ny
        self.mode, self.balanced, self.residual_p, self.bc = mode, balanced, residual_p, bc
        self.mu, self.rho, self.gamma = float(mu), float(rho), float(gamma)
        D = div_matrix(nx, ny, bc).toarray()
        N, E = D.shape
        self.N, self.E = N, E
        blocks = [D]
        names = ["m"]
        if mode == PROX:
            blocks += [-np.eye(N), np.eye(N)]
            names += ["x0", "x1"]
        elif mode == PROX_FIXED:
            blocks += [np.eye(N)]
            names += ["x1"]
        if not balanced:
            blocks += [-np.eye(N)]
            names += ["r"]
        self.K = np.hstack(blocks)
        self.names = names
        offs, o = {}, 0
        for nm, blk in zip(names, blocks):
            offs[nm] = (o, o + blk.shape[1])
            o += blk.shape[1]
        self.offs = offs
        if mode == DIST:
            b = (self.src - self.dst).reshape(-1)
        elif mode == PROX:
            b = np.zeros(N)
        else:
            b = self.src.reshape(-1).copy()
        self.b = b
        KKt = self.K @ self.K.T
        Kp = np.linalg.pinv(KKt)
        self.P = np.eye(self.K.shape[1]) - self.K.T @ Kp @ self.K
        self.z0 = self.K.T @ (Kp @ b)
        # pixel of each flux entry and component, for the group shrink
        ent = flux_index(nx, ny, bc)
        self.fpix = np.array([j * nx + i for _, i, j in ent])
        self.fcomp = np.array([c for c, _, _ in ent])

    def project(self, y):
        return self.P @ y + self.z0

    def _prox_flux(self, v, t):
        # group soft threshold per pixel of the (Mx, My) pair, written out
        sq = np.zeros(self.N)
        np.add.at(sq, self.fpix, v * v)
        nrm = np.sqrt(sq)
        fac = np.where(nrm > t, 1.0 - t / np.where(nrm > 0, nrm, 1.0), 0.0)
        return v * fac[self.fpix]

    def prox_G(self, w):
        g = self.gamma
        z = w.copy()
        a, b = self.offs["m"]
        z[a:b] = self._prox_flux(w[a:b], g)
        if "r" in self.offs:
            a, b = self.offs["r"]
            v = w[a:b]
            if self.residual_p == 1:
                z[a:b] = np.sign(v) * np.maximum(np.abs(v) - g * self.mu, 0.0)
            else:
                z[a:b] = v / (1.0 + 2.0 * g * self.mu)
        for nm, p in (("x0", self.src), ("x1", self.dst)):
            if nm in self.offs:
                a, b = self.offs[nm]
                pv = p.reshape(-1)
                z[a:b] = np.maximum((g * pv + self.rho * w[a:b]) / (self.rho + g), 0.0)
        return z

    def objective(self, z):
        a, b = self.offs["m"]
        sq = np.zeros(self.N)
        np.add.at(sq, self.fpix, z[a:b] ** 2)
        val = float(np.sum(np.sqrt(sq)))
        if "r" in self.offs:
            a, b = self.offs["r"]
            val += self.mu * float(np.sum(np.abs(z[a:b])) if self.residual_p == 1 else np.sum(z[a:b] ** 2))
        for nm, p in (("x0", self.src), ("x1", self.dst)):
            if nm in self.offs:
                a, b = self.offs[nm]
                val += float(np.sum((z[a:b] - p.reshape(-1)) ** 2)) / (2 * self.rho)
        return val

    def solve(self, iters=20000, w0=None, tol=1e-13):
        w = np.zeros(self.K.shape[1]) if w0 is None else w0.copy()
        z = self.prox_G(w)
        for k in range(iters):
            z = self.prox_G(w)
            y = self.project(2 * z - w)
            step = y - z
            w = w + step
            if k % 200 == 0 and np.linalg.norm(step) <= tol * max(1.0, np.linalg.norm(z)):
                break
        return z

    def unpack(self, z):
        out = {}
        a, b = self.offs["m"]
        Mx = np.zeros((self.ny, self.nx))
        My = np.zeros((self.ny, self.nx))
        for val, pix, c in zip(z[a:b], self.fpix, self.fcomp):
            (Mx if c == 0 else My).flat[pix] = val
        out["Mx"], out["My"] = Mx, My
        for nm in ("x0", "x1", "r"):
            if nm in self.offs:
                a, b = self.offs[nm]
                out[nm] = z[a:b].reshape(self.ny, self.nx)
        return out
