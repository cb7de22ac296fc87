"""Discrete operators of the Beckmann formulation, FP64 (test infrastructure).

Follows Sec. II-A of the paper (Beckmann's formulation, the l2,1 flux norm
and the divergence with zero-flux boundary) and the closed-form proximal
maps of Sec. III-B (the group shrink of the flux update and the scalar
shrink of the residual update).

Boundary readings (the text says flux is zero outside the support, but the
flux entries on the last column / last row are inside it):
  bc = 0  zero flux through the right and top edges: Mx[:, nx-1] and
          My[ny-1, :] are structurally zero.  D D* is then the Neumann
          Laplacian.  This is the default.
  bc = 1  the literal text: those entries are free variables, so mass may
          leave through the right / top edge.
"""
from __future__ import annotations

import numpy as np

DIST, PROX, PROX_FIXED = 0, 1, 2


def div(Mx, My, bc=0):
    """D M at every pixel: (Mx[i,j] - Mx[i-1,j]) + (My[i,j] - My[i,j-1]),
    flux outside the grid being zero (divergence definition, Sec. II-A)."""
    Mx = np.array(Mx, dtype=np.float64)
    My = np.array(My, dtype=np.float64)
    if bc == 0:
        Mx[:, -1] = 0.0
        My[-1, :] = 0.0
    out = Mx.copy()
    out[:, 1:] -= Mx[:, :-1]
    out += My
    out[1:, :] -= My[:-1, :]
    return out


def div_adj(a, bc=0):
    """D* a, the adjoint of ``div``: a negative forward difference,
    gx[i,j] = a[i,j] - a[i+1,j], gy[i,j] = a[i,j] - a[i,j+1], with a = 0
    outside the grid; under bc = 0 the components paired with structurally
    zero flux are zero."""
    a = np.asarray(a, dtype=np.float64)
    gx = a.copy()
    gx[:, :-1] -= a[:, 1:]
    gy = a.copy()
    gy[:-1, :] -= a[1:, :]
    if bc == 0:
        gx[:, -1] = 0.0
        gy[-1, :] = 0.0
    return gx, gy


def flux_norm(Mx, My, norm="iso"):
    """||M||_{2,1} = sum over pixels of sqrt(Mx^2 + My^2) (Sec. II-A).
    ``norm='aniso'`` gives the l1,1 variant sum |Mx| + |My| used by LP pins."""
    Mx = np.asarray(Mx, dtype=np.float64)
    My = np.asarray(My, dtype=np.float64)
    if norm == "iso":
        return float(np.sum(np.hypot(Mx, My)))
    return float(np.sum(np.abs(Mx)) + np.sum(np.abs(My)))


def dual_norm_max(gx, gy, norm="iso"):
    """max over pixels of the dual norm of (gx, gy): l2 for iso, l_inf for aniso."""
    if gx.size == 0:
        return 0.0
    if norm == "iso":
        return float(np.max(np.hypot(gx, gy)))
    return float(max(np.max(np.abs(gx)), np.max(np.abs(gy))))


def shrink2(vx, vy, sigma):
    """Group (vector) soft shrinkage of each 2-vector v:
    max(||v|| - sigma, 0) * v / ||v||, and 0 at v = 0 (flux update, Sec. III-B)."""
    vx = np.asarray(vx, dtype=np.float64)
    vy = np.asarray(vy, dtype=np.float64)
    n = np.hypot(vx, vy)
    scale = np.zeros_like(n)
    pos = n > sigma
    scale[pos] = (n[pos] - sigma) / n[pos]
    return scale * vx, scale * vy


def shrink1(v, sigma):
    """Scalar soft shrinkage sign(v) * max(|v| - sigma, 0), with sign(0) = 0
    (residual update for p = 1, Sec. III-B)."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v) * np.maximum(np.abs(v) - sigma, 0.0)


def prox_flux(vx, vy, sigma, norm="iso"):
    """Prox of sigma * ||.||_{2,1} (iso) or sigma * ||.||_{1,1} (aniso)."""
    if norm == "iso":
        return shrink2(vx, vy, sigma)
    return shrink1(vx, sigma), shrink1(vy, sigma)


def lam_max_1d(n, bc=0):
    """Largest eigenvalue of D1 D1^T for the 1-D difference operator of length n.

    bc = 0: the path-graph Laplacian, eigenvalues 4 sin^2(pi k / (2n)), k = 0..n-1.
    bc = 1: the tridiagonal matrix with diagonal (1, 2, ..., 2) and off-diagonal
            -1, eigenvalues 4 sin^2(pi (2k-1) / (2(2n+1))), k = 1..n.
    """
    n = int(n)
    if n < 1:
        raise ValueError("n >= 1 required")
    if bc == 0:
        return 4.0 * np.sin(np.pi * (n - 1) / (2.0 * n)) ** 2
    return 4.0 * np.sin(np.pi * (2 * n - 1) / (2.0 * (2 * n + 1))) ** 2


def lam_max(nx, ny, bc=0):
    """lambda_max(D D*) of the 2-D operator: D D* is the Kronecker sum of the
    two 1-D factors, so its top eigenvalue is the sum of theirs.  This is the
    discrete-Laplacian eigenvalue of Theorem 1."""
    return lam_max_1d(nx, bc) + lam_max_1d(ny, bc)


def n_identity_blocks(mode, balanced):
    """Number of +-I blocks in the constraint operator K besides D:
    DIST: r; PROX: x0, x1, r; PROX_FIXED: x, r (balanced drops r)."""
    base = {DIST: 1, PROX: 3, PROX_FIXED: 2}[mode]
    return base - (1 if balanced else 0)


def knorm2(nx, ny, mode, balanced, bc=0):
    """||K||^2 = lambda_max(K K*) = lambda_max(D D*) + (number of identity
    blocks), by the eigenvalue argument in the proof of Theorem 1."""
    return lam_max(nx, ny, bc) + n_identity_blocks(mode, balanced)
