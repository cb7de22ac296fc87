"""Neumann-Poisson solves, FP64.  Test infrastructure only.

Under the zero-flux boundary D D* is the grid Laplacian with Neumann ends,
whose eigenvectors are the DCT-II basis, with eigenvalues
    4 sin^2(pi kx / (2 nx)) + 4 sin^2(pi ky / (2 ny)).
``dct_solve`` solves (alpha I + D D*) phi = c through that diagonalisation;
``direct_solve`` does the same with a dense solve of the loop-assembled
matrix (least squares when alpha = 0, where the constant mode is the
null space and c must have zero mean).
"""
from __future__ import annotations

import numpy as np
from scipy.fft import dctn, idctn

from .sparse_ops import div_matrix


def eigenvalues(nx, ny):
    kx = np.arange(nx)
    ky = np.arange(ny)
    lx = 4.0 * np.sin(np.pi * kx / (2.0 * nx)) ** 2
    ly = 4.0 * np.sin(np.pi * ky / (2.0 * ny)) ** 2
    return ly[:, None] + lx[None, :]


def dct_solve(c, alpha=0.0):
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    lam = alpha + eigenvalues(nx, ny)
    ch = dctn(c, type=2, norm="ortho")
    with np.errstate(divide="ignore", invalid="ignore"):
        ph = np.where(lam > 0, ch / np.where(lam > 0, lam, 1.0), 0.0)
    return idctn(ph, type=2, norm="ortho")


def direct_solve(c, alpha=0.0, bc=0):
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    D = div_matrix(nx, ny, bc).toarray()
    A = alpha * np.eye(nx * ny) + D @ D.T
    if alpha > 0 or bc == 1:
        return np.linalg.solve(A, c.reshape(-1)).reshape(ny, nx)
    phi, *_ = np.linalg.lstsq(A, c.reshape(-1), rcond=None)
    phi -= phi.mean()
    return phi.reshape(ny, nx)
