"""The divergence D assembled entry by entry as a sparse matrix (FP64).

A second, independent implementation of the operator of Sec. II-A (the
divergence with at most 4 nonzeros per row), written with explicit loops over
pixels instead of array slicing.  Used by the pins (adjointness, lambda_max,
the Douglas-Rachford solver, the LP pins); test infrastructure only.

Vector layout: a pixel image is flattened with x fastest (k = j*nx + i, the
paper's column-major vec with i first).  The flux vector is [vec(Mx); vec(My)]
restricted to the entries that exist under the boundary reading:
  bc = 0  Mx[i, j] exists for i < nx-1, My[i, j] for j < ny-1
  bc = 1  every Mx[i, j] and My[i, j] exists
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def flux_index(nx, ny, bc=0):
    """Lists of (component, i, j) for the flux entries that exist."""
    ent = []
    for j in range(ny):
        for i in range(nx):
            if bc == 1 or i < nx - 1:
                ent.append((0, i, j))
    for j in range(ny):
        for i in range(nx):
            if bc == 1 or j < ny - 1:
                ent.append((1, i, j))
    return ent


def div_matrix(nx, ny, bc=0):
    """Sparse N x E matrix of D: flux entry Mx[i,j] adds +1 at pixel (i,j)
    and -1 at pixel (i+1,j) when that pixel exists; My[i,j] adds +1 at (i,j)
    and -1 at (i,j+1)."""
    ent = flux_index(nx, ny, bc)
    rows, cols, vals = [], [], []
    for e, (comp, i, j) in enumerate(ent):
        rows.append(j * nx + i)
        cols.append(e)
        vals.append(1.0)
        if comp == 0 and i + 1 < nx:
            rows.append(j * nx + i + 1)
            cols.append(e)
            vals.append(-1.0)
        if comp == 1 and j + 1 < ny:
            rows.append((j + 1) * nx + i)
            cols.append(e)
            vals.append(-1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nx * ny, len(ent)))


def pack_flux(Mx, My, bc=0):
    """(ny, nx) flux planes -> flux vector in ``flux_index`` order."""
    ny, nx = Mx.shape
    return np.array([(Mx if c == 0 else My)[j, i] for c, i, j in flux_index(nx, ny, bc)],
                    dtype=np.float64)


def unpack_flux(v, nx, ny, bc=0):
    """Flux vector -> (Mx, My) planes, structurally absent entries zero."""
    Mx = np.zeros((ny, nx))
    My = np.zeros((ny, nx))
    for val, (c, i, j) in zip(v, flux_index(nx, ny, bc)):
        (Mx if c == 0 else My)[j, i] = val
    return Mx, My


def pixel_pairs_of_flux(nx, ny, bc=0):
    """For each flux entry, the pixel it starts at (row of the +1)."""
    return np.array([j * nx + i for _, i, j in flux_index(nx, ny, bc)], dtype=np.int64)
