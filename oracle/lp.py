"""Linear-programming pins (scipy HiGHS), FP64.  Test infrastructure only.

Two independent LP routes to the anisotropic (l1,1 flux norm) value:

  beckmann_aniso   min sum|M| + mu sum|r|  s.t.  D M - p + q = r, written with
                   the loop-assembled sparse D (the Beckmann form, eq.
                   ``OT_beckman`` / ``Unbal_OT_beckman`` with l1,1 in place of
                   l2,1); balanced drops r.
  kantorovich      eq. ``Unbal_OT`` with exponent 1 and the Manhattan ground
                   cost |i-i'| + |j-j'|:  min <P, C> + mu(|P1 - p| + |P^T 1 - q|)
                   over P >= 0; balanced is eq. ``OT`` (P1 = p, P^T 1 = q).

Under the zero-flux boundary the grid's 4-neighbour graph distance is the
Manhattan distance, so the two LPs have the same value; both pin the
anisotropic variant of the iteration.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

from .sparse_ops import div_matrix


def beckmann_aniso(p, q, mu=None, bc=0, balanced=False):
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    ny, nx = p.shape
    D = div_matrix(nx, ny, bc)
    N, E = D.shape
    b = (p - q).reshape(-1)
    if balanced:
        # variables [M+, M-]
        A = sp.hstack([D, -D]).tocsr()
        c = np.ones(2 * E)
    else:
        I = sp.identity(N, format="csr")
        A = sp.hstack([D, -D, -I, I]).tocsr()
        c = np.concatenate([np.ones(2 * E), mu * np.ones(2 * N)])
    res = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun)


def manhattan_cost(nx, ny):
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ii, jj = ii.reshape(-1), jj.reshape(-1)
    return (np.abs(ii[:, None] - ii[None, :]) + np.abs(jj[:, None] - jj[None, :])).astype(np.float64)


def kantorovich(p, q, mu=None, balanced=False, cost=None):
    p = np.asarray(p, dtype=np.float64).reshape(-1)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    N = p.size
    C = cost if cost is not None else None
    if C is None:
        raise ValueError("cost matrix required")
    nP = N * N
    # row sums (P 1)_i: coefficient 1 on P[i, :]; column sums on P[:, j]
    rows_r = np.repeat(np.arange(N), N)
    cols_r = np.arange(nP)
    R = sp.csr_matrix((np.ones(nP), (rows_r, cols_r)), shape=(N, nP))
    rows_c = np.tile(np.arange(N), N)
    Cm = sp.csr_matrix((np.ones(nP), (rows_c, cols_r)), shape=(N, nP))
    if balanced:
        A = sp.vstack([R, Cm]).tocsr()
        b = np.concatenate([p, q])
        c = C.reshape(-1)
    else:
        # P1 - p = u+ - u-,  P^T1 - q = v+ - v-
        I = sp.identity(N, format="csr")
        Z = sp.csr_matrix((N, N))
        A = sp.vstack([sp.hstack([R, -I, I, Z, Z]), sp.hstack([Cm, Z, Z, -I, I])]).tocsr()
        b = np.concatenate([p, q])
        c = np.concatenate([C.reshape(-1), mu * np.ones(4 * N)])
    res = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun)
