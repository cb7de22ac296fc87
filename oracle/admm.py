"""ADMM solvers of Sec. IV that call the UOT prox, in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

UOT-DF (Sec. IV-A, eqs. ``UOT-DF`` and ``BPDN+UOT-DF``, Algorithm 2):

    min_{s >= 0}  1/2 ||y - Phi s||^2 + lam ||s||_1 + kappa V_mu(s, s0)

split as s = x = z with multipliers a, b and penalty rho; one ADMM iteration,
in the order of Algorithm 2:

    s <- argmin lam ||s||_1 + indicator(s >= 0)
                + rho/2 (||x - s + a||^2 + ||z - s + b||^2)
       = max(((x + a) + (z + b))/2 - lam/(2 rho), 0)
    x <- (Phi^T Phi + rho I)^{-1} (Phi^T y + rho (s - a))
    z <- prox of (kappa/rho) V_mu(., s0) at s - b      (Algorithm 1, warm-started,
                                                         a fixed number of passes)
    a <- a + x - s
    b <- b + z - s

Stopping (the paper's, after Boyd et al. Sec. 3.3.1): both
    ||[x - s; z - s]||  and  rho ||[x - x_prev; z - z_prev]||  below eps.

Readings:
  - The s-step minimises the augmented Lagrangian the paper writes down,
    which holds both penalty terms in s.  The printed line keeps only the
    x-block, max(x + a - ., 0); with it the z-block never feeds back into s
    and the iteration settles at the transport-free least-squares point
    (s = y for Phi = I), which the single-pixel closed form rules out.  The
    step taken is the average of both blocks, the s-step of Algorithm 3 with
    sigma = 2.  Its threshold is lam/(2 rho); the printed rho/lam is the
    reciprocal of the one-block threshold lam/rho.
  - V_mu is symmetric in its arguments (swap M -> -M, r -> -r), so the
    z-prox of V_mu(z, s0) is the one-argument-fixed prox (Prox_UOT_specialcase)
    with the fixed argument s0 and prox centre s - b, prox step kappa/rho.
  - Phi is diagonal here (a vector phi, None = identity): the x-step is then
    element-wise.  Dense Phi (the 10x10 compressed-sensing experiment) is not
    part of the path.
  - Algorithm 2 starts every variable, and the prox state, at zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import uot
from .ops import PROX_FIXED


@dataclass
class DfReport:
    iters: int = 0
    converged: bool = False
    r_primal: float = float("nan")
    r_dual: float = float("nan")
    history: list = field(default_factory=list)


@dataclass
class DfState:
    s: np.ndarray
    x: np.ndarray
    z: np.ndarray
    a: np.ndarray
    b: np.ndarray
    prox: uot.State


def df_problem(s0, centre, kappa, mu, rho, balanced=False, residual_p=1, bc=0):
    """The z-subproblem as an Algorithm-1 problem: PROX_FIXED with the fixed
    argument s0, prox centre `centre` and prox step kappa/rho."""
    return uot.Problem(np.asarray(s0, float), np.asarray(centre, float), mode=PROX_FIXED, balanced=balanced,
                       residual_p=residual_p, bc=bc, mu=mu, rho=kappa / rho)


def df_initial_state(s0, kappa, mu, rho, balanced=False, residual_p=1, bc=0) -> DfState:
    s0 = np.asarray(s0, float)
    z = np.zeros_like(s0)
    prob = df_problem(s0, z, kappa, mu, rho, balanced, residual_p, bc)
    return DfState(z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), uot.initial_state(prob))


def df_iterate(y, s0, st: DfState, kappa, mu, rho, phi=None, lam=0.0, balanced=False, residual_p=1, bc=0,
               prox_iters=1, tau=None) -> DfState:
    """One ADMM iteration of Algorithm 2 (see the module docstring)."""
    y = np.asarray(y, float)
    ph = np.ones_like(y) if phi is None else np.asarray(phi, float)
    s = np.maximum(0.5 * ((st.x + st.a) + (st.z + st.b)) - lam / (2.0 * rho), 0.0)
    x = (ph * y + rho * (s - st.a)) / (ph * ph + rho)
    prob = df_problem(s0, s - st.b, kappa, mu, rho, balanced, residual_p, bc)
    t1, t2 = prob.default_steps() if tau is None else tau
    pst = st.prox
    for _ in range(prox_iters):
        pst = uot.iterate(prob, pst, t1, t2)
    z = pst.x1.copy()
    a = st.a + x - s
    b = st.b + z - s
    return DfState(s, x, z, a, b, pst)


def df_residuals(prev: DfState, cur: DfState, rho):
    rp = np.sqrt(np.sum((cur.x - cur.s) ** 2) + np.sum((cur.z - cur.s) ** 2))
    rd = rho * np.sqrt(np.sum((cur.x - prev.x) ** 2) + np.sum((cur.z - prev.z) ** 2))
    return float(rp), float(rd)


def uotdf(y, s0, kappa, mu, rho, phi=None, lam=0.0, balanced=False, residual_p=1, bc=0, prox_iters=1,
          max_iter=5000, eps=1e-3, check_every=1, tau=None, record=False):
    """Algorithm 2 until both residuals are below eps (tested every
    check_every iterations) or max_iter; returns (s, state, report)."""
    st = df_initial_state(s0, kappa, mu, rho, balanced, residual_p, bc)
    rep = DfReport()
    for k in range(1, max_iter + 1):
        nxt = df_iterate(y, s0, st, kappa, mu, rho, phi, lam, balanced, residual_p, bc, prox_iters, tau)
        if k % check_every == 0 or k == max_iter:
            rp, rd = df_residuals(st, nxt, rho)
            rep.r_primal, rep.r_dual = rp, rd
            if record:
                rep.history.append((k, rp, rd))
            if rp < eps and rd < eps:
                rep.iters, rep.converged = k, True
                return nxt.s, nxt, rep
        st = nxt
    rep.iters = max_iter
    return st.s, st, rep


def uotdf_objective(y, s, s0, kappa, mu, phi=None, lam=0.0, balanced=False):
    """1/2 ||y - Phi s||^2 + lam ||s||_1 + kappa V(s, s0), with V from the
    linear program (exact for grids one pixel high or wide, where the flux
    norms coincide)."""
    from .lp import beckmann_aniso
    y = np.asarray(y, float)
    s = np.asarray(s, float)
    ph = np.ones_like(y) if phi is None else np.asarray(phi, float)
    v = beckmann_aniso(s, np.asarray(s0, float), mu=None if balanced else mu, balanced=balanced)
    return 0.5 * float(np.sum((y - ph * s) ** 2)) + lam * float(np.sum(np.abs(s))) + kappa * v
