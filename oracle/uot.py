"""Algorithm 1 of the paper (the primal-dual prox iteration) in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

What is computed (Sec. III, eqs. ``Unbal_OT_beckman``, ``Prox_UOT`` and the
special case ``Prox_UOT_specialcase``), with one constraint operator for all
modes,  K(z) = D M - x0 + x1 - r  (the sign convention of the prox and the
special case; the distance is symmetric, so values do not depend on it):

  DIST        x0 = p, x1 = q fixed:  min ||M||_{2,1} + mu ||r||_p^p  s.t. K = 0
  PROX        min over x0, x1 >= 0 of the above + ||x - (p0, p1)||^2 / (2 rho)
  PROX_FIXED  x0 = s fixed, min over x1 >= 0 of the above + ||x1 - p||^2/(2 rho)
  balanced    r is dropped (footnote to the balanced-vs-unbalanced experiment)

One iteration (Sec. III-B, the Chambolle-Pock updates and Algorithm 1):
  M  <- group-shrink_{tau1}(M - tau1 D* a)
  x  <- max(theta p + (1 - theta)(x - tau1 A^T a), 0),  theta = tau1/(rho + tau1)
  r  <- shrink_{mu tau1}(r + tau1 a)            (p = 1)
        (r + tau1 a) / (1 + 2 mu tau1)           (p = 2, the "averaging" update)
  a  <- a + tau2 (2 K(z_new) - K(z_old))

Reading of rho: the prox is defined with the weight 1/(2 rho); the exact
argmin of the x-subproblem under that definition is theta = tau1/(rho+tau1).
The paper's printed theta, rho tau1/(1 + rho tau1), is the same map with rho
read as the quadratic weight; both agree at rho = 1.

Stopping rule (the paper leaves "while not converged" open):
  rel_res = max( ||K z^k|| / max(||x0^k|| + ||x1^k||, 1e-30),
                 ||(z^{k-1} - z^k)/tau1 - K*(a^{k-1} - a^k)|| / max(||K* a^k||, 1e-30) )
the primal-feasibility and stationarity residuals of the saddle-point
conditions of the Lagrangian (eq. ``eqn:saddle``).

Certified duality gap: a feasible primal value P_hat >= V >= D_hat, a dual
value of the scaled multiplier a / s that satisfies the dual constraints
(derived from the Lagrangian of Sec. III-B).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import ops
from .ops import DIST, PROX, PROX_FIXED


@dataclass
class Problem:
    """Inputs in the paper's problem statement.

    src, dst: DIST -> (p, q); PROX -> (p0, p1); PROX_FIXED -> (s, p).
    """
    src: np.ndarray
    dst: np.ndarray
    mode: int = DIST
    balanced: bool = False
    residual_p: int = 1
    bc: int = 0
    mu: float = 1.0
    rho: float = 1.0
    norm: str = "iso"

    def __post_init__(self):
        self.src = np.asarray(self.src, dtype=np.float64)
        self.dst = np.asarray(self.dst, dtype=np.float64)
        if self.src.shape != self.dst.shape or self.src.ndim != 2:
            raise ValueError("src and dst must be 2-D arrays of one shape")

    @property
    def shape(self):
        return self.src.shape

    def knorm2(self):
        ny, nx = self.shape
        return ops.knorm2(nx, ny, self.mode, self.balanced, self.bc)

    def image_scale(self):
        """s = the largest |pixel| of the two images (1 if both are zero)."""
        s = max(float(np.max(np.abs(self.src), initial=0.0)), float(np.max(np.abs(self.dst), initial=0.0)))
        return s if np.isfinite(s) and s > 0.0 else 1.0

    def unit_steps(self):
        """tau1 = tau2 = 0.99 / ||K||, so tau1 tau2 ||K||^2 = 0.98 < 1 (Theorem 1)."""
        t = 0.99 / np.sqrt(self.knorm2())
        return t, t

    def default_steps(self):
        """Steps that follow the image scale s (``image_scale``):
        tau1 = 0.99 s / ||K||, tau2 = 0.99 / (s ||K||).

        The paper tunes its steps by search.  This default uses the
        1-homogeneity of the problem: with both images scaled by t the
        minimisers M, r scale by t and the multiplier a does not change, and
        one iteration on the scaled images with (tau1, tau2) is one iteration
        on the originals with (tau1 / t, tau2 t).  Tying tau1 / tau2 to s^2
        makes the iterates of scaled images the scaled iterates.  The product
        tau1 tau2 ||K||^2 = 0.98 < 1 (Theorem 1) does not depend on s."""
        k = np.sqrt(self.knorm2())
        s = self.image_scale()
        return 0.99 * s / k, 0.99 / (s * k)


@dataclass
class State:
    Mx: np.ndarray
    My: np.ndarray
    r: np.ndarray
    a: np.ndarray
    x0: np.ndarray
    x1: np.ndarray

    def copy(self):
        return State(*(np.array(v, dtype=np.float64, copy=True) for v in
                       (self.Mx, self.My, self.r, self.a, self.x0, self.x1)))


def initial_state(prob: Problem, warm: State | None = None) -> State:
    """Zero start (the paper initialises the prox variables to 0), or the
    caller's state; the fixed arguments are pinned to the inputs."""
    ny, nx = prob.shape
    z = np.zeros((ny, nx))
    if warm is None:
        st = State(z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy())
    else:
        st = warm.copy()
    if prob.bc == 0:
        st.Mx[:, -1] = 0.0
        st.My[-1, :] = 0.0
    if prob.balanced:
        st.r[:] = 0.0
    if prob.mode == DIST:
        st.x0, st.x1 = prob.src.copy(), prob.dst.copy()
    elif prob.mode == PROX_FIXED:
        st.x0 = prob.src.copy()
    return st


def constraint(prob: Problem, Mx, My, x0, x1, r):
    """K(z) = D M - x0 + x1 - r (r absent when balanced)."""
    k = ops.div(Mx, My, prob.bc) - x0 + x1
    if not prob.balanced:
        k = k - r
    return k


def iterate(prob: Problem, st: State, tau1: float, tau2: float) -> State:
    """One pass of Algorithm 1: flux, projection, residual, dual steps."""
    gx, gy = ops.div_adj(st.a, prob.bc)
    Mx, My = ops.prox_flux(st.Mx - tau1 * gx, st.My - tau1 * gy, tau1, prob.norm)
    x0, x1 = st.x0, st.x1
    theta = tau1 / (prob.rho + tau1)
    if prob.mode == PROX:
        x0 = np.maximum(theta * prob.src + (1.0 - theta) * (st.x0 + tau1 * st.a), 0.0)
        x1 = np.maximum(theta * prob.dst + (1.0 - theta) * (st.x1 - tau1 * st.a), 0.0)
    elif prob.mode == PROX_FIXED:
        x1 = np.maximum(theta * prob.dst + (1.0 - theta) * (st.x1 - tau1 * st.a), 0.0)
    if prob.balanced:
        r = st.r
    elif prob.residual_p == 1:
        r = ops.shrink1(st.r + tau1 * st.a, prob.mu * tau1)
    else:
        r = (st.r + tau1 * st.a) / (1.0 + 2.0 * prob.mu * tau1)
    k_old = constraint(prob, st.Mx, st.My, st.x0, st.x1, st.r)
    k_new = constraint(prob, Mx, My, x0, x1, r)
    a = st.a + tau2 * (2.0 * k_new - k_old)
    return State(Mx, My, r, a, x0, x1)


def _kstar_sq(prob, a):
    gx, gy = ops.div_adj(a, prob.bc)
    nid = ops.n_identity_blocks(prob.mode, prob.balanced)
    return float(np.sum(gx * gx) + np.sum(gy * gy) + nid * np.sum(a * a))


def residuals(prob: Problem, prev: State, cur: State, tau1: float):
    """(primal, stationarity, rel_res) of the stopping rule in the header."""
    kz = constraint(prob, cur.Mx, cur.My, cur.x0, cur.x1, cur.r)
    pnorm = float(np.linalg.norm(kz))
    xn = float(np.linalg.norm(cur.x0) + np.linalg.norm(cur.x1))
    da = prev.a - cur.a
    dgx, dgy = ops.div_adj(da, prob.bc)
    sx = (prev.Mx - cur.Mx) / tau1 - dgx
    sy = (prev.My - cur.My) / tau1 - dgy
    if prob.bc == 0:
        sx[:, -1] = 0.0
        sy[-1, :] = 0.0
    s2 = float(np.sum(sx * sx) + np.sum(sy * sy))
    if not prob.balanced:
        sr = (prev.r - cur.r) / tau1 + da
        s2 += float(np.sum(sr * sr))
    if prob.mode == PROX:
        s0 = (prev.x0 - cur.x0) / tau1 + da
        s2 += float(np.sum(s0 * s0))
    if prob.mode in (PROX, PROX_FIXED):
        s1 = (prev.x1 - cur.x1) / tau1 - da
        s2 += float(np.sum(s1 * s1))
    snorm = np.sqrt(s2)
    ka = np.sqrt(_kstar_sq(prob, cur.a))
    rel = max(pnorm / max(xn, 1e-30), snorm / max(ka, 1e-30))
    return pnorm, snorm, rel


def _poisson_pinv(nx, ny, bc, rhs):
    """phi = (D D*)^+ rhs by dense least squares (small grids only)."""
    from .sparse_ops import div_matrix
    D = div_matrix(nx, ny, bc).toarray()
    L = D @ D.T
    phi, *_ = np.linalg.lstsq(L, rhs.reshape(-1), rcond=None)
    return phi.reshape(ny, nx)


def feasible_flux(prob: Problem, Mx, My, e, poisson=None):
    """Least-change feasible flux: M_hat = M - D*(D D*)^+ e, so that D M_hat
    equals D M - e where e lies in the range of D.  ``poisson(rhs)`` solves
    (D D*) phi = rhs; by default a dense solve."""
    ny, nx = prob.shape
    solve = poisson if poisson is not None else (lambda r: _poisson_pinv(nx, ny, prob.bc, r))
    phi = solve(e)
    gx, gy = ops.div_adj(phi, prob.bc)
    return Mx - gx, My - gy


@dataclass
class Gap:
    primal: float
    dual: float
    rel_gap: float
    feas: float
    objective: float   # raw objective of the iterate (no feasibility repair)


def certified_gap(prob: Problem, st: State, poisson=None) -> Gap:
    """Primal upper bound P_hat, dual lower bound D_hat and their relative gap."""
    ny, nx = prob.shape
    mu, rho = prob.mu, prob.rho
    e = constraint(prob, st.Mx, st.My, st.x0, st.x1, np.zeros_like(st.a))  # D M - x0 + x1
    feas = float(np.linalg.norm(constraint(prob, st.Mx, st.My, st.x0, st.x1, st.r)))
    mnorm = ops.flux_norm(st.Mx, st.My, prob.norm)
    quad = 0.0
    if prob.mode == PROX:
        quad = float(np.sum((st.x0 - prob.src) ** 2) + np.sum((st.x1 - prob.dst) ** 2)) / (2 * rho)
    elif prob.mode == PROX_FIXED:
        quad = float(np.sum((st.x1 - prob.dst) ** 2)) / (2 * rho)
    if prob.balanced:
        obj = mnorm + quad
    elif prob.residual_p == 1:
        obj = mnorm + mu * float(np.sum(np.abs(st.r))) + quad
    else:
        obj = mnorm + mu * float(np.sum(st.r ** 2)) + quad

    # ---- primal bound from a feasible point ----
    if not prob.balanced:
        # absorb the infeasibility into r: r_hat = D M - x0 + x1
        pen = np.sum(np.abs(e)) if prob.residual_p == 1 else np.sum(e * e)
        primal = mnorm + mu * float(pen) + quad
    else:
        x0, x1 = st.x0, st.x1
        if prob.bc == 0 and prob.mode != DIST:
            # D M sums to zero under bc=0: rescale the free argument so the
            # masses agree before repairing the flux.
            t0, t1 = float(np.sum(x0)), float(np.sum(x1))
            if prob.mode == PROX and t1 > 0:
                x1 = x1 * (t0 / t1)
            elif prob.mode == PROX_FIXED and t1 > 0:
                x1 = x1 * (t0 / t1)
        e2 = ops.div(st.Mx, st.My, prob.bc) - x0 + x1
        Mh_x, Mh_y = feasible_flux(prob, st.Mx, st.My, e2, poisson)
        q2 = 0.0
        if prob.mode == PROX:
            q2 = float(np.sum((x0 - prob.src) ** 2) + np.sum((x1 - prob.dst) ** 2)) / (2 * rho)
        elif prob.mode == PROX_FIXED:
            q2 = float(np.sum((x1 - prob.dst) ** 2)) / (2 * rho)
        primal = ops.flux_norm(Mh_x, Mh_y, prob.norm) + q2

    # ---- dual bound from the scaled multiplier ----
    gx, gy = ops.div_adj(st.a, prob.bc)
    s = max(1.0, ops.dual_norm_max(gx, gy, prob.norm))
    if not prob.balanced and prob.residual_p == 1:
        s = max(s, float(np.max(np.abs(st.a))) / mu if st.a.size else 0.0)
    ah = st.a / s
    if prob.mode == DIST:
        dual = float(np.sum(ah * (prob.dst - prob.src)))
    elif prob.mode == PROX:
        x0s = np.maximum(prob.src + rho * ah, 0.0)
        x1s = np.maximum(prob.dst - rho * ah, 0.0)
        dual = float(np.sum((x0s - prob.src) ** 2 / (2 * rho) - ah * x0s)
                     + np.sum((x1s - prob.dst) ** 2 / (2 * rho) + ah * x1s))
    else:
        x1s = np.maximum(prob.dst - rho * ah, 0.0)
        dual = float(-np.sum(ah * prob.src)
                     + np.sum((x1s - prob.dst) ** 2 / (2 * rho) + ah * x1s))
    if not prob.balanced and prob.residual_p == 2:
        dual -= float(np.sum(ah * ah)) / (4.0 * mu)
    rel_gap = (primal - dual) / max(abs(primal), 1e-30)
    return Gap(primal, dual, rel_gap, feas, obj)


@dataclass
class Report:
    iters: int = 0
    status: str = "MAX_ITER"
    rel_res: float = float("inf")
    history: list = field(default_factory=list)
    tau1: float = 0.0
    tau2: float = 0.0


def relative_residuals(prob: Problem, prev: State, cur: State, tau1: float):
    """(feasibility / (||x0|| + ||x1||), stationarity / ||K* a||): the two
    parts of the stopping rule, each scale-free."""
    pn, sn, _ = residuals(prob, prev, cur, tau1)
    xn = float(np.linalg.norm(cur.x0) + np.linalg.norm(cur.x1))
    ka = np.sqrt(_kstar_sq(prob, cur.a))
    return pn / max(xn, 1e-30), sn / max(ka, 1e-30)


def solve(prob: Problem, tau1=None, tau2=None, max_iter=1000, check_every=20, tol=0.0,
          state: State | None = None, record=False, adaptive=False, gap_tol=0.0, gap_every=1000):
    """Run Algorithm 1 from zero (or ``state``) until rel_res <= tol at a
    check (every ``check_every`` iterations) or ``max_iter`` iterations.
    tol <= 0 runs exactly ``max_iter`` iterations.

    gap_tol > 0 also stops (status "CONVERGED") at the first multiple of
    ``gap_every`` where the certified relative gap (``certified_gap``) is
    <= gap_tol, so that a run can be certified rather than trusted.

    adaptive: the paper fixes no step rule (its steps come from a parameter
    search).  With ``adaptive`` the product tau1 tau2 is kept and the ratio
    is rebalanced at every check by residual balancing (the adaptive
    primal-dual hybrid gradient method of Goldstein, Li and Yuan): if the
    relative stationarity residual exceeds 1.5 times the relative
    feasibility residual, tau1 /= (1 - alpha), tau2 *= (1 - alpha); in the
    opposite case the reverse; alpha starts at 0.5 and shrinks by 0.95 per
    change, so the steps settle."""
    d1, d2 = prob.default_steps()
    tau1 = d1 if tau1 is None else float(tau1)
    tau2 = d2 if tau2 is None else float(tau2)
    st = initial_state(prob, state)
    rep = Report()
    alpha = 0.5
    if prob.mode == DIST and not np.any(prob.src) and not np.any(prob.dst) and state is None:
        rep.status, rep.rel_res = "CONVERGED", 0.0
        return st, rep
    for k in range(1, max_iter + 1):
        prev = st
        st = iterate(prob, st, tau1, tau2)
        if not np.all(np.isfinite(st.a)):
            rep.iters, rep.status = k, "DIVERGED"
            return st, rep
        if gap_tol > 0 and k % gap_every == 0 and certified_gap(prob, st).rel_gap <= gap_tol:
            rep.iters, rep.status = k, "CONVERGED"
            rep.rel_res = max(relative_residuals(prob, prev, st, tau1))
            rep.tau1, rep.tau2 = tau1, tau2
            return st, rep
        if (tol > 0 and k % check_every == 0) or (k == max_iter):
            rp, rd = relative_residuals(prob, prev, st, tau1)
            rel = max(rp, rd)
            rep.rel_res = rel
            if record:
                rep.history.append((k, rel))
            if tol > 0 and rel <= tol:
                rep.iters, rep.status = k, "CONVERGED"
                rep.tau1, rep.tau2 = tau1, tau2
                return st, rep
            if adaptive and tol > 0 and k < max_iter:
                if rd > 1.5 * rp:
                    tau1, tau2, alpha = tau1 / (1 - alpha), tau2 * (1 - alpha), alpha * 0.95
                elif rp > 1.5 * rd:
                    tau1, tau2, alpha = tau1 * (1 - alpha), tau2 / (1 - alpha), alpha * 0.95
    rep.iters = max_iter
    rep.tau1, rep.tau2 = tau1, tau2
    return st, rep


def value(prob: Problem, **kw) -> float:
    """V_mu(p, q) (DIST) or the prox objective, by running Algorithm 1 and
    returning the certified primal bound."""
    st, _ = solve(prob, **kw)
    return certified_gap(prob, st).primal


def with_(prob: Problem, **kw) -> Problem:
    return replace(prob, **kw)
