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
    which holds both penalty terms in s.  The printed update keeps only the
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
    t1, t2 = prob.unit_steps() if tau is None else tau
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


# ---------------------------------------------------------------------------
# RPCA+UOT-DF (Sec. IV-B, eq. RPCA_UOTDF, Algorithm 3):
#
#   min_{S, L >= 0} 1/2 sum_t ||y_t - Phi_t (s_t + l_t)||^2 + lam ||S||_1
#                   + gam ||L||_* + kappa sum_{t<T} V_mu(s_t, s_{t+1})
#
# frames are the first axis (S[t] is frame t, an ny x nx image).  Splitting
# X = S + L, Tn = L, z_t = s_t, w_{t+1} = s_{t+1} with multipliers A, D, b, c
# and penalty rho, one ADMM iteration in the order of Algorithm 3:
#
#   k_t  = (x_t - l_t + a_t) + wz_t (z_t + b_t) + ww_t (w_t + c_t)
#   s_t  = max(k_t / sig_t - lam / (rho sig_t), 0),  sig_t = 1 + wz_t + ww_t
#   L    = max((Tn - D + X - S + A) / 2, 0)
#   x_t  = (Phi_t^T Phi_t + rho I)^{-1} (Phi_t^T y_t + rho (s_t + l_t - a_t))
#   Tn   = SVT_{gam/rho}(L + D)          (singular-value soft threshold)
#   (z_t, w_{t+1}) = prox_{(kappa/rho) V_mu}(s_t - b_t, s_{t+1} - c_{t+1})
#   A   += X - S - L,   D += L - Tn
#   b_t += z_t - s_t,   c_{t+1} += w_{t+1} - s_{t+1}
#
# with wz_t = 1 for t < T and ww_t = 1 for t > 1 (zero otherwise).
#
# Readings:
#   - S >= 0 makes the s-step the one-sided shrink max(k/sig - lam/(rho sig), 0).
#   - x-step: the augmented Lagrangian's block rho/2 ||X - S - L + A||^2 gives
#     Phi^T y + rho (s + l - a); the printed update omits rho on the second term.
#   - A-step: the same block gives A += X - S - L; the printed update has + L.
#   - The prox of each frame pair is the full prox (eq. Prox_UOT) with both
#     arguments free and prox step kappa / rho, warm-started per pair.
#   - Residuals (the paper cites Boyd et al. Sec. 3.3 and, for Algorithm 2,
#     stacks the constraint violations and the changes of the split
#     variables): primal ||[X - S - L; L - Tn; z - s; w - s]||, dual
#     rho ||[dX; dTn; dz; dw]||.
# ---------------------------------------------------------------------------


@dataclass
class RpcaState:
    S: np.ndarray
    L: np.ndarray
    X: np.ndarray
    Tn: np.ndarray
    A: np.ndarray
    D: np.ndarray
    b: np.ndarray   # frames 1..T-1 (index t-1 ... stored for pairs 0..T-2)
    c: np.ndarray   # multipliers of w: pair t holds c_{t+1}
    prox: list      # per frame pair: uot.State (x0 = z_t, x1 = w_{t+1})

    @property
    def Z(self):
        return np.stack([p.x0 for p in self.prox]) if self.prox else np.zeros((0,) + self.S.shape[1:])

    @property
    def W(self):
        return np.stack([p.x1 for p in self.prox]) if self.prox else np.zeros((0,) + self.S.shape[1:])


def svt(M, thr):
    """Singular-value soft threshold of the N x T matrix whose columns are
    the frames of M (frames on the first axis)."""
    T = M.shape[0]
    flat = M.reshape(T, -1).T
    U, sv, Vt = np.linalg.svd(flat, full_matrices=False)
    out = (U * np.maximum(sv - thr, 0.0)) @ Vt
    return out.T.reshape(M.shape)


def rpca_problem(p0, p1, kappa, mu, rho, balanced=False, residual_p=1, bc=0):
    """The (z_t, w_{t+1}) subproblem as an Algorithm-1 problem: PROX with
    centres p0 = s_t - b_t, p1 = s_{t+1} - c_{t+1}, prox step kappa / rho."""
    from .ops import PROX
    return uot.Problem(np.asarray(p0, float), np.asarray(p1, float), mode=PROX, balanced=balanced,
                       residual_p=residual_p, bc=bc, mu=mu, rho=kappa / rho)


def rpca_initial_state(shape, kappa, mu, rho, balanced=False, residual_p=1, bc=0) -> RpcaState:
    T = shape[0]
    z = np.zeros(shape)
    zf = np.zeros(shape[1:])
    prox = [uot.initial_state(rpca_problem(zf, zf, kappa, mu, rho, balanced, residual_p, bc)) for _ in range(T - 1)]
    return RpcaState(z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), np.zeros((T - 1,) + shape[1:]),
                     np.zeros((T - 1,) + shape[1:]), prox)


def rpca_iterate(Y, st: RpcaState, kappa, mu, rho, lam, gam, phi=None, balanced=False, residual_p=1, bc=0,
                 prox_iters=1, tau=None) -> RpcaState:
    """One ADMM iteration of Algorithm 3 (see the comment above)."""
    Y = np.asarray(Y, float)
    T = Y.shape[0]
    ph = np.ones_like(Y) if phi is None else np.asarray(phi, float)
    Z, W = st.Z, st.W
    k = st.X - st.L + st.A
    sig = np.ones((T,) + Y.shape[1:])
    if T > 1:
        k[:-1] += Z + st.b
        k[1:] += W + st.c
        sig[:-1] += 1.0
        sig[1:] += 1.0
    S = np.maximum(k / sig - lam / (rho * sig), 0.0)
    L = np.maximum(0.5 * (st.Tn - st.D + st.X - S + st.A), 0.0)
    X = (ph * Y + rho * (S + L - st.A)) / (ph * ph + rho)
    Tn = svt(L + st.D, gam / rho)
    prox = []
    for t in range(T - 1):
        prob = rpca_problem(S[t] - st.b[t], S[t + 1] - st.c[t], kappa, mu, rho, balanced, residual_p, bc)
        t1, t2 = prob.unit_steps() if tau is None else tau
        pst = st.prox[t]
        for _ in range(prox_iters):
            pst = uot.iterate(prob, pst, t1, t2)
        prox.append(pst)
    nz = np.stack([p.x0 for p in prox]) if prox else Z
    nw = np.stack([p.x1 for p in prox]) if prox else W
    A = st.A + X - S - L
    D = st.D + L - Tn
    b = st.b + (nz - S[:-1])
    c = st.c + (nw - S[1:])
    return RpcaState(S, L, X, Tn, A, D, b, c, prox)


def rpca_residuals(prev: RpcaState, cur: RpcaState, rho):
    S = cur.S
    rp2 = np.sum((cur.X - S - cur.L) ** 2) + np.sum((cur.L - cur.Tn) ** 2)
    rd2 = np.sum((cur.X - prev.X) ** 2) + np.sum((cur.Tn - prev.Tn) ** 2)
    if cur.prox:
        rp2 += np.sum((cur.Z - S[:-1]) ** 2) + np.sum((cur.W - S[1:]) ** 2)
        rd2 += np.sum((cur.Z - prev.Z) ** 2) + np.sum((cur.W - prev.W) ** 2)
    return float(np.sqrt(rp2)), float(rho * np.sqrt(rd2))


def rpca_uotdf(Y, kappa, mu, rho, lam, gam, phi=None, balanced=False, residual_p=1, bc=0, prox_iters=1,
               max_iter=5000, eps=1e-4, check_every=1, tau=None, record=False):
    """Algorithm 3 until both residuals are below eps (tested every
    check_every iterations) or max_iter; returns (state, report)."""
    Y = np.asarray(Y, float)
    st = rpca_initial_state(Y.shape, kappa, mu, rho, balanced, residual_p, bc)
    rep = DfReport()
    for k in range(1, max_iter + 1):
        nxt = rpca_iterate(Y, st, kappa, mu, rho, lam, gam, phi, balanced, residual_p, bc, prox_iters, tau)
        if k % check_every == 0 or k == max_iter:
            rp, rd = rpca_residuals(st, nxt, rho)
            rep.r_primal, rep.r_dual = rp, rd
            if record:
                rep.history.append((k, rp, rd))
            if rp < eps and rd < eps:
                rep.iters, rep.converged = k, True
                return nxt, rep
        st = nxt
    rep.iters = max_iter
    return st, rep


def rpca_objective(Y, S, L, kappa, mu, lam, gam, phi=None, balanced=False):
    """The objective of eq. RPCA_UOTDF with V from the linear program (exact
    on grids one pixel high or wide)."""
    from .lp import beckmann_aniso
    Y = np.asarray(Y, float)
    ph = np.ones_like(Y) if phi is None else np.asarray(phi, float)
    T = Y.shape[0]
    f = 0.5 * float(np.sum((Y - ph * (S + L)) ** 2)) + lam * float(np.sum(np.abs(S)))
    f += gam * float(np.sum(np.linalg.svd(L.reshape(T, -1).T, compute_uv=False)))
    for t in range(T - 1):
        f += kappa * beckmann_aniso(S[t], S[t + 1], mu=None if balanced else mu, balanced=balanced)
    return f


# ---------------------------------------------------------------------------
# RPCA+UOT-DF with a signed sparse part (Sec. IV-B, eq. RPCA_UOTDF_PN):
#
#   min_{S+, S-, L >= 0} 1/2 sum_t ||y_t - Phi_t (s+_t - s-_t + l_t)||^2
#       + lam (||S+||_1 + ||S-||_1) + gam ||L||_*
#       + kappa sum_{t<T} (V_mu(s+_t, s+_{t+1}) + V_mu(s-_t, s-_{t+1}))
#
# The paper states the objective and no algorithm.  This is Algorithm 3's
# splitting with the sparse block in two signs: X = S+ - S- + L, Tn = L,
# z+-_t = s+-_t, w+-_{t+1} = s+-_{t+1} (multipliers A, D, b+-, c+-), the
# blocks minimised in the order S+, S-, L, X, Tn, the prox of every frame
# pair of both signs, then the multipliers:
#
#   k+ = (x - l + s- + a) + wz (z+ + b+) + ww (w+ + c+),  s+ = max(k+/sig - lam/(rho sig), 0)
#   k- = (l - x + s+ - a) + wz (z- + b-) + ww (w- + c-),  s- = max(k-/sig - lam/(rho sig), 0)
#   L  = max((Tn - D + X - S+ + S- + A) / 2, 0)
#   x  = (Phi^T y + rho (s+ - s- + l - a)) / (Phi^T Phi + rho)
#   Tn = SVT_{gam/rho}(L + D)
#   (z+-_t, w+-_{t+1}) = prox_{(kappa/rho) V_mu}(s+-_t - b+-_t, s+-_{t+1} - c+-_{t+1})
#   A += X - S+ + S- - L,  D += L - Tn,  b+- += z+- - s+-,  c+- += w+- - s+-
#
# Residuals: primal ||[X - S+ + S- - L; L - Tn; z+- - s+-; w+- - s+-]||,
# dual rho ||[dX; dTn; dz+-; dw+-]||.
# ---------------------------------------------------------------------------


@dataclass
class RpcaPnState:
    Sp: np.ndarray
    Sm: np.ndarray
    L: np.ndarray
    X: np.ndarray
    Tn: np.ndarray
    A: np.ndarray
    D: np.ndarray
    bp: np.ndarray
    cp: np.ndarray
    bm: np.ndarray
    cm: np.ndarray
    prox_p: list
    prox_m: list

    @staticmethod
    def _stack(prox, which, like):
        return np.stack([getattr(p, which) for p in prox]) if prox else np.zeros((0,) + like.shape[1:])

    @property
    def S(self):
        return self.Sp - self.Sm

    @property
    def Zp(self):
        return self._stack(self.prox_p, "x0", self.Sp)

    @property
    def Wp(self):
        return self._stack(self.prox_p, "x1", self.Sp)

    @property
    def Zm(self):
        return self._stack(self.prox_m, "x0", self.Sm)

    @property
    def Wm(self):
        return self._stack(self.prox_m, "x1", self.Sm)


def rpca_pn_initial_state(shape, kappa, mu, rho, balanced=False, residual_p=1, bc=0) -> RpcaPnState:
    T = shape[0]
    z = np.zeros(shape)
    zp = np.zeros((T - 1,) + shape[1:])
    zf = np.zeros(shape[1:])

    def fresh():
        return [uot.initial_state(rpca_problem(zf, zf, kappa, mu, rho, balanced, residual_p, bc))
                for _ in range(T - 1)]
    return RpcaPnState(z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), zp.copy(), zp.copy(),
                       zp.copy(), zp.copy(), fresh(), fresh())


def _pair_prox(S, b, c, prox, kappa, mu, rho, balanced, residual_p, bc, prox_iters, tau):
    out = []
    for t in range(S.shape[0] - 1):
        prob = rpca_problem(S[t] - b[t], S[t + 1] - c[t], kappa, mu, rho, balanced, residual_p, bc)
        t1, t2 = prob.unit_steps() if tau is None else tau
        pst = prox[t]
        for _ in range(prox_iters):
            pst = uot.iterate(prob, pst, t1, t2)
        out.append(pst)
    return out


def rpca_pn_iterate(Y, st: RpcaPnState, kappa, mu, rho, lam, gam, phi=None, balanced=False, residual_p=1, bc=0,
                    prox_iters=1, tau=None) -> RpcaPnState:
    """One ADMM iteration of the signed RPCA+UOT-DF (see the comment above)."""
    Y = np.asarray(Y, float)
    T = Y.shape[0]
    ph = np.ones_like(Y) if phi is None else np.asarray(phi, float)
    sig = np.ones(Y.shape)
    kp = st.X - st.L + st.Sm + st.A
    if T > 1:
        kp[:-1] += st.Zp + st.bp
        kp[1:] += st.Wp + st.cp
        sig[:-1] += 1.0
        sig[1:] += 1.0
    Sp = np.maximum(kp / sig - lam / (rho * sig), 0.0)
    km = st.L - st.X + Sp - st.A
    if T > 1:
        km[:-1] += st.Zm + st.bm
        km[1:] += st.Wm + st.cm
    Sm = np.maximum(km / sig - lam / (rho * sig), 0.0)
    L = np.maximum(0.5 * (st.Tn - st.D + st.X - Sp + Sm + st.A), 0.0)
    X = (ph * Y + rho * (Sp - Sm + L - st.A)) / (ph * ph + rho)
    Tn = svt(L + st.D, gam / rho)
    prox_p = _pair_prox(Sp, st.bp, st.cp, st.prox_p, kappa, mu, rho, balanced, residual_p, bc, prox_iters, tau)
    prox_m = _pair_prox(Sm, st.bm, st.cm, st.prox_m, kappa, mu, rho, balanced, residual_p, bc, prox_iters, tau)
    nxt = RpcaPnState(Sp, Sm, L, X, Tn, st.A + X - Sp + Sm - L, st.D + L - Tn, st.bp, st.cp, st.bm, st.cm,
                      prox_p, prox_m)
    if T > 1:
        nxt.bp = st.bp + (nxt.Zp - Sp[:-1])
        nxt.cp = st.cp + (nxt.Wp - Sp[1:])
        nxt.bm = st.bm + (nxt.Zm - Sm[:-1])
        nxt.cm = st.cm + (nxt.Wm - Sm[1:])
    return nxt


def rpca_pn_residuals(prev: RpcaPnState, cur: RpcaPnState, rho):
    rp2 = np.sum((cur.X - cur.Sp + cur.Sm - cur.L) ** 2) + np.sum((cur.L - cur.Tn) ** 2)
    rd2 = np.sum((cur.X - prev.X) ** 2) + np.sum((cur.Tn - prev.Tn) ** 2)
    if cur.prox_p:
        for S, Z, W, Zo, Wo in ((cur.Sp, cur.Zp, cur.Wp, prev.Zp, prev.Wp), (cur.Sm, cur.Zm, cur.Wm, prev.Zm, prev.Wm)):
            rp2 += np.sum((Z - S[:-1]) ** 2) + np.sum((W - S[1:]) ** 2)
            rd2 += np.sum((Z - Zo) ** 2) + np.sum((W - Wo) ** 2)
    return float(np.sqrt(rp2)), float(rho * np.sqrt(rd2))


def rpca_pn_uotdf(Y, kappa, mu, rho, lam, gam, phi=None, balanced=False, residual_p=1, bc=0, prox_iters=1,
                  max_iter=5000, eps=1e-4, check_every=1, tau=None, record=False):
    """The signed RPCA+UOT-DF until both residuals are below eps (tested
    every check_every iterations) or max_iter; returns (state, report)."""
    Y = np.asarray(Y, float)
    st = rpca_pn_initial_state(Y.shape, kappa, mu, rho, balanced, residual_p, bc)
    rep = DfReport()
    for k in range(1, max_iter + 1):
        nxt = rpca_pn_iterate(Y, st, kappa, mu, rho, lam, gam, phi, balanced, residual_p, bc, prox_iters, tau)
        if k % check_every == 0 or k == max_iter:
            rp, rd = rpca_pn_residuals(st, nxt, rho)
            rep.r_primal, rep.r_dual = rp, rd
            if record:
                rep.history.append((k, rp, rd))
            if rp < eps and rd < eps:
                rep.iters, rep.converged = k, True
                return nxt, rep
        st = nxt
    rep.iters = max_iter
    return st, rep


def rpca_pn_objective(Y, Sp, Sm, L, kappa, mu, lam, gam, phi=None, balanced=False):
    """The objective of eq. RPCA_UOTDF_PN with V from the linear program
    (exact on grids one pixel high or wide)."""
    from .lp import beckmann_aniso
    Y = np.asarray(Y, float)
    ph = np.ones_like(Y) if phi is None else np.asarray(phi, float)
    T = Y.shape[0]
    f = 0.5 * float(np.sum((Y - ph * (Sp - Sm + L)) ** 2)) + lam * float(np.sum(Sp) + np.sum(Sm))
    f += gam * float(np.sum(np.linalg.svd(L.reshape(T, -1).T, compute_uv=False)))
    for t in range(T - 1):
        for P in (Sp, Sm):
            f += kappa * beckmann_aniso(P[t], P[t + 1], mu=None if balanced else mu, balanced=balanced)
    return f
