"""Pins of the ADMM oracle of the signed RPCA+UOT-DF (eq. RPCA_UOTDF_PN,
S = S+ - S-) against what the mathematics fixes: with no low-rank part and
no transport weight the minimiser is the two-sided soft threshold; a
constrained quadratic program (SLSQP) minimises the objective of two frames
of one pixel; the problem is symmetric under Y -> -Y when L is switched off
and under reversing time; a planted sign error in the S- step misses the
minimum."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import admm

KW = dict(prox_iters=5, eps=1e-8, max_iter=40000, check_every=10)


def test_no_low_rank_no_transport_is_the_soft_threshold():
    """gam -> infinity forces L = 0; kappa -> 0 drops the transport terms;
    what is left is min 1/2 ||Y - S||^2 + lam ||S||_1 over S = S+ - S-, whose
    minimiser is sign(Y) max(|Y| - lam, 0), split with S+ S- = 0."""
    rng = np.random.default_rng(0)
    Y = rng.normal(0.1, 0.5, (3, 4, 5))
    st, rep = admm.rpca_pn_uotdf(Y, 1e-9, 1.0, 1.0, 0.15, 1e6, **KW)
    assert rep.converged
    np.testing.assert_allclose(st.L, 0.0, atol=1e-7)
    np.testing.assert_allclose(st.S, np.sign(Y) * np.maximum(np.abs(Y) - 0.15, 0.0), atol=1e-6)
    np.testing.assert_allclose(st.Sp, np.maximum(Y - 0.15, 0.0), atol=1e-6)
    np.testing.assert_allclose(st.Sm, np.maximum(-Y - 0.15, 0.0), atol=1e-6)


def qp_two_single_pixel_frames(y, kappa, mu, lam, gam):
    """min over s+ (2), s- (2), l (2) >= 0 of
    1/2 sum (y - s+ + s- - l)^2 + lam sum (s+ + s-) + gam ||l||_2
      + kappa mu (|s+_1 - s+_2| + |s-_1 - s-_2|)
    (one pixel: V_mu(a, b) = mu |a - b|, no flux), as smooth programs:
    |d| = u + v with u, v >= 0 and d = u - v; ||l||_2 <= tau, or l = 0 (the
    cone's apex, where SLSQP's constraint gradient vanishes, solved as a
    plain quadratic program)."""
    def f(v):
        sp, sm, l = v[0:2], v[2:4], v[4:6]
        up, vp, um, vm, tau = v[6:11]
        return (0.5 * float(np.sum((y - sp + sm - l) ** 2)) + lam * float(sp.sum() + sm.sum()) + gam * tau
                + kappa * mu * (up + vp + um + vm))
    lin = [dict(type="eq", fun=lambda v: v[0] - v[1] - v[6] + v[7]),
           dict(type="eq", fun=lambda v: v[2] - v[3] - v[8] + v[9])]
    cone = lin + [dict(type="ineq", fun=lambda v: v[10] ** 2 - v[4] ** 2 - v[5] ** 2)]
    apex = lin + [dict(type="eq", fun=lambda v: v[4]), dict(type="eq", fun=lambda v: v[5]),
                  dict(type="eq", fun=lambda v: v[10])]
    best = np.inf
    rng = np.random.default_rng(1)
    for cons in (cone, apex):
        for _ in range(4):
            x0 = rng.uniform(0, 1.5, 11)
            r = minimize(f, x0, method="SLSQP", bounds=[(0, None)] * 11, constraints=cons,
                         options=dict(ftol=1e-14, maxiter=300))
            ok = all(c["fun"](r.x) > -1e-9 if c["type"] == "ineq" else abs(c["fun"](r.x)) < 1e-9 for c in cons)
            if ok and np.all(r.x >= -1e-12):
                best = min(best, r.fun)
    assert np.isfinite(best)
    return best


@pytest.mark.parametrize("y,rho", [((0.9, -0.6), 1.0), ((-0.4, 1.2), 2.0), ((1.1, 0.8), 0.7)])
def test_two_single_pixel_frames_against_a_quadratic_program(y, rho):
    y = np.array(y)
    kappa, mu, lam, gam = 0.3, 0.9, 0.1, 0.3
    st, rep = admm.rpca_pn_uotdf(y.reshape(2, 1, 1), kappa, mu, rho, lam, gam, **KW)
    assert rep.converged
    sp, sm, l = st.Sp.reshape(2), st.Sm.reshape(2), st.L.reshape(2)
    got = (0.5 * float(np.sum((y - sp + sm - l) ** 2)) + lam * float(sp.sum() + sm.sum())
           + gam * float(np.hypot(*l)) + kappa * mu * (abs(sp[0] - sp[1]) + abs(sm[0] - sm[1])))
    best = qp_two_single_pixel_frames(y, kappa, mu, lam, gam)
    assert got <= best + 1e-7 and got >= best - 1e-6


def test_objective_on_a_strip_is_the_lp_value():
    """On frames one pixel high the flux norms coincide and V is the linear
    program; the converged ADMM point is no worse than small random feasible
    perturbations of it."""
    rng = np.random.default_rng(3)
    Y = rng.normal(0.2, 0.6, (3, 1, 4))
    kw = dict(kappa=0.4, mu=0.7, rho=1.0, lam=0.05, gam=0.5)
    st, rep = admm.rpca_pn_uotdf(Y, **kw, **KW)
    assert rep.converged
    obj = lambda Sp, Sm, L: admm.rpca_pn_objective(Y, Sp, Sm, L, kw["kappa"], kw["mu"], kw["lam"], kw["gam"])
    base = obj(st.Sp, st.Sm, st.L)
    for _ in range(20):
        d = [1e-3 * rng.normal(0, 1, Y.shape) for _ in range(3)]
        cand = [np.maximum(a + e, 0.0) for a, e in zip((st.Sp, st.Sm, st.L), d)]
        assert obj(*cand) >= base - 1e-7


def test_sign_flip_swaps_the_parts():
    """With L switched off the objective is invariant under Y -> -Y,
    S+ <-> S-."""
    rng = np.random.default_rng(4)
    Y = rng.normal(0.0, 0.6, (3, 3, 4))
    kw = dict(kappa=0.3, mu=0.8, rho=1.0, lam=0.05, gam=1e6, prox_iters=3, max_iter=20000, eps=1e-8,
              check_every=10)
    a, ra = admm.rpca_pn_uotdf(Y, **kw)
    b, rb = admm.rpca_pn_uotdf(-Y, **kw)
    assert ra.converged and rb.converged
    np.testing.assert_allclose(b.Sp, a.Sm, atol=1e-5)
    np.testing.assert_allclose(b.Sm, a.Sp, atol=1e-5)


def test_time_reversal_symmetry():
    rng = np.random.default_rng(6)
    Y = rng.normal(0.3, 0.5, (4, 3, 5))
    kw = dict(kappa=0.3, mu=0.8, rho=1.0, lam=0.1, gam=0.4, prox_iters=3, max_iter=20000, eps=1e-8,
              check_every=10)
    a, ra = admm.rpca_pn_uotdf(Y, **kw)
    b, rb = admm.rpca_pn_uotdf(Y[::-1].copy(), **kw)
    assert ra.converged and rb.converged
    np.testing.assert_allclose(b.S[::-1], a.S, atol=1e-5)
    np.testing.assert_allclose(b.L[::-1], a.L, atol=1e-5)


def test_planted_sign_error_misses_the_minimum(monkeypatch):
    """The S- step sees the X block with the opposite sign of the S+ step;
    planting the S+ sign there (k- built from x - l instead of l - x) moves
    the fixed point away from the quadratic program's minimum."""
    import oracle.admm as M
    y = np.array([0.9, -0.6])
    kappa, mu, lam, gam, rho = 0.3, 0.9, 0.1, 0.3, 1.0
    orig = M.rpca_pn_iterate

    def planted(Y, st, *a, **k):
        nxt = orig(Y, st, *a, **k)
        T = Y.shape[0]
        sig = np.ones(Y.shape)
        km = st.X - st.L + nxt.Sp - st.A
        km[:-1] += st.Zm + st.bm
        km[1:] += st.Wm + st.cm
        sig[:-1] += 1.0
        sig[1:] += 1.0
        nxt.Sm = np.maximum(km / sig - lam / (rho * sig), 0.0)
        return nxt
    monkeypatch.setattr(M, "rpca_pn_iterate", planted)
    st, rep = M.rpca_pn_uotdf(y.reshape(2, 1, 1), kappa, mu, rho, lam, gam, prox_iters=5, eps=1e-8,
                              max_iter=4000, check_every=10)
    sp, sm, l = st.Sp.reshape(2), st.Sm.reshape(2), st.L.reshape(2)
    got = (0.5 * float(np.sum((y - sp + sm - l) ** 2)) + lam * float(sp.sum() + sm.sum())
           + gam * float(np.hypot(*l)) + kappa * mu * (abs(sp[0] - sp[1]) + abs(sm[0] - sm[1])))
    best = qp_two_single_pixel_frames(y, kappa, mu, lam, gam)
    assert (not rep.converged) or got > best + 1e-3
