"""Pins of the ADMM oracle of Algorithm 3 (RPCA+UOT-DF) against what the
mathematics fixes: the two ends of the parameter range (no low-rank part:
the l1 projection; no sparse part: the singular-value threshold itself),
brute-force minimisation of the objective on two frames of one and two
pixels, and the symmetry of the problem under reversing time."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import admm

KW = dict(prox_iters=5, eps=1e-8, max_iter=40000, check_every=10)


def test_huge_low_rank_weight_leaves_the_l1_projection():
    """gam -> infinity forces L = 0; with a vanishing transport weight the
    problem is min_{S>=0} 1/2 ||Y - S||^2 + lam ||S||_1: S = max(Y - lam, 0)."""
    rng = np.random.default_rng(0)
    Y = rng.normal(0.3, 0.4, (3, 4, 5))
    st, rep = admm.rpca_uotdf(Y, 1e-9, 1.0, 1.0, 0.15, 1e6, **KW)
    assert rep.converged
    np.testing.assert_allclose(st.L, 0.0, atol=1e-7)
    np.testing.assert_allclose(st.S, np.maximum(Y - 0.15, 0.0), atol=1e-6)


def test_huge_sparse_weight_leaves_the_singular_value_threshold():
    """lam -> infinity forces S = 0; for a positive rank-one Y the threshold
    SVT_gam(Y) = (1 - gam / sigma) Y is itself nonnegative, so L = SVT_gam(Y)."""
    rng = np.random.default_rng(1)
    u = rng.uniform(0.2, 1.0, 4 * 5)
    v = rng.uniform(0.5, 1.5, 3)
    Y = (u[:, None] * v[None, :]).T.reshape(3, 4, 5)
    gam = 0.4
    st, rep = admm.rpca_uotdf(Y, 1e-9, 1.0, 1.0, 1e6, gam, **KW)
    assert rep.converged
    sigma = np.linalg.norm(u) * np.linalg.norm(v)
    np.testing.assert_allclose(st.S, 0.0, atol=1e-7)
    np.testing.assert_allclose(st.L, (1.0 - gam / sigma) * Y, atol=1e-6)


def brute(f, starts, n):
    return min(minimize(f, x0 + 1e-3, method="Nelder-Mead",
                        options=dict(xatol=1e-10, fatol=1e-13, maxiter=20000, maxfev=40000)).fun
               for x0 in starts)


@pytest.mark.parametrize("seed,rho", [(0, 1.0), (1, 2.5), (2, 0.6)])
def test_two_single_pixel_frames_brute_force(seed, rho):
    """T = 2 frames of one pixel: ||L||_* = sqrt(l1^2 + l2^2) (one singular
    value) and V(s1, s2) = mu |s1 - s2| (no flux on one pixel), so the
    objective is explicit in (s1, s2, l1, l2) >= 0; ADMM reaches its minimum
    for every penalty rho (the x-step's rho matters once rho != 1)."""
    rng = np.random.default_rng(seed)
    Y = rng.uniform(0.2, 1.5, (2, 1, 1))
    kappa, mu, lam, gam = 0.3, 0.9, 0.1, 0.3
    st, rep = admm.rpca_uotdf(Y, kappa, mu, rho, lam, gam, **KW)
    assert rep.converged
    y = Y.reshape(2)

    def f(v):
        s, l = v[:2], v[2:]
        if np.any(v < 0):
            return 1e6 + float(np.sum(np.minimum(v, 0) ** 2))
        return (0.5 * float(np.sum((y - s - l) ** 2)) + lam * float(s.sum()) + gam * float(np.hypot(*l))
                + kappa * mu * abs(s[0] - s[1]))
    got = f(np.concatenate([st.S.reshape(2), st.L.reshape(2)]))
    best = brute(f, [np.concatenate([st.S.reshape(2), st.L.reshape(2)]), np.array([y[0], y[1], 0, 0]),
                     np.array([0, 0, y[0], y[1]])], 4)
    # ADMM's point is feasible, so it cannot beat the true minimum; the
    # lower slack is the accuracy of the simplex search at the kinks
    assert got <= best + 1e-7 and got >= best - 1e-5


@pytest.mark.parametrize("seed,balanced", [(3, False), (4, False), (5, True)])
def test_two_strip_frames_brute_force(seed, balanced):
    """T = 2 frames of a 1 x 2 strip with the low-rank part switched off
    (gam huge): min over S >= 0 of 1/2 ||Y - S||^2 + lam ||S||_1 +
    kappa V(s1, s2), with V from the linear program; balanced transport
    keeps the two frames' masses equal, so there the search runs over
    mass-equal pairs."""
    rng = np.random.default_rng(seed)
    Y = rng.uniform(0.1, 1.2, (2, 1, 2))
    kappa, mu, rho, lam, gam = 0.4, 0.7, 1.0, 0.05, 1e6
    st, rep = admm.rpca_uotdf(Y, kappa, mu, rho, lam, gam, balanced=balanced, **KW)
    assert rep.converged
    got = admm.rpca_objective(Y, st.S, st.L, kappa, mu, lam, 0.0, balanced=balanced)
    if balanced:
        def f(v):
            s1 = v[:2]
            s2 = np.array([v[2], s1.sum() - v[2]])
            S = np.stack([s1, s2]).reshape(2, 1, 2)
            if np.any(S < 0):
                return 1e6 + float(np.sum(np.minimum(S, 0) ** 2))
            return admm.rpca_objective(Y, S, np.zeros_like(S), kappa, mu, lam, 0.0, balanced=True)
        starts = [st.S.reshape(4)[:3], Y.reshape(4)[:3]]
    else:
        def f(v):
            S = v.reshape(2, 1, 2)
            if np.any(S < 0):
                return 1e6 + float(np.sum(np.minimum(S, 0) ** 2))
            return admm.rpca_objective(Y, S, np.zeros_like(S), kappa, mu, lam, 0.0)
        starts = [st.S.reshape(4), np.maximum(Y - lam, 0).reshape(4)]
    best = brute(f, starts, 4)
    assert got <= best + 1e-6 and got >= best - 1e-5


def test_time_reversal_symmetry():
    """V is symmetric and the other terms do not see the order of the frames,
    so reversing time reverses the solution."""
    rng = np.random.default_rng(6)
    Y = rng.uniform(0, 1, (4, 3, 5))
    kw = dict(kappa=0.3, mu=0.8, rho=1.0, lam=0.1, gam=0.4, prox_iters=3, max_iter=20000, eps=1e-8,
              check_every=10)
    a, ra = admm.rpca_uotdf(Y, **kw)
    b, rb = admm.rpca_uotdf(Y[::-1].copy(), **kw)
    assert ra.converged and rb.converged
    np.testing.assert_allclose(b.S[::-1], a.S, atol=1e-5)
    np.testing.assert_allclose(b.L[::-1], a.L, atol=1e-5)


def test_svt_is_the_prox_of_the_nuclear_norm():
    """SVT_t(M) minimises t ||X||_* + 1/2 ||X - M||^2: no random perturbation
    of it does better."""
    rng = np.random.default_rng(7)
    M = rng.normal(0, 1, (5, 3, 4))
    thr = 0.8
    X = admm.svt(M, thr)

    def obj(X):
        return thr * np.sum(np.linalg.svd(X.reshape(5, -1).T, compute_uv=False)) + 0.5 * np.sum((X - M) ** 2)
    base = obj(X)
    for _ in range(50):
        assert obj(X + 1e-3 * rng.normal(0, 1, X.shape)) >= base - 1e-12


@pytest.mark.parametrize("variant", ["x_without_rho", "a_plus_l"])
def test_printed_variants_miss_the_minimum(variant, monkeypatch):
    """The readings of the x-step (rho on s + l - a) and of the A-step
    (A += X - S - L): the printed forms, planted here in a copy of the
    oracle's iteration, converge elsewhere (x-step) or diverge (A-step) on
    the two-pixel problem whose minimum the brute-force pin finds."""
    import oracle.admm as M
    rng = np.random.default_rng(1)
    Y = rng.uniform(0.2, 1.5, (2, 1, 1))
    orig = M.rpca_iterate

    def planted(Y, st, kappa, mu, rho, lam, gam, *a, **k):
        nxt = orig(Y, st, kappa, mu, rho, lam, gam, *a, **k)
        if variant == "x_without_rho":
            nxt.X = (np.asarray(Y) + (nxt.S + nxt.L - st.A)) / (1 + rho)
            nxt.A = st.A + nxt.X - nxt.S - nxt.L
        else:
            nxt.A = st.A + nxt.X - nxt.S + nxt.L
        return nxt
    good, _ = M.rpca_uotdf(Y, 0.3, 0.9, 2.5, 0.1, 0.3, prox_iters=5, eps=1e-8, max_iter=4000, check_every=10)
    monkeypatch.setattr(M, "rpca_iterate", planted)
    bad, rep = M.rpca_uotdf(Y, 0.3, 0.9, 2.5, 0.1, 0.3, prox_iters=5, eps=1e-8, max_iter=4000, check_every=10)
    assert (not rep.converged) or np.abs(bad.S - good.S).max() > 0.1
