"""Pins of the ADMM oracle of Algorithm 2 (UOT-DF / BPDN+UOT-DF) against
what the mathematics fixes: closed forms on a single pixel, the trivial
solutions at the ends of the parameter range, and brute-force minimisation
of the objective (with V from the linear program) on grids of two and three
pixels."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import admm

KW = dict(prox_iters=10, eps=1e-9, max_iter=20000, check_every=10)


def shrink(v, t):
    return np.sign(v) * max(abs(v) - t, 0.0)


@pytest.mark.parametrize("y,s0,phi,lam", [(1.3, 0.4, 1.0, 0.0), (0.2, 1.1, 1.0, 0.0), (1.3, 0.4, 0.6, 0.15),
                                          (-0.5, 0.3, 1.0, 0.0), (0.9, 0.0, 1.5, 0.05), (0.7, 0.5, 0.0, 0.0)])
def test_single_pixel_closed_form(y, s0, phi, lam):
    """One pixel carries no flux, so V(s, s0) = mu |s - s0| and the problem is
    min_{s>=0} 1/2 (y - phi s)^2 + lam s + kappa mu |s - s0|: the prox of the
    absolute value around s0 at the unconstrained least-squares point, then
    clamped at zero (exact for a convex function of one variable)."""
    kappa, mu, rho = 0.5, 0.8, 1.0
    if phi == 0.0:
        ref = s0  # no data: only the transport term, whose minimum is at s0
    else:
        c = (phi * y - lam) / phi ** 2
        ref = max(s0 + shrink(c - s0, kappa * mu / phi ** 2), 0.0)
    s, _, rep = admm.uotdf(np.array([[y]]), np.array([[s0]]), kappa, mu, rho, phi=np.array([[phi]]), lam=lam, **KW)
    assert rep.converged
    assert abs(s[0, 0] - ref) < 1e-6


def test_single_pixel_balanced_keeps_the_prediction():
    """Balanced transport on one pixel allows no change of mass: s = s0."""
    s, _, rep = admm.uotdf(np.array([[1.7]]), np.array([[0.6]]), 0.5, 1.0, 1.0, balanced=True, **KW)
    assert rep.converged and abs(s[0, 0] - 0.6) < 1e-6


def test_prediction_equal_to_observation_is_optimal():
    """y = s0 >= 0 and Phi = I: s = y makes both terms zero."""
    rng = np.random.default_rng(0)
    y = rng.uniform(0, 1, (5, 6)) * (rng.uniform(0, 1, (5, 6)) < 0.5)
    s, _, rep = admm.uotdf(y, y.copy(), 0.7, 0.9, 1.0, **KW)
    assert rep.converged
    np.testing.assert_allclose(s, y, atol=1e-6)


@pytest.mark.parametrize("lam", [0.0, 0.2])
def test_vanishing_transport_weight_gives_the_projection(lam):
    """kappa -> 0 leaves min_{s>=0} 1/2 ||y - s||^2 + lam ||s||_1, solved by
    max(y - lam, 0) entry by entry."""
    rng = np.random.default_rng(1)
    y = rng.normal(0.2, 0.5, (4, 5))
    s0 = rng.uniform(0, 1, (4, 5))
    s, _, rep = admm.uotdf(y, s0, 1e-9, 1.0, 1.0, lam=lam, **KW)
    assert rep.converged
    np.testing.assert_allclose(s, np.maximum(y - lam, 0.0), atol=1e-6)


@pytest.mark.parametrize("shape,seed,lam,balanced", [((1, 2), 0, 0.0, False), ((1, 3), 1, 0.0, False),
                                                     ((2, 1), 2, 0.1, False), ((1, 3), 3, 0.0, True)])
def test_brute_force_objective(shape, seed, lam, balanced):
    """On a strip of two or three pixels (where the Euclidean and the
    Manhattan flux norms coincide) the objective, with V computed by the
    linear program, is minimised directly over s; ADMM must reach the same
    optimal value.  Balanced transport fixes the total mass, so there the
    search runs over mass-preserving s."""
    rng = np.random.default_rng(seed)
    s0 = rng.uniform(0.2, 1.0, shape)
    y = np.clip(np.roll(s0, 1) * rng.uniform(0.6, 1.4) + rng.normal(0, 0.05, shape), 0, None)
    kappa, mu, rho = 0.4, 0.7, 1.0
    s, _, rep = admm.uotdf(y, s0, kappa, mu, rho, lam=lam, balanced=balanced, **KW)
    assert rep.converged
    got = admm.uotdf_objective(y, s, s0, kappa, mu, lam=lam, balanced=balanced)
    n = s0.size
    if balanced:
        m = s0.sum()

        def f(v):
            w = np.append(v, m - v.sum()).reshape(shape)
            if np.any(w < 0):
                return 1e6 + float(np.sum(np.minimum(w, 0) ** 2))
            return admm.uotdf_objective(y, w, s0, kappa, mu, lam=lam, balanced=True)
        starts = [s.reshape(-1)[:-1], s0.reshape(-1)[:-1]]
    else:
        def f(v):
            w = v.reshape(shape)
            if np.any(w < 0):
                return 1e6 + float(np.sum(np.minimum(w, 0) ** 2))
            return admm.uotdf_objective(y, w, s0, kappa, mu, lam=lam)
        starts = [s.reshape(-1), s0.reshape(-1), np.maximum(y, 0).reshape(-1)]
    best = min(minimize(f, x0 + 1e-3, method="Nelder-Mead", options=dict(xatol=1e-9, fatol=1e-12, maxiter=4000)).fun
               for x0 in starts)
    assert got <= best + 1e-7
    assert got >= best - 1e-6


def test_residuals_shrink_and_iterates_agree_at_convergence():
    rng = np.random.default_rng(4)
    s0 = rng.uniform(0, 1, (6, 7))
    y = np.roll(s0, 1, axis=1) + rng.normal(0, 0.02, (6, 7))
    s, st, rep = admm.uotdf(y, s0, 0.3, 1.0, 1.0, prox_iters=2, eps=1e-6, max_iter=20000, check_every=5, record=True)
    assert rep.converged
    assert np.max(np.abs(st.x - st.s)) < 1e-5 and np.max(np.abs(st.z - st.s)) < 1e-5
    rp = [h[1] for h in rep.history]
    assert rp[-1] < 1e-2 * rp[0]


def test_printed_one_block_s_step_ignores_the_transport_term():
    """The reading of the s-step: with the printed update (only the x-block,
    max(x + a, 0)) ADMM settles at s = y on one pixel, whatever kappa is,
    while the closed form moves s towards s0.  Planted here, in a copy of the
    oracle's iteration, to show why the step minimises both blocks."""
    import dataclasses
    from oracle import uot

    y, s0 = np.array([[1.3]]), np.array([[0.4]])
    kappa, mu, rho = 0.5, 0.8, 1.0
    st = admm.df_initial_state(s0, kappa, mu, rho)
    for _ in range(400):
        s = np.maximum(st.x + st.a, 0.0)  # the printed s-step
        x = (y + rho * (s - st.a)) / (1.0 + rho)
        prob = admm.df_problem(s0, s - st.b, kappa, mu, rho)
        t1, t2 = prob.unit_steps()
        pst = st.prox
        for _ in range(10):
            pst = uot.iterate(prob, pst, t1, t2)
        st = dataclasses.replace(st, s=s, x=x, z=pst.x1.copy(), a=st.a + x - s, b=st.b + pst.x1 - s, prox=pst)
    assert abs(st.s[0, 0] - 1.3) < 1e-6  # the transport-free point
    good, _, _ = admm.uotdf(y, s0, kappa, mu, rho, **KW)
    assert abs(good[0, 0] - 0.9) < 1e-6  # 0.4 + shrink(0.9, kappa mu)
