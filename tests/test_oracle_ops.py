"""Pins of the oracle's operators and single-step maps against what the paper
and mathematics fix: adjointness, the closed-form top eigenvalue against a
library eigensolver, each closed-form update against brute-force minimisation
of the subproblem that defines it, and the DCT Poisson solve against a dense
solve."""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle import ops, poisson, sparse_ops, uot
from oracle.ops import DIST, PROX, PROX_FIXED

SHAPES = [(1, 7), (7, 1), (5, 7), (8, 8), (16, 9)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [0, 1])
def test_adjoint_identity(shape, bc):
    """<D M, a> = <M, D* a> (D* named in the flux update of Sec. III-B)."""
    ny, nx = shape
    rng = np.random.default_rng(ny * 100 + nx + bc)
    Mx, My, a = rng.standard_normal((3, ny, nx))
    lhs = np.sum(ops.div(Mx, My, bc) * a)
    gx, gy = ops.div_adj(a, bc)
    if bc == 0:
        Mx[:, -1] = 0.0
        My[-1, :] = 0.0
    rhs = np.sum(Mx * gx + My * gy)
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [0, 1])
def test_div_matches_loop_assembled_matrix(shape, bc):
    """Slicing D equals the entry-by-entry sparse D; D* equals its transpose."""
    ny, nx = shape
    rng = np.random.default_rng(7 + nx + bc)
    Mx, My, a = rng.standard_normal((3, ny, nx))
    D = sparse_ops.div_matrix(nx, ny, bc)
    v = sparse_ops.pack_flux(Mx, My, bc)
    assert np.allclose((D @ v).reshape(ny, nx), ops.div(Mx, My, bc), atol=1e-14, rtol=0)
    gx, gy = ops.div_adj(a, bc)
    gvx, gvy = sparse_ops.unpack_flux(D.T @ a.reshape(-1), nx, ny, bc)
    assert np.allclose(gx, gvx, atol=1e-14) and np.allclose(gy, gvy, atol=1e-14)
    # at most 4 nonzeros per row (Sec. III-B cost analysis)
    assert np.diff(D.indptr).max() <= 4


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (3, 5), (8, 8), (16, 7), (5, 16), (16, 16)])
@pytest.mark.parametrize("bc", [0, 1])
def test_lambda_max_closed_form(shape, bc):
    ny, nx = shape
    D = sparse_ops.div_matrix(nx, ny, bc).toarray()
    lam = np.linalg.eigvalsh(D @ D.T).max()
    assert abs(lam - ops.lam_max(nx, ny, bc)) <= 1e-12 * max(1.0, lam)


def test_lambda_max_small_factors():
    # 1-D factor at n = 2: spectrum {0, 2} (zero flux) and {0.382, 2.618} (literal)
    assert abs(ops.lam_max_1d(2, 0) - 2.0) < 1e-14
    assert abs(ops.lam_max_1d(2, 1) - (3 + 5 ** 0.5) / 2) < 1e-14
    assert ops.lam_max_1d(1, 0) == 0.0 and abs(ops.lam_max_1d(1, 1) - 1.0) < 1e-14


def test_knorm_blocks():
    for mode, bal, k in [(DIST, False, 1), (DIST, True, 0), (PROX, False, 3), (PROX, True, 2),
                         (PROX_FIXED, False, 2), (PROX_FIXED, True, 1)]:
        nx, ny = 6, 4
        prob = uot.Problem(np.zeros((ny, nx)), np.zeros((ny, nx)), mode=mode, balanced=bal)
        # ||K||^2 from the dense operator
        D = sparse_ops.div_matrix(nx, ny, 0).toarray()
        N = nx * ny
        K = np.hstack([D] + [np.eye(N)] * k)
        assert abs(np.linalg.eigvalsh(K @ K.T).max() - prob.knorm2()) < 1e-11


def _brute_group(v, sigma):
    f = lambda m: sigma * np.hypot(*m) + 0.5 * np.sum((m - v) ** 2)
    best = minimize(f, v * 0.5, method="Nelder-Mead", options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
    cand = [best.x, np.zeros(2)]
    return min(cand, key=f)


def test_group_shrink_vs_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(40):
        v = rng.standard_normal(2) * rng.choice([0.1, 1.0, 3.0])
        sigma = rng.uniform(0.05, 2.0)
        mx, my = ops.shrink2(np.array([v[0]]), np.array([v[1]]), sigma)
        b = _brute_group(v, sigma)
        assert np.allclose([mx[0], my[0]], b, atol=1e-6)
    # zero vector maps to zero, no NaN
    mx, my = ops.shrink2(np.zeros(3), np.zeros(3), 0.5)
    assert np.all(mx == 0) and np.all(my == 0)


def test_scalar_shrink_vs_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(40):
        v, s = rng.standard_normal() * 2, rng.uniform(0.01, 1.5)
        res = minimize_scalar(lambda r: s * abs(r) + 0.5 * (r - v) ** 2, bounds=(-10, 10),
                              method="bounded", options=dict(xatol=1e-12))
        assert abs(ops.shrink1(v, s) - res.x) < 1e-7
    assert ops.shrink1(0.0, 0.3) == 0.0


def _one_step(mode, bal, p_res, seed=5, bc=0, ny=4, nx=5):
    rng = np.random.default_rng(seed)
    src = rng.uniform(0, 1, (ny, nx))
    dst = rng.uniform(0, 1, (ny, nx))
    prob = uot.Problem(src, dst, mode=mode, balanced=bal, residual_p=p_res, bc=bc, mu=0.7, rho=1.9)
    st = uot.initial_state(prob, uot.State(*rng.standard_normal((4, ny, nx)) * 0.3,
                                           rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 1, (ny, nx))))
    tau1, tau2 = 0.21, 0.33
    return prob, st, uot.iterate(prob, st, tau1, tau2), tau1, tau2


@pytest.mark.parametrize("bc", [0, 1])
def test_flux_update_vs_brute_force(bc):
    """M^{k+1} = argmin ||M||_{2,1} + <a, D M> + ||M - M^k||^2/(2 tau1) (eq. Prox_UOT_M),
    minimised per pixel with D^T a taken from the loop-assembled matrix."""
    prob, st, new, tau1, _ = _one_step(DIST, False, 1, bc=bc)
    ny, nx = prob.shape
    D = sparse_ops.div_matrix(nx, ny, bc)
    gx, gy = sparse_ops.unpack_flux(D.T @ st.a.reshape(-1), nx, ny, bc)
    for j in range(ny):
        for i in range(nx):
            exist = np.array([bc == 1 or i < nx - 1, bc == 1 or j < ny - 1], dtype=float)
            m0 = np.array([st.Mx[j, i], st.My[j, i]]) * exist
            g = np.array([gx[j, i], gy[j, i]])
            f = lambda m: (np.hypot(*(m * exist)) + g @ (m * exist)
                           + np.sum(((m - m0) * exist) ** 2) / (2 * tau1))
            b = minimize(f, m0, method="Nelder-Mead", options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000)).x
            b = min([b * exist, np.zeros(2)], key=f)
            assert np.allclose([new.Mx[j, i], new.My[j, i]], b * exist, atol=1e-6)


@pytest.mark.parametrize("mode", [PROX, PROX_FIXED])
def test_projection_update_vs_brute_force(mode):
    """x^{k+1} = argmin_{x>=0} ||x-p||^2/(2 rho) + <a, A x> + ||x-x^k||^2/(2 tau1) (eq. Prox_UOT_x)
    with the prox weight 1/(2 rho) of the prox definition."""
    prob, st, new, tau1, _ = _one_step(mode, False, 1)
    rho = prob.rho
    blocks = [("x1", prob.dst, +1.0)] + ([("x0", prob.src, -1.0)] if mode == PROX else [])
    for name, p, sgn in blocks:
        xk, xn = getattr(st, name), getattr(new, name)
        for idx in np.ndindex(xk.shape):
            a = st.a[idx]
            f = lambda x: (x - p[idx]) ** 2 / (2 * rho) + sgn * a * x + (x - xk[idx]) ** 2 / (2 * tau1)
            res = minimize_scalar(f, bounds=(0, 20), method="bounded", options=dict(xatol=1e-12))
            assert abs(xn[idx] - res.x) < 1e-6
    if mode == PROX_FIXED:
        assert np.array_equal(new.x0, prob.src)


@pytest.mark.parametrize("p_res", [1, 2])
def test_residual_update_vs_brute_force(p_res):
    """r^{k+1} = argmin mu |r|^p + <a, -r> + ||r - r^k||^2/(2 tau1) (eq. Prox_UOT_r)."""
    prob, st, new, tau1, _ = _one_step(DIST, False, p_res)
    mu = prob.mu
    for idx in np.ndindex(st.r.shape):
        f = lambda r: mu * (abs(r) if p_res == 1 else r * r) - st.a[idx] * r + (r - st.r[idx]) ** 2 / (2 * tau1)
        res = minimize_scalar(f, bounds=(-10, 10), method="bounded", options=dict(xatol=1e-12))
        assert abs(new.r[idx] - res.x) < 1e-6


@pytest.mark.parametrize("mode", [DIST, PROX, PROX_FIXED])
@pytest.mark.parametrize("bal", [False, True])
def test_dual_update_extrapolation(mode, bal):
    """a^{k+1} = a^k + tau2 (2 K(z^{k+1}) - K(z^k)) with K assembled from the
    loop-built D and the block signs [D, -I, +I, -I] (eq. Prox_UOT_a)."""
    prob, st, new, _, tau2 = _one_step(mode, bal, 1)
    ny, nx = prob.shape
    D = sparse_ops.div_matrix(nx, ny, 0)

    def K(s):
        v = D @ sparse_ops.pack_flux(s.Mx, s.My, 0) - s.x0.reshape(-1) + s.x1.reshape(-1)
        if not bal:
            v = v - s.r.reshape(-1)
        return v.reshape(ny, nx)
    assert np.allclose(new.a, st.a + tau2 * (2 * K(new) - K(st)), atol=1e-13)


@pytest.mark.parametrize("shape", [(1, 5), (6, 1), (4, 7), (16, 16), (9, 32)])
@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_dct_poisson_vs_direct(shape, alpha):
    ny, nx = shape
    rng = np.random.default_rng(nx * ny)
    c = rng.standard_normal((ny, nx))
    if alpha == 0.0:
        c -= c.mean()
    a = poisson.dct_solve(c, alpha)
    b = poisson.direct_solve(c, alpha)
    if alpha == 0.0:
        a = a - a.mean()
    assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max())
