"""Pins of the oracle's Algorithm 1 at the solution level, against routes
that share no code with it: closed forms, LPs, an independent splitting
solver, invariants and the duality certificate."""
import json
import os

import numpy as np
import pytest

from oracle import dr, lp, ops, uot
from oracle.ops import DIST, PROX, PROX_FIXED

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lp_values.json")


def _solve(prob, tol=1e-11, max_iter=200000, **kw):
    st, rep = uot.solve(prob, max_iter=max_iter, tol=tol, check_every=100, **kw)
    return st, rep, uot.certified_gap(prob, st)


def _instance(seed, ny, nx, density=0.35):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, (ny, nx)) * (rng.uniform(0, 1, (ny, nx)) < density)
    q = rng.uniform(0, 1, (ny, nx)) * (rng.uniform(0, 1, (ny, nx)) < density)
    p[0, 0] += 0.1
    q[-1, -1] += 0.1
    return p, q


@pytest.mark.parametrize("n", [2, 9, 40])
def test_1d_balanced_is_cumsum(n):
    """On an n x 1 grid with zero-flux ends the balanced value is
    sum |cumsum(p - q)| (W1 on a line) and the flux is that cumsum (unique)."""
    rng = np.random.default_rng(n)
    p = rng.uniform(0, 1, (1, n))
    q = rng.uniform(0, 1, (1, n))
    q *= p.sum() / q.sum()
    prob = uot.Problem(p, q, balanced=True)
    st, rep, g = _solve(prob, tol=1e-12)
    cs = np.cumsum(p - q)
    ref = np.sum(np.abs(cs[:-1]))
    assert rep.status == "CONVERGED"
    assert abs(g.primal - ref) <= 1e-10 * ref and abs(g.dual - ref) <= 1e-9 * ref
    assert np.abs(st.Mx[0, :-1] - cs[:-1]).max() <= 1e-8
    # the same grid stood on end (1 x n -> n x 1) gives the same value
    prob_t = uot.Problem(p.T, q.T, balanced=True)
    _, _, gt = _solve(prob_t, tol=1e-12)
    assert abs(gt.primal - ref) <= 1e-9 * ref


@pytest.mark.parametrize("mu", [0.3, 1.7, 6.0])
def test_1d_unbalanced_vs_kantorovich_lp(mu):
    n = 24
    rng = np.random.default_rng(int(mu * 10))
    p = rng.uniform(0, 1, (1, n)) * (rng.uniform(0, 1, (1, n)) < 0.4)
    q = rng.uniform(0, 1, (1, n)) * (rng.uniform(0, 1, (1, n)) < 0.4)
    p[0, 2] += 0.5
    q[0, -3] += 0.2
    ref = lp.kantorovich(p, q, mu, False, lp.manhattan_cost(n, 1))
    _, _, g = _solve(uot.Problem(p, q, mu=mu))
    assert abs(g.primal - ref) <= 1e-9 * ref


def _golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: f"s{c['seed']}-mu{c['mu']}-bc{c['bc']}-b{int(c['balanced'])}")
def test_aniso_vs_lp_golden(case):
    """The anisotropic variant of Algorithm 1 against stored values of the
    Beckmann LP and (zero-flux boundary) the Kantorovich LP with Manhattan cost."""
    from tests.golden.make_golden import instance
    p, q = instance(case["seed"], case["ny"], case["nx"])
    if case["balanced"]:
        q = q * (p.sum() / q.sum())
    if "kantorovich" in case:
        assert abs(case["kantorovich"] - case["beckmann"]) <= 1e-9 * case["beckmann"]
    prob = uot.Problem(p, q, mu=case["mu"] or 1.0, bc=case["bc"], balanced=case["balanced"], norm="aniso")
    _, rep, g = _solve(prob)
    ref = case["beckmann"]
    assert abs(g.primal - ref) <= 1e-8 * ref and abs(g.dual - ref) <= 1e-8 * ref


@pytest.mark.parametrize("seed", [21, 22])
def test_iso_between_aniso_bounds(seed):
    """ANISO*/sqrt(2) <= ISO* <= ANISO* (the l2 and l1 norms of a 2-vector)."""
    p, q = _instance(seed, 6, 7)
    for bal in (False, True):
        qq = q * (p.sum() / q.sum()) if bal else q
        iso = _solve(uot.Problem(p, qq, mu=1.1, balanced=bal), tol=1e-9)[2].primal
        an = lp.beckmann_aniso(p, qq, 1.1, 0, bal)
        assert an / np.sqrt(2) - 1e-9 <= iso <= an + 1e-9


DR_CASES = [
    dict(mode=DIST, balanced=False, residual_p=1, bc=0),
    dict(mode=DIST, balanced=True, residual_p=1, bc=0),
    dict(mode=DIST, balanced=False, residual_p=2, bc=0),
    dict(mode=DIST, balanced=False, residual_p=1, bc=1),
    dict(mode=DIST, balanced=True, residual_p=1, bc=1),
    dict(mode=PROX, balanced=False, residual_p=1, bc=0),
    dict(mode=PROX, balanced=True, residual_p=1, bc=0),
    dict(mode=PROX, balanced=False, residual_p=2, bc=1),
    dict(mode=PROX_FIXED, balanced=False, residual_p=1, bc=0),
    dict(mode=PROX_FIXED, balanced=True, residual_p=1, bc=0),
]


@pytest.mark.parametrize("case", DR_CASES, ids=lambda c: "-".join(f"{k}{int(v)}" for k, v in c.items()))
def test_iso_vs_douglas_rachford(case):
    """Algorithm 1 and an independent Douglas-Rachford solver (dense
    projection onto the divergence constraint) reach one optimal value; the
    prox output x is unique (strong convexity) and must agree too."""
    p, q = _instance(31, 5, 6)
    if case["balanced"] and case["mode"] == DIST:
        q = q * (p.sum() / q.sum())
    if case["balanced"] and case["mode"] == PROX_FIXED:
        q = q * (p.sum() / q.sum())
    kw = dict(mu=0.9, rho=0.6)
    prob = uot.Problem(p, q, **case, **kw)
    st, rep, g = _solve(prob, tol=1e-12, max_iter=400000)
    s = dr.DRSolver(p, q, **case, **kw)
    z = s.solve(iters=200000)
    ref = s.objective(z)
    assert abs(g.primal - ref) <= 1e-8 * max(ref, 1.0)
    assert g.rel_gap <= 1e-8
    u = s.unpack(z)
    if case["mode"] == PROX:
        assert np.abs(u["x0"] - st.x0).max() <= 1e-7 and np.abs(u["x1"] - st.x1).max() <= 1e-7
    if case["mode"] == PROX_FIXED:
        assert np.abs(u["x1"] - st.x1).max() <= 1e-7


@pytest.mark.parametrize("d,mu,m1,m2", [(2, 1.3, 1.0, 0.7), (3, 0.9, 0.5, 0.8), (4, 1.2, 1.0, 1.0),
                                        (6, 1.0, 1.0, 0.6)])
@pytest.mark.parametrize("axis", [0, 1])
def test_point_masses_closed_form(d, mu, m1, m2, axis):
    """Point masses m1, m2 at axis-aligned distance d, away from the edge:
    V = min(d, 2 mu) min(m1, m2) + mu |m1 - m2|; when d < 2 mu the flux is the
    straight segment carrying min(m1, m2)."""
    shape = (7, 11) if axis == 0 else (11, 7)
    p = np.zeros(shape)
    q = np.zeros(shape)
    if axis == 0:
        p[3, 2] = m1
        q[3, 2 + d] = m2
    else:
        p[2, 3] = m1
        q[2 + d, 3] = m2
    prob = uot.Problem(p, q, mu=mu)
    st, rep, g = _solve(prob, tol=1e-10, max_iter=60000)
    ref = min(d, 2 * mu) * min(m1, m2) + mu * abs(m1 - m2)
    # the closed form lies inside the certified interval [D_hat, P_hat],
    # which is narrow
    assert g.dual - 1e-12 <= ref <= g.primal + 1e-12
    assert g.rel_gap <= 1e-5
    if d < 2 * mu:
        M = st.Mx if axis == 0 else st.My
        seg = M[3, 2:2 + d] if axis == 0 else M[2:2 + d, 3]
        assert np.abs(seg - min(m1, m2)).max() <= 1e-3
        other = st.My if axis == 0 else st.Mx
        assert np.abs(other).max() <= 1e-3


def test_mu_large_gives_balanced():
    """For balanced inputs and 2 mu above the grid diameter, V_mu equals the
    balanced value (the mu -> infinity remark of Sec. III-A)."""
    p, q = _instance(41, 5, 6)
    q = q * (p.sum() / q.sum())
    vb = _solve(uot.Problem(p, q, balanced=True))[2].primal
    vu = _solve(uot.Problem(p, q, mu=0.5 * (5 + 6) + 1.0))[2].primal
    assert abs(vb - vu) <= 1e-8 * vb


def _interval(prob, iters=20000, scale=1.0):
    st, _ = uot.solve(prob, max_iter=iters, tol=1e-11, check_every=100)
    g = uot.certified_gap(prob, st)
    assert g.rel_gap <= 1e-4
    return g.dual * scale, g.primal * scale


def _overlap(i1, i2):
    return max(i1[0], i2[0]) <= min(i1[1], i2[1]) + 1e-12


def test_invariants():
    """Symmetry, 1-homogeneity, V(p,p) = 0, translation away from edges and
    transposition of both images.  Each value is bracketed by its certified
    interval [D_hat, P_hat]; an invariance holds only if the intervals meet."""
    p, q = _instance(51, 6, 6)
    P = np.zeros((10, 12))
    Q = np.zeros((10, 12))
    P[2:8, 3:9], Q[2:8, 3:9] = p, q
    mu = 1.3
    base = _interval(uot.Problem(P, Q, mu=mu))
    assert _overlap(base, _interval(uot.Problem(Q, P, mu=mu)))
    assert _overlap(base, _interval(uot.Problem(2.5 * P, 2.5 * Q, mu=mu), scale=1 / 2.5))
    assert _solve(uot.Problem(P, P, mu=mu))[2].primal <= 1e-10
    P2 = np.roll(np.roll(P, 1, 0), -2, 1)
    Q2 = np.roll(np.roll(Q, 1, 0), -2, 1)
    assert _overlap(base, _interval(uot.Problem(P2, Q2, mu=mu)))
    assert _overlap(base, _interval(uot.Problem(P.T.copy(), Q.T.copy(), mu=mu)))
    # and a pair that is not a symmetry image must fall outside: swapping
    # only one image for its transpose changes the value
    other = _interval(uot.Problem(P, np.ascontiguousarray(Q[::-1, ::-1]), mu=mu))
    assert not _overlap(base, other)


def test_gap_certificate_and_ergodic_decrease():
    """The certified gap closes and rel_res goes to zero with it.  The gap of
    the ergodic average at k = 25 * 2^j does not increase (the O(1/k)
    ergodic rate of the primal-dual method; a per-iterate gap need not be
    monotone)."""
    p, q = _instance(61, 8, 8)
    prob = uot.Problem(p, q, mu=1.4)
    t1, t2 = prob.default_steps()
    st = uot.initial_state(prob)
    acc = None
    checks = {25 * 2 ** j for j in range(8)}
    gaps = []
    for k in range(1, max(checks) + 1):
        prev, st = st, uot.iterate(prob, st, t1, t2)
        acc = st.copy() if acc is None else uot.State(*(a + b for a, b in zip(
            (acc.Mx, acc.My, acc.r, acc.a, acc.x0, acc.x1), (st.Mx, st.My, st.r, st.a, st.x0, st.x1))))
        if k in checks:
            avg = uot.State(*(v / k for v in (acc.Mx, acc.My, acc.r, acc.a, acc.x0, acc.x1)))
            g = uot.certified_gap(prob, avg)
            gaps.append(g.primal - g.dual)
    assert all(g >= -1e-12 for g in gaps)
    assert all(b <= a + 1e-12 for a, b in zip(gaps, gaps[1:]))
    g = uot.certified_gap(prob, st)
    _, _, rel = uot.residuals(prob, prev, st, t1)
    assert g.rel_gap <= 1e-6 and rel <= 1e-6


def test_step_bound():
    """tau1 tau2 ||K||^2 = 0.98 converges; far above the bound of Theorem 1
    the iterates blow up."""
    p, q = _instance(71, 6, 6)
    prob = uot.Problem(p, q, mu=1.0)
    _, rep = uot.solve(prob, max_iter=20000, tol=1e-9, check_every=50)
    assert rep.status == "CONVERGED"
    t = 2.2 / np.sqrt(prob.knorm2())
    st, rep = uot.solve(prob, tau1=t, tau2=t, max_iter=2000, tol=0)
    assert rep.status == "DIVERGED" or np.abs(st.a).max() > 1e6


def test_prox_small_rho_returns_argument_and_fixed_point():
    p, q = _instance(81, 5, 5)
    prob = uot.Problem(p, q, mode=PROX, mu=1.0, rho=1e-4)
    st, rep, g = _solve(prob, tol=1e-12)
    assert np.abs(st.x0 - p).max() <= 1e-3 and np.abs(st.x1 - q).max() <= 1e-3
    prob = uot.Problem(p, q, mode=PROX, mu=1.0, rho=0.8)
    st, rep, g = _solve(prob, tol=1e-12)
    t1, t2 = prob.default_steps()
    nxt = uot.iterate(prob, st, t1, t2)
    assert np.abs(nxt.x0 - st.x0).max() <= 1e-9 and np.abs(nxt.x1 - st.x1).max() <= 1e-9


def test_determinism_and_resume():
    """Two runs agree bitwise; 2k iterations equal k iterations followed by a
    warm-started k (the caller's state is the checkpoint)."""
    p, q = _instance(91, 6, 7)
    prob = uot.Problem(p, q, mu=1.1)
    a, _ = uot.solve(prob, max_iter=300, tol=0)
    b, _ = uot.solve(prob, max_iter=300, tol=0)
    assert all(np.array_equal(x, y) for x, y in zip(vars(a).values(), vars(b).values()))
    h, _ = uot.solve(prob, max_iter=150, tol=0)
    c, _ = uot.solve(prob, max_iter=150, tol=0, state=h)
    assert all(np.array_equal(x, y) for x, y in zip(vars(a).values(), vars(c).values()))
