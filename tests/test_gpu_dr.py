"""The Douglas-Rachford splitting on the GPU (uot_dr_solve: separable prox,
then the exact projection onto {K z = b} through the DCT Poisson solve)
against the oracle's independent Douglas-Rachford solver (oracle/dr.py:
dense pseudo-inverse projection), iterate for iterate; its converged value
against Algorithm 1's certified optimum; graph replay against direct
launches; and the input checks."""
import numpy as np
import pytest
import torch

from oracle import dr as odr
from oracle import uot as ora
from oracle.ops import DIST, PROX, PROX_FIXED
from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def inputs(shape, seed, balanced, mode):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.4)
    q = rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.4)
    p[0, 0] += 0.2
    q[-1, -1] += 0.2
    if balanced and mode in (DIST, PROX_FIXED):
        q = q * (p.sum() / q.sum())
    return p.astype(np.float32), q.astype(np.float32)


CASES = [(DIST, False, 1), (DIST, True, 1), (DIST, False, 2), (PROX, False, 1), (PROX, True, 1),
         (PROX, False, 2), (PROX_FIXED, False, 1), (PROX_FIXED, True, 1)]


def gpu_dr(dev, p, q, mode, balanced, resid, iters, gamma, tol=0.0, check_every=10, flags=0, norm=0):
    ny, nx = p.shape
    s = G.Solver(G.Params(nx=nx, ny=ny, mode=mode, balanced=balanced, residual_p=resid, mu=0.9, rho=0.6,
                          max_iter=iters, check_every=check_every, tol=tol, flags=flags, norm=norm))
    st, rep = s.dr_solve(to_dev(p, dev), to_dev(q, dev), gamma=gamma)
    torch.cuda.synchronize()
    s.close()
    return st, rep


@pytest.mark.parametrize("mode,balanced,resid", CASES)
@pytest.mark.parametrize("shape", [(6, 7), (13, 20), (1, 24)])
@pytest.mark.parametrize("gamma", [0.5, 2.0])
def test_iterates_match_the_dense_oracle(dev, mode, balanced, resid, shape, gamma):
    """47 iterations (windows of 10 and a tail of 7): the GPU's z (FP32, DCT
    projection) against the oracle's (FP64, pseudo-inverse projection)."""
    p, q = inputs(shape, 40 + shape[0] + shape[1], balanced, mode)
    iters = 47
    st, rep = gpu_dr(dev, p, q, mode, balanced, resid, iters, gamma)
    assert rep["iters"] == iters
    o = odr.DRSolver(p.astype(np.float64), q.astype(np.float64), mode=mode, balanced=balanced, residual_p=resid,
                     bc=0, mu=0.9, rho=0.6, gamma=gamma)
    z = o.solve(iters=iters, tol=0.0)
    ref = o.unpack(z)
    for k in ("Mx", "My", "r", "x0", "x1"):
        if k not in ref:
            continue
        g = st[k].double().cpu().numpy().reshape(shape)
        err = float(np.abs(g - ref[k]).max())
        assert err <= 2e-4 * max(1.0, float(np.abs(ref[k]).max())), (k, err)
    assert abs(rep["objective"] - o.objective(z)) <= 1e-4 * max(1.0, o.objective(z))


@pytest.mark.parametrize("mode,balanced,resid", [(DIST, False, 1), (DIST, True, 1), (PROX, False, 1),
                                                 (PROX_FIXED, False, 2)])
@pytest.mark.parametrize("norm", [0, 1])
def test_converged_value_is_algorithm_1s(dev, mode, balanced, resid, norm):
    """Run to a fixed-point residual of 1e-5 (FP32 iterates stall near 1e-6),
    the DR point is feasible to FP32 accuracy and its value is the optimum
    that Algorithm 1's oracle certifies (both flux norms; the oracle's
    anisotropic Algorithm 1 is pinned to the stored linear programs)."""
    p, q = inputs((16, 19), 77, balanced, mode)
    st, rep = gpu_dr(dev, p, q, mode, balanced, resid, 40000, 1.0, tol=1e-5, check_every=50, norm=norm)
    assert rep["status_name"] == "CONVERGED", rep
    prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), mode=mode, balanced=balanced, residual_p=resid,
                       mu=0.9, rho=0.6, norm=["iso", "aniso"][norm])
    ref, _ = ora.solve(prob, max_iter=200000, tol=1e-10, check_every=50, adaptive=True)
    g = ora.certified_gap(prob, ref)
    assert g.rel_gap <= 1e-7
    scale = max(1.0, float(np.abs(p).sum() + np.abs(q).sum()))
    assert rep["infeasibility"] <= 1e-4 * scale
    assert abs(rep["objective"] - g.primal) <= 1e-4 * max(g.primal, 1.0), (rep["objective"], g.primal)


def test_graph_replay_equals_direct_launches(dev):
    p, q = inputs((33, 70), 5, False, DIST)
    a, ra = gpu_dr(dev, p, q, DIST, False, 1, 57, 1.5, check_every=8)
    b, rb = gpu_dr(dev, p, q, DIST, False, 1, 57, 1.5, check_every=8, flags=G.UOT_NO_GRAPH)
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert ra["fixed_point_res"] == rb["fixed_point_res"] and ra["objective"] == rb["objective"]


def test_input_checks(dev):
    p, q = inputs((8, 9), 1, False, DIST)
    s = G.Solver(G.Params(nx=9, ny=8, mode=DIST, bc=1, max_iter=10, check_every=5))
    with pytest.raises(G.UOTError):
        s.dr_solve(to_dev(p, dev), to_dev(q, dev))
    s = G.Solver(G.Params(nx=9, ny=8, mode=DIST, max_iter=10, check_every=5))
    with pytest.raises(G.UOTError):
        s.dr_solve(to_dev(p, dev), to_dev(q, dev), gamma=0.0)
    bad = p.copy()
    bad[2, 2] = -1.0
    with pytest.raises(G.UOTError):
        s.dr_solve(to_dev(bad, dev), to_dev(q, dev))
    qb = q * 2.0
    s = G.Solver(G.Params(nx=9, ny=8, mode=DIST, balanced=True, max_iter=10, check_every=5))
    with pytest.raises(G.UOTError):
        s.dr_solve(to_dev(p, dev), to_dev(qb, dev))
