"""The DCT-diagonalised Neumann-Poisson solve (GPU, FP32) against the
oracle's dense direct solve, and what is built on it: the Poisson-flux
warm start and the certified gap of the balanced mode."""
import numpy as np
import pytest
import torch

from oracle import ops, poisson, uot as ora
from oracle.ops import DIST
from paper_1909_00149_amd import synth
from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


@pytest.mark.parametrize("shape", [(5, 7), (16, 16), (33, 20), (1, 40), (40, 1), (70, 129)])
@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_poisson_vs_direct_solve(dev, shape, alpha):
    ny, nx = shape
    rng = np.random.default_rng(ny * 1000 + nx)
    c = rng.standard_normal(shape).astype(np.float32)
    s = G.Solver(G.Params(nx=nx, ny=ny))
    phi = s.poisson(torch.from_numpy(c).to(dev), alpha).double().cpu().numpy()
    cc = c.astype(np.float64)
    if alpha == 0.0:
        cc = cc - cc.mean()
    ref = poisson.direct_solve(cc, alpha)
    if alpha == 0.0:
        phi = phi - phi.mean()
    err = np.abs(phi - ref).max()
    assert err <= 2e-5 * max(1.0, np.abs(ref).max()), err


def test_poisson_start_satisfies_constraint(dev):
    p, q = synth.unbalanced_pair(8, side=96)
    s = G.Solver(G.Params(nx=96, ny=96, mu=8.0))
    P, Q = torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev)
    st = s.init_poisson(P, Q)
    torch.cuda.synchronize()
    Mx, My, r, a = (st[k].double().cpu().numpy() for k in ("Mx", "My", "r", "a"))
    c = (q.astype(np.float64) - p.astype(np.float64))
    # K z0 = D M0 + c - r0 = 0
    assert np.abs(ops.div(Mx, My, 0) + c - r).max() <= 1e-6
    assert np.abs(a).max() == 0.0
    # M0 = -D* phi with D D* phi = c - mean(c) (oracle: dense least squares)
    phi = poisson.direct_solve(c - c.mean(), 0.0)
    gx, gy = ops.div_adj(phi, 0)
    assert np.abs(Mx + gx).max() <= 1e-5 * max(1.0, np.abs(gx).max())
    assert np.abs(My + gy).max() <= 1e-5 * max(1.0, np.abs(gy).max())
    # r0 is the uniform residual mean(c)
    assert np.abs(r - c.mean()).max() <= 1e-6


def test_poisson_warm_start_converges_to_same_value(dev):
    p, q = synth.unbalanced_pair(9, side=64)
    kw = dict(nx=64, ny=64, mu=8.0, max_iter=40000, check_every=20, tol=1e-5)
    P, Q = torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev)
    cold = G.Solver(G.Params(flags=G.UOT_ADAPTIVE_STEPS, **kw))
    _, rc = cold.solve(P, Q)
    warm = G.Solver(G.Params(flags=G.UOT_ADAPTIVE_STEPS | G.UOT_WARM_START, **kw))
    st = warm.init_poisson(P, Q)
    _, rw = warm.solve(P, Q, st)
    torch.cuda.synchronize()
    assert rc["status_name"] == "CONVERGED" and rw["status_name"] == "CONVERGED", (rc, rw)
    assert abs(rc["primal"] - rw["primal"]) <= 1e-3 * rc["primal"], (rc, rw)


@pytest.mark.parametrize("seed", [0, 3])
def test_balanced_certified_gap_matches_oracle(dev, seed):
    """The balanced primal bound repairs the flux with the Poisson solve;
    at the same iterate it must equal the oracle's dense-repair bound."""
    p, q = synth.balanced_pair(seed, side=40)
    it = 300
    s = G.Solver(G.Params(nx=40, ny=40, balanced=True, max_iter=it))
    st, rep = s.solve(torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev))
    torch.cuda.synchronize()
    prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), balanced=True)
    t1, t2 = prob.default_steps()
    ref, _ = ora.solve(prob, tau1=np.float32(t1), tau2=np.float32(t2), max_iter=it, tol=0)
    g = ora.certified_gap(prob, ref)
    assert abs(rep["primal"] - g.primal) <= 1e-5 * g.primal, (rep["primal"], g.primal)
    assert abs(rep["dual"] - g.dual) <= 1e-5 * g.primal, (rep["dual"], g.dual)
    assert rep["dual"] <= rep["primal"]


def test_balanced_converged_gap_closes(dev):
    p, q = synth.balanced_pair(2, side=32)
    s = G.Solver(G.Params(nx=32, ny=32, balanced=True, max_iter=40000, tol=1e-6, flags=G.UOT_ADAPTIVE_STEPS))
    _, rep = s.solve(torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev))
    torch.cuda.synchronize()
    assert rep["rel_gap"] <= 1e-3, rep
