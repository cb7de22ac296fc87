"""The anisotropic flux norm (l1,1: sum |Mx| + |My|, component shrink in the
flux step) on the GPU against the FP64 oracle's anisotropic Algorithm 1:
iterates and certified bounds at a fixed iteration count for every mode and
both boundary readings, bitwise agreement of every tile shape, and the
converged value against the stored Beckmann linear programs
(tests/golden/lp_values.json, written by tests/golden/make_golden.py)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import uot as ora
from oracle.ops import DIST, PROX, PROX_FIXED
from paper_1909_00149_amd import uot as G
from tests.golden.make_golden import instance

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4
VAL_TOL = 1e-5


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def planes_for(mode, balanced):
    keys = ["Mx", "My", "a"] + ([] if balanced else ["r"])
    if mode == PROX:
        keys += ["x0", "x1"]
    if mode == PROX_FIXED:
        keys += ["x1"]
    return keys


def inputs(shape, seed):
    rng = np.random.default_rng(seed)
    p = (rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.5)).astype(np.float32)
    q = (rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.5)).astype(np.float32)
    p[0, 0] += 0.25
    q[-1, -1] += 0.25
    return p, q


def gpu(dev, p, q, mode, balanced, resid=1, bc=0, iters=150, tile_rows=0, mu=1.3, rho=0.7, tol=0.0,
        check_every=20, flags=0, max_iter=None):
    ny, nx = p.shape
    prm = G.Params(nx=nx, ny=ny, mode=mode, balanced=balanced, residual_p=resid, bc=bc, mu=mu, rho=rho,
                   max_iter=iters if max_iter is None else max_iter, check_every=check_every, tol=tol,
                   tile_rows=tile_rows, flags=flags, norm=G.NORM_ANISO)
    s = G.Solver(prm)
    out, rep = s.solve(to_dev(p, dev), to_dev(q, dev))
    torch.cuda.synchronize()
    s.close()
    return out, rep


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-30)


MODES = [(DIST, False, 1), (DIST, True, 1), (DIST, False, 2), (PROX, False, 1), (PROX, True, 1),
         (PROX_FIXED, False, 1), (PROX_FIXED, True, 1)]


@pytest.mark.parametrize("mode,balanced,resid", MODES)
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(29, 37), (1, 50), (13, 70), (9, 130)])
def test_fixed_iterations_match_oracle(dev, mode, balanced, resid, bc, shape):
    p, q = inputs(shape, 500 + 3 * shape[0] + shape[1])
    if balanced and mode == DIST and bc == 0:
        q = (q * (p.astype(np.float64).sum() / q.astype(np.float64).sum())).astype(np.float32)
    st, rep = gpu(dev, p, q, mode, balanced, resid, bc)
    prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), mode=mode, balanced=balanced,
                       residual_p=resid, bc=bc, mu=1.3, rho=0.7, norm="aniso")
    t1, t2 = prob.default_steps()
    ref, _ = ora.solve(prob, tau1=np.float32(t1), tau2=np.float32(t2), max_iter=150, tol=0.0, check_every=20)
    for k in planes_for(mode, balanced):
        g = st[k].double().cpu().numpy().reshape(shape)
        o = getattr(ref, k)
        err = float(np.abs(g - o).max())
        assert err <= ITER_TOL * max(1.0, float(np.abs(o).max())), (k, err)
    g = ora.certified_gap(prob, ref)
    assert rel(rep["objective"], g.objective) <= VAL_TOL
    if not balanced:
        assert rel(rep["primal"], g.primal) <= VAL_TOL
        assert abs(rep["dual"] - g.dual) <= VAL_TOL * max(abs(g.dual), abs(g.primal))


@pytest.mark.parametrize("ty", [4, 8, 16, 32, 116, 132, 316, 332, 4004, 4008, 2016, 4016, 8016, 4032, 8032])
@pytest.mark.parametrize("mode,balanced,resid", [(DIST, False, 1), (PROX, False, 2), (PROX_FIXED, True, 1)])
@pytest.mark.parametrize("shape", [(45, 133), (19, 66)])
def test_tile_shapes_agree_bitwise(dev, ty, mode, balanced, resid, shape):
    p, q = inputs(shape, 9)
    base, _ = gpu(dev, p, q, mode, balanced, resid, iters=40, tile_rows=4)
    st, _ = gpu(dev, p, q, mode, balanced, resid, iters=40, tile_rows=ty)
    for k in planes_for(mode, balanced):
        assert torch.equal(base[k], st[k]), k


def golden_cases():
    with open(os.path.join(os.path.dirname(__file__), "golden", "lp_values.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: f"s{c['seed']}-mu{c['mu']}-bc{c['bc']}-b{int(c['balanced'])}")
def test_converged_value_is_the_lp_value(dev, case):
    """Solved to rel_res <= 1e-6 (adaptive steps), the anisotropic value is
    the Beckmann linear program's to FP32 accuracy; the GPU's certified
    interval contains it."""
    p, q = instance(case["seed"], case["ny"], case["nx"])
    if case["balanced"]:
        q = q * (p.sum() / q.sum())
    mu = case["mu"] or 1.0
    st, rep = gpu(dev, p.astype(np.float32), q.astype(np.float32), DIST, case["balanced"], bc=case["bc"], mu=mu,
                  tol=1e-6, max_iter=100000, flags=G.UOT_ADAPTIVE_STEPS)
    ref = case["beckmann"]
    if case["balanced"]:
        assert rel(rep["objective"], ref) <= 2e-5, (rep, ref)
    else:
        assert rel(rep["primal"], ref) <= 2e-5, (rep, ref)
        assert rep["dual"] <= ref * (1 + 2e-5) and rep["primal"] >= ref * (1 - 2e-5)
