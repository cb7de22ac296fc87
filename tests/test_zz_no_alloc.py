"""uot_solve_noalloc (the entry point for callers that cannot allocate)
against uot_solve through the C ABI: the same kernels on the same inputs,
so the iterates and reports must agree bitwise.  Two calls in a row, the
second on a smaller grid, so the second runs on the scratch the first left
behind; plus the size limit and the argument checks."""
import numpy as np
import pytest
import torch

from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def inputs(shape, seed):
    rng = np.random.default_rng(seed)
    p = (rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.5)).astype(np.float32)
    q = (rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.5)).astype(np.float32)
    p[0, 0] += 0.25
    q[-1, -1] += 0.25
    return p, q


CASES = [
    # (mode, balanced, resid, first shape, second (smaller) shape, tol)
    (G.DIST, False, 1, (300, 257), (40, 70), 1e-3),
    (G.PROX, False, 2, (130, 190), (33, 65), 0.0),
    (G.DIST, True, 1, (96, 160), (17, 23), 1e-4),
    (G.PROX_FIXED, False, 1, (200, 64), (9, 130), 1e-5),
]


def run_both(dev, mode, balanced, resid, shape, tol, seed):
    p, q = inputs(shape, seed)
    if balanced:
        q = (q * (p.astype(np.float64).sum() / q.astype(np.float64).sum())).astype(np.float32)
    ny, nx = shape
    prm = G.Params(nx=nx, ny=ny, mode=mode, balanced=balanced, residual_p=resid, mu=1.2, rho=0.8, max_iter=700,
                   check_every=20, tol=tol, flags=G.UOT_ADAPTIVE_STEPS if tol > 0 else 0)
    src, dst = torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev)
    ref, rref = G.Solver(prm).solve(src, dst)
    got, rgot = G.solve_noalloc(prm, src, dst)
    torch.cuda.synchronize()
    return ref, rref, got, rgot


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_uot_solve_twice(dev, case):
    mode, balanced, resid, big, small, tol = CASES[case]
    for i, shape in enumerate((big, small)):
        ref, rref, got, rgot = run_both(dev, mode, balanced, resid, shape, tol, 100 * case + i)
        for k in G.required_planes(mode, balanced):
            assert torch.equal(ref[k], got[k]), (shape, k)
        assert float(ref["Mx"].abs().max()) > 0.0  # the flux moved
        for f in ("iters", "status", "tile_rows"):
            assert rref[f] == rgot[f], (shape, f)
        for f in ("rel_res", "objective", "feas", "tau1", "tau2"):
            assert rref[f] == rgot[f], (shape, f)
        if balanced:
            assert np.isnan(rgot["primal"])  # no Poisson certificate without allocations
        else:
            for f in ("primal", "dual"):
                assert rref[f] == rgot[f] or (np.isnan(rref[f]) and np.isnan(rgot[f])), (shape, f)


def test_noalloc_limits_and_arguments(dev):
    n = G._lib.UOT_NOALLOC_MAX_PIXELS
    p = torch.zeros((1025, 1024), dtype=torch.float32, device=dev)
    with pytest.raises(G.UOTError) as e:
        G.solve_noalloc(G.Params(nx=1024, ny=1025, max_iter=10), p, p)
    assert e.value.code == 9 and 1025 * 1024 > n
    q = torch.zeros((1, 1 << 18), dtype=torch.float32, device=dev)  # 2^18 px fit, their 4-row tiles do not
    with pytest.raises(G.UOTError) as e:
        G.solve_noalloc(G.Params(nx=1, ny=1 << 18, max_iter=10, tile_rows=4), q.reshape(-1, 1), q.reshape(-1, 1))
    assert e.value.code == 9
    a = torch.ones((8, 8), dtype=torch.float32, device=dev)
    with pytest.raises(G.UOTError) as e:
        G.solve_noalloc(G.Params(nx=8, ny=8, max_iter=10, flags=G.UOT_AUTOTUNE), a, a)
    assert e.value.code == 1
