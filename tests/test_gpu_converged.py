"""Converged GPU solutions against results the mathematics fixes.

The flux of the Beckmann problem is unique in two families of instances,
and there it is compared element by element (FP32 GPU against the exact
flux, max-abs error <= 1e-4 with unit-scale masses):

  * the balanced problem on a line (an n x 1 or 1 x n grid, zero-flux
    boundary; eq. OT_beckman with the divergence of Sec. II-A): the
    constraint alone fixes the flux, M = cumsum(p - q), and the value is
    sum |cumsum(p - q)| (the 1-D Wasserstein-1 distance);
  * two point masses m1, m2 a distance d < 2 mu apart along one grid axis
    (eq. Unbal_OT_beckman): min(m1, m2) travels the straight path, the
    excess |m1 - m2| is created or destroyed in place, and the value is
    d min(m1, m2) + mu |m1 - m2|.

Elsewhere only the optimal value is unique; the 512 x 512 unbalanced
workload and a 128 x 128 cut-down are compared with values the FP64 oracle
certified by its primal and dual bounds (tests/golden/converged_values.json,
written by tests/golden/make_converged.py).
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1909_00149_amd import synth
from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "converged_values.json")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def line_pair(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, n) * (rng.uniform(0, 1, n) < 0.4)
    q = rng.uniform(0, 1, n) * (rng.uniform(0, 1, n) < 0.4)
    p = (p / p.sum()).astype(np.float32)
    q = (q / q.sum() * p.astype(np.float64).sum()).astype(np.float32)
    return p, q


@pytest.mark.parametrize("n,seed,axis", [(64, 1, "x"), (64, 1, "y"), (96, 2, "x"), (96, 2, "y")])
def test_line_flux_at_convergence(dev, n, seed, axis):
    """Balanced pair on a line, solved to rel_res <= 1e-6: the flux equals
    cumsum(p - q) to 1e-4 and the certified value sum |cumsum(p - q)| to
    1e-5 relative."""
    p, q = line_pair(n, seed)
    shape = (1, n) if axis == "x" else (n, 1)
    P, Q = p.reshape(shape), q.reshape(shape)
    ny, nx = shape
    s = G.Solver(G.Params(nx=nx, ny=ny, balanced=True, max_iter=400000, check_every=20, tol=1e-6,
                          flags=G.UOT_ADAPTIVE_STEPS))
    st, rep = s.solve(to_dev(P, dev), to_dev(Q, dev))
    torch.cuda.synchronize()
    assert rep["status_name"] == "CONVERGED", rep
    flux = np.cumsum(p.astype(np.float64) - q.astype(np.float64))
    M = (st["Mx"] if axis == "x" else st["My"]).double().cpu().numpy().reshape(-1)
    other = (st["My"] if axis == "x" else st["Mx"]).double().cpu().numpy()
    assert np.abs(flux).max() > 0.05  # the transport is not trivial
    err = float(np.abs(M - flux).max())
    assert err <= 1e-4, err
    assert float(np.abs(other).max()) == 0.0  # no flux across the zero-flux edge
    value = float(np.abs(flux[:-1]).sum())
    assert abs(rep["primal"] - value) <= 1e-5 * value, (rep["primal"], value)
    assert rep["dual"] <= value * (1 + 1e-5)


def point_pair(ny, nx, u, v, m1, m2):
    p = np.zeros((ny, nx), np.float32)
    q = np.zeros((ny, nx), np.float32)
    p[u[1], u[0]] = m1
    q[v[1], v[0]] = m2
    return p, q


# (grid, source pixel (x, y), target pixel, masses, mu, iterations): the
# FP64 iteration's flux error on these instances falls to 5e-5 only after
# 2.5e5-1e6 iterations (the primal iterate of the method converges slowly
# where the optimum is a degenerate vertex), so they run a fixed count
POINT_CASES = [
    ((8, 12), (2, 4), (6, 4), 1.0, 0.6, 3.5, 500000),
    ((8, 12), (5, 1), (5, 6), 0.7, 1.0, 3.5, 1000000),
    ((12, 20), (3, 3), (12, 3), 1.0, 0.8, 3.5, 2000),   # d = 9 > 2 mu: no transport
]


@pytest.mark.parametrize("case", range(len(POINT_CASES)))
def test_point_mass_flux(dev, case):
    (ny, nx), u, v, m1, m2, mu, iters = POINT_CASES[case]
    p, q = point_pair(ny, nx, u, v, m1, m2)
    s = G.Solver(G.Params(nx=nx, ny=ny, mu=mu, max_iter=iters, check_every=20, tol=1e-12,
                          flags=G.UOT_ADAPTIVE_STEPS))
    st, rep = s.solve(to_dev(p, dev), to_dev(q, dev))
    torch.cuda.synchronize()
    d = abs(u[0] - v[0]) + abs(u[1] - v[1])
    Mx = np.zeros((ny, nx))
    My = np.zeros((ny, nx))
    m = min(m1, m2)
    if d < 2 * mu:
        if u[1] == v[1]:
            Mx[u[1], u[0]:v[0]] = m
        else:
            My[u[1]:v[1], u[0]] = m
    # r = D M - p + q: the excess appears at the heavier end
    r = -p.astype(np.float64) + q.astype(np.float64)
    if d < 2 * mu:
        r[u[1], u[0]] += m
        r[v[1], v[0]] -= m
    value = min(d, 2 * mu) * m + mu * abs(m1 - m2)
    for k, want in (("Mx", Mx), ("My", My), ("r", r)):
        err = float(np.abs(st[k].double().cpu().numpy() - want).max())
        assert err <= 1e-4, (k, err)
    assert abs(rep["primal"] - value) <= 1e-5 * value, (rep["primal"], value)
    assert rep["dual"] <= value * (1 + 1e-5)


def golden_cases():
    if not os.path.exists(GOLDEN):
        return []
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: c["name"])
def test_unbalanced_blob_value_at_convergence(dev, case):
    """The seeded blob pair solved on the GPU to rel_res <= 1e-6 (adaptive
    steps): its certified primal bound equals the value the oracle certified
    (the midpoint of its [dual, primal] interval) to 1e-5 relative plus the
    interval's half-width, and the GPU's certified interval overlaps the
    oracle's up to 1e-5.  The oracle's interval is 1.4e-6 wide at 128^2
    (4e5 FP64 iterations), 6e-6 and 1.2e-5 wide on the two held-out 256^2
    pairs of the learned-start evaluation (2.5e5 iterations) and 1.75e-5
    wide at 512^2 (3e5 iterations, 99 minutes on one core): there the value
    is pinned to about 2e-5."""
    side = case["side"]
    p, q = synth.unbalanced_pair(case["seed"], side=side, nblobs=case["blobs"], margin=min(24.0, side / 4))
    s = G.Solver(G.Params(nx=side, ny=side, mu=case["mu"], max_iter=600000, check_every=20, tol=1e-6,
                          flags=G.UOT_ADAPTIVE_STEPS))
    st, rep = s.solve(to_dev(p, dev), to_dev(q, dev))
    torch.cuda.synchronize()
    print(case["name"], {k: rep[k] for k in ("iters", "status_name", "rel_res", "primal", "dual", "objective")})
    assert rep["status_name"] == "CONVERGED", {k: rep[k] for k in ("iters", "rel_res", "primal", "dual")}
    lo, hi = case["dual"], case["primal"]
    assert 0.0 <= hi - lo <= abs(case["rel_gap"]) * hi * (1 + 1e-9)
    vstar = 0.5 * (lo + hi)
    slack = 1e-5 * vstar + 0.5 * (hi - lo)
    assert abs(rep["primal"] - vstar) <= slack, (rep["primal"], lo, hi)
    assert rep["dual"] <= hi + 1e-5 * vstar and rep["primal"] >= lo - 1e-5 * vstar
    # the flux moved: the value is carried by transport, not only by r
    assert float(st["Mx"].abs().max()) > 0.0
