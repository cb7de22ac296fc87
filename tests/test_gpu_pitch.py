"""Row-pitched layouts (uot_solve_batched_pitched, uot_init_poisson_pitched,
uot_params.pitch): the pitch only moves where a pixel lives, so every pair
must come out bit for bit as in the back-to-back layout, with every tile
shape, and the padding between rows (NaN here) must be neither read into a
result nor written."""
import numpy as np
import pytest
import torch

from oracle.ops import DIST, PROX, PROX_FIXED
from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu

SHAPES = [(1, 77), (60, 1), (2, 2), (29, 37), (64, 64), (33, 100), (9, 130), (70, 70), (17, 65)]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def pairs_of(shapes, seed0, balanced=False):
    out = []
    for i, s in enumerate(shapes):
        rng = np.random.default_rng(seed0 + i)
        p = (rng.uniform(0, 1, s) * (rng.uniform(0, 1, s) < 0.5)).astype(np.float32)
        q = (rng.uniform(0, 1, s) * (rng.uniform(0, 1, s) < 0.5)).astype(np.float32)
        p[0, 0] += 0.25
        q[-1, -1] += 0.25
        if balanced:
            q = (q * np.float32(p.astype(np.float64).sum() / q.astype(np.float64).sum())).astype(np.float32)
        out.append((p, q))
    return out


def pitched(images, pitch_of, dev, fill=float("nan")):
    """Packs with pitch_of(nx) per pair and one padding element between
    pairs; returns (flat, nx, ny, pitch, offsets, padding mask)."""
    nx = [im.shape[1] for im in images]
    ny = [im.shape[0] for im in images]
    pitch = [pitch_of(a) for a in nx]
    offs, o = [], 0
    for pt, b in zip(pitch, ny):
        o = -(-o // 4) * 4 if pt % 4 == 0 else o + 1
        offs.append(o)
        o += pt * b
    flat = torch.full((o,), fill, dtype=torch.float32)
    pad = torch.ones(o, dtype=torch.bool)
    for im, pt, b, off in zip(images, pitch, ny, offs):
        flat[off:off + pt * b].view(b, pt)[:, :im.shape[1]] = torch.from_numpy(im)
        pad[off:off + pt * b].view(b, pt)[:, :im.shape[1]] = False
    return flat.to(dev), nx, ny, pitch, offs, pad.to(dev)


def by_pair(planes, nx, ny, pitch, offs):
    return [{k: v[o:o + pt * b].view(b, pt)[:, :a] for k, v in planes.items()}
            for a, b, pt, o in zip(nx, ny, pitch, offs)]


def solve_layout(dev, pairs, pitch_of, mode, balanced, ty, iters, tol=0.0, **kw):
    src, nx, ny, pitch, offs, pad = pitched([p for p, _ in pairs], pitch_of, dev)
    dst, _, _, _, _, _ = pitched([q for _, q in pairs], pitch_of, dev)
    st = G.new_state(mode, balanced, src.numel(), dev)
    for v in st.values():
        v[pad] = float("nan")
    prm = G.Params(mode=mode, balanced=balanced, mu=1.5, rho=0.7, max_iter=iters, tol=tol, tile_rows=ty, **kw)
    st, reps = G.Solver(prm).solve_batched(src, dst, nx, ny, offs, st, pitch=pitch)
    torch.cuda.synchronize()
    for k, v in st.items():
        assert bool(torch.isnan(v[pad]).all()), f"padding of {k} was written"
    return by_pair(st, nx, ny, pitch, offs), reps


@pytest.mark.parametrize("ty", [4, 16, 116, 316, 4032])
@pytest.mark.parametrize("mode,balanced", [(DIST, False), (PROX, False), (PROX_FIXED, True)])
def test_pitched_batch_equals_packed_batch_bitwise(dev, ty, mode, balanced):
    pairs = pairs_of(SHAPES, 100)
    ref, rref = solve_layout(dev, pairs, lambda a: a, mode, balanced, ty, 41)
    for pitch_of in (lambda a: -(-a // 4) * 4, lambda a: -(-a // 16) * 16, lambda a: a + 3):
        got, rgot = solve_layout(dev, pairs, pitch_of, mode, balanced, ty, 41)
        for b, (x, y) in enumerate(zip(ref, got)):
            for k in x:
                assert torch.equal(x[k], y[k]), (b, k)
        for x, y in zip(rref, rgot):
            assert x["iters"] == y["iters"] == 41
            for f in ("rel_res", "objective", "feas"):
                assert x[f] == y[f], f


def test_pitched_balanced_gap_and_stopping_match(dev):
    """Balanced DIST: the certified gap uses the Poisson feasibility repair,
    which reads the pitched state; tol > 0 exercises the device-side stop."""
    pairs = pairs_of(SHAPES[3:7], 200, balanced=True)
    kw = dict(check_every=10, tol=2e-2, flags=G.UOT_ADAPTIVE_STEPS)
    ref, rref = solve_layout(dev, pairs, lambda a: a, DIST, True, 116, 300, **kw)
    got, rgot = solve_layout(dev, pairs, lambda a: -(-a // 4) * 4, DIST, True, 116, 300, **kw)
    for x, y in zip(rref, rgot):
        for f in ("iters", "status", "rel_res", "primal", "dual", "rel_gap"):
            assert x[f] == y[f] or (np.isnan(x[f]) and np.isnan(y[f])), f
    for x, y in zip(ref, got):
        for k in x:
            assert torch.equal(x[k], y[k]), k


def test_single_grid_pitch_param(dev):
    p, q = pairs_of([(37, 53)], 300)[0]
    ny, nx = p.shape
    kw = dict(nx=nx, ny=ny, mode=DIST, mu=1.5, max_iter=40, tol=0.0, tile_rows=116)
    ref, rep_ref = G.Solver(G.Params(**kw)).solve(torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev))
    P = torch.full((ny, 56), float("nan"), device=dev)
    Q = torch.full((ny, 56), float("nan"), device=dev)
    P[:, :nx] = torch.from_numpy(p).to(dev)
    Q[:, :nx] = torch.from_numpy(q).to(dev)
    st = G.new_state(DIST, False, (ny, 56), dev)
    st, rep = G.Solver(G.Params(pitch=56, **kw)).solve(P, Q, st)
    torch.cuda.synchronize()
    assert rep["tile_rows"] == 116
    for k in ref:
        assert torch.equal(ref[k], st[k][:, :nx]), k
        assert bool((st[k][:, nx:] == 0).all()), k  # zeroed planes: padding untouched
    assert rep["objective"] == rep_ref["objective"]


def test_pitched_poisson_start_equals_packed(dev):
    pairs = pairs_of(SHAPES[3:8], 400)
    out = []
    for pitch_of in (lambda a: a, lambda a: -(-a // 4) * 4 + 4):
        src, nx, ny, pitch, offs, pad = pitched([p for p, _ in pairs], pitch_of, dev, fill=0.0)
        dst, _, _, _, _, _ = pitched([q for _, q in pairs], pitch_of, dev, fill=0.0)
        s = G.Solver(G.Params(mode=DIST, mu=2.0))
        st = G.new_state(DIST, False, src.numel(), dev)
        st = s.init_poisson(src, dst, st, nx=nx, ny=ny, offset=offs, pitch=pitch)
        torch.cuda.synchronize()
        out.append(by_pair(st, nx, ny, pitch, offs))
    for x, y in zip(*out):
        for k in x:
            assert torch.equal(x[k], y[k]), k


def test_pitch_validation(dev):
    src = torch.zeros(1000, device=dev)
    s = G.Solver(G.Params(mode=DIST, mu=1.0))
    with pytest.raises(G.UOTError):  # pitch below nx
        s.solve_batched(src, src, [10], [10], [0], pitch=[9])
    with pytest.raises(G.UOTError):  # second pair starts inside the first's last row span
        s.solve_batched(src, src, [10, 10], [10, 10], [0, 9 * 12 + 5], pitch=[12, 12])
    assert G.check_params(G.Params(nx=10, ny=10, pitch=9)) != 0
    assert G.check_params(G.Params(nx=10, ny=10, pitch=12)) == 0


def test_pitched_timing_matches_solve(dev):
    pairs = pairs_of(SHAPES, 500)
    src, nx, ny, pitch, offs, pad = pitched([p for p, _ in pairs], lambda a: -(-a // 4) * 4, dev, fill=0.0)
    dst, _, _, _, _, _ = pitched([q for _, q in pairs], lambda a: -(-a // 4) * 4, dev, fill=0.0)
    kw = dict(mode=DIST, mu=2.0, tile_rows=316)
    ref, _ = G.Solver(G.Params(max_iter=8, tol=0.0, **kw)).solve_batched(src, dst, nx, ny, offs, pitch=pitch)
    st = G.new_state(DIST, False, src.numel(), dev)
    ms, ran = G.Solver(G.Params(**kw)).time_iterations_batched(src, dst, nx, ny, offs, st, 4, pitch=pitch)
    torch.cuda.synchronize()
    assert ran == 316 and ms > 0
    for k in ref:
        assert torch.equal(ref[k], st[k]), k


def test_wide_pitch_runs_the_single_step_kernel(dev):
    """Row pitches above 2^24 pixels: the blocked kernels address a region
    by 32-bit byte offsets, so the solver runs the single-step kernel of the
    same rows instead, and the iterates equal those of the blocked kernel on
    the packed layout bit for bit."""
    pairs = pairs_of([(3, 100), (2, 70)], 300)
    wide = (1 << 24) + 64
    st, reps = solve_layout(dev, pairs, lambda a: wide, DIST, False, 4016, 30)
    ref, rr = solve_layout(dev, pairs, lambda a: a, DIST, False, 4016, 30)
    assert all(r["tile_rows"] < 1000 for r in reps), [r["tile_rows"] for r in reps]
    assert all(r["tile_rows"] == 4016 for r in rr)
    for a, b in zip(st, ref):
        for k in a:
            assert torch.equal(a[k], b[k]), k
