"""Ragged batches through uot_solve_batched: each pair of a batch must come
out exactly as if it had been solved alone (the per-pixel arithmetic and
the per-pair reductions do not depend on the neighbours in the batch), and
match the FP64 oracle to the iterate tolerance."""
import numpy as np
import pytest
import torch

from oracle import uot as ora
from oracle.ops import DIST, PROX
from paper_1909_00149_amd import synth
from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu

SHAPES = [(1, 77), (60, 1), (2, 2), (29, 37), (64, 64), (33, 100), (9, 130), (200, 5), (70, 70)]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def inputs(shape, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = (rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.5)).astype(np.float32) * scale
    q = (rng.uniform(0, 1, shape) * (rng.uniform(0, 1, shape) < 0.5)).astype(np.float32) * scale
    p[0, 0] += 0.25 * scale
    q[-1, -1] += 0.25 * scale
    return p.astype(np.float32), q.astype(np.float32)


def batch_of(shapes, dev, seed0=0, order=None, gap=0, scale=1.0):
    pairs = [inputs(s, seed0 + i, scale) for i, s in enumerate(shapes)]
    order = list(range(len(shapes))) if order is None else order
    nx = [s[1] for s in shapes]
    ny = [s[0] for s in shapes]
    offs = [0] * len(shapes)
    o = 0
    for i in order:  # pack in a chosen order with optional gaps between pairs
        offs[i] = o
        o += nx[i] * ny[i] + gap
    src = np.zeros(o, np.float32)
    dst = np.zeros(o, np.float32)
    for i, (p, q) in enumerate(pairs):
        src[offs[i]:offs[i] + p.size] = p.reshape(-1)
        dst[offs[i]:offs[i] + q.size] = q.reshape(-1)
    return pairs, torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev), nx, ny, offs


def single(dev, p, q, **kw):
    ny, nx = p.shape
    s = G.Solver(G.Params(nx=nx, ny=ny, **kw))
    st, rep = s.solve(torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev))
    torch.cuda.synchronize()
    return st, rep


def planes(mode, balanced):
    return G.required_planes(mode, balanced)


@pytest.mark.parametrize("mode,balanced", [(DIST, False), (PROX, False), (DIST, True)])
@pytest.mark.parametrize("tol", [0.0, 1e-3])
def test_batch_equals_single_solves_bitwise(dev, mode, balanced, tol):
    pairs, src, dst, nx, ny, offs = batch_of(SHAPES, dev, seed0=10, order=list(range(len(SHAPES)))[::-1], gap=13)
    if balanced:
        pairs = [(p, (q * (p.astype(np.float64).sum() / q.astype(np.float64).sum())).astype(np.float32))
                 for p, q in pairs]
        d = dst.cpu().numpy()
        for i, (p, q) in enumerate(pairs):
            d[offs[i]:offs[i] + q.size] = q.reshape(-1)
        dst = torch.from_numpy(d).to(dev)
    kw = dict(mode=mode, balanced=balanced, mu=1.1, rho=0.8, max_iter=300, check_every=10, tol=tol,
              tile_rows=8, flags=G.UOT_ADAPTIVE_STEPS if tol > 0 else 0)
    s = G.Solver(G.Params(**kw))
    st, reps = s.solve_batched(src, dst, nx, ny, offs)
    torch.cuda.synchronize()
    for i, (p, q) in enumerate(pairs):
        one, rep = single(dev, p, q, **kw)
        assert reps[i]["iters"] == rep["iters"] and reps[i]["status"] == rep["status"], (i, reps[i], rep)
        n = p.size
        for k in planes(mode, balanced):
            got = st[k][offs[i]:offs[i] + n].view(p.shape)
            assert torch.equal(got, one[k]), (i, k)
        assert reps[i]["rel_res"] == rep["rel_res"]


def test_batch_matches_oracle(dev):
    shapes = [(17, 45), (64, 3), (40, 40)]
    pairs, src, dst, nx, ny, offs = batch_of(shapes, dev, seed0=40)
    s = G.Solver(G.Params(mode=PROX, mu=1.3, rho=0.7, max_iter=120))
    st, reps = s.solve_batched(src, dst, nx, ny, offs)
    torch.cuda.synchronize()
    for i, (p, q) in enumerate(pairs):
        prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), mode=PROX, mu=1.3, rho=0.7)
        t1, t2 = prob.default_steps()
        ref, _ = ora.solve(prob, tau1=np.float32(t1), tau2=np.float32(t2), max_iter=120, tol=0)
        for k in planes(PROX, False):
            g = st[k][offs[i]:offs[i] + p.size].double().cpu().numpy().reshape(p.shape)
            o = getattr(ref, k)
            assert np.abs(g - o).max() <= 1e-4 * max(1.0, np.abs(o).max()), (i, k)
        assert abs(reps[i]["tau1"] - np.float32(t1)) <= 1e-7


def test_pairs_stop_independently(dev):
    """An easy pair (identical images) stops at its first check; a hard one
    keeps going; the easy pair's state is left at its own stopping point."""
    p, q = inputs((48, 48), 3)
    shapes = [(48, 48), (48, 48)]
    src = torch.from_numpy(np.concatenate([p.reshape(-1), p.reshape(-1)])).to(dev)
    dst = torch.from_numpy(np.concatenate([p.reshape(-1), q.reshape(-1)])).to(dev)
    s = G.Solver(G.Params(mu=1.1, max_iter=400, check_every=20, tol=1e-6))
    st, reps = s.solve_batched(src, dst, [48, 48], [48, 48], [0, 48 * 48])
    torch.cuda.synchronize()
    assert reps[0]["status_name"] == "CONVERGED" and reps[0]["iters"] == 20
    assert reps[1]["iters"] == 400
    assert float(st["Mx"][:48 * 48].abs().max()) == 0.0


def test_batch_errors(dev):
    pairs, src, dst, nx, ny, offs = batch_of([(8, 8), (8, 8)], dev)
    s = G.Solver(G.Params(mu=1.0, max_iter=10))
    with pytest.raises(G.UOTError) as e:
        s.solve_batched(src, dst, nx, ny, [0, 10])  # overlapping ranges
    assert e.value.code == 2
    with pytest.raises(G.UOTError) as e:
        s.solve_batched(src, dst, [8, 0], ny, offs)
    assert e.value.code == 2
    bad = src.clone()
    bad[70] = float("nan")
    with pytest.raises(G.UOTError) as e:
        s.solve_batched(bad, dst, nx, ny, offs)
    assert e.value.code == 4


def test_video_pairs_prox_batch(dev):
    """Consecutive frame pairs of a small synthetic video as one PROX batch,
    against the oracle pair by pair."""
    S, _, _ = synth.video_frames(1, frames=6, side=48, nblobs=6)
    imgs_p = [torch.from_numpy(S[t].copy()).to(dev) for t in range(5)]
    imgs_q = [torch.from_numpy(S[t + 1].copy()).to(dev) for t in range(5)]
    src, nx, ny, offs = G.pack(imgs_p)
    dst, _, _, _ = G.pack(imgs_q)
    s = G.Solver(G.Params(mode=PROX, mu=2.0, rho=1.0, max_iter=100))
    st, reps = s.solve_batched(src, dst, nx, ny, offs)
    torch.cuda.synchronize()
    for t in range(5):
        prob = ora.Problem(S[t].astype(np.float64), S[t + 1].astype(np.float64), mode=PROX, mu=2.0, rho=1.0)
        t1, t2 = prob.default_steps()
        ref, _ = ora.solve(prob, tau1=np.float32(t1), tau2=np.float32(t2), max_iter=100, tol=0)
        for k in ("x0", "x1", "a", "Mx"):
            g = st[k][offs[t]:offs[t] + 48 * 48].double().cpu().numpy().reshape(48, 48)
            o = getattr(ref, k)
            assert np.abs(g - o).max() <= 1e-4 * max(1.0, np.abs(o).max()), (t, k)


def test_autotuner_picks_a_shape_and_keeps_results(dev, tmp_path, monkeypatch):
    """With the autotune flag the first solve of a size class times every
    tile shape; results stay bitwise equal to a fixed-shape solve and the
    table is written to the cache file."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("UOT_AUTOTUNE_CACHE", str(cache))
    pairs, src, dst, nx, ny, offs = batch_of([(100, 300), (257, 129), (64, 64)], dev, seed0=70)
    kw = dict(mu=1.2, max_iter=60)
    s = G.Solver(G.Params(flags=G.UOT_AUTOTUNE, **kw))
    st, _ = s.solve_batched(src, dst, nx, ny, offs)
    ref = G.Solver(G.Params(tile_rows=4, **kw))
    st2, _ = ref.solve_batched(src, dst, nx, ny, offs)
    torch.cuda.synchronize()
    for k in ("Mx", "My", "r", "a"):
        assert torch.equal(st[k], st2[k])
    text = cache.read_text()
    assert "gfx950:m0:r1:b0" in text


@pytest.mark.parametrize("ty", [116, 316, 4016])
def test_vectorised_kernel_on_odd_offsets_with_nan_gaps(dev, ty):
    """Pairs packed at offsets that are not multiples of 4, with NaN in the
    gaps between them (images and state): the vectorised kernel must agree
    bitwise with the scalar one on every pair, never read a gap into a
    result, and leave the gaps untouched (61 iterations: the odd tail is
    copied back too)."""
    pairs, src, dst, nx, ny, offs = batch_of(SHAPES, dev, seed0=40, gap=3)
    gaps = torch.ones(src.numel(), dtype=torch.bool, device=dev)
    for i in range(len(nx)):
        gaps[offs[i]:offs[i] + nx[i] * ny[i]] = False
    assert any(o % 4 for o in offs) and bool(gaps.any())
    src[gaps] = float("nan")
    dst[gaps] = float("nan")
    kw = dict(mode=DIST, balanced=False, mu=1.5, max_iter=61, tol=0.0)

    def run(t):
        st = G.new_state(DIST, False, src.numel(), dev)
        for v in st.values():
            v[gaps] = float("nan")
        st, reps = G.Solver(G.Params(tile_rows=t, **kw)).solve_batched(src, dst, nx, ny, offs, st)
        torch.cuda.synchronize()
        return st, reps

    ref, _ = run(4)
    st, reps = run(ty)
    assert all(r["tile_rows"] == ty and r["iters"] == 61 for r in reps)
    for k in ("Mx", "My", "r", "a"):
        assert torch.equal(ref[k][~gaps], st[k][~gaps]), k
        assert bool(torch.isfinite(st[k][~gaps]).all()), k
        assert bool(torch.isnan(st[k][gaps]).all()), k


@pytest.mark.parametrize("max_groups", [0, 8])
@pytest.mark.parametrize("mode,tol", [(DIST, 2e-4), (PROX, 1e-7)])
def test_fused_check_agrees_with_the_separate_check(dev, mode, tol, max_groups):
    """A blocked shape evaluates each window's check inside the window's
    last launch, accumulating over a workgroup's run of tiles of one pair;
    a single-step shape runs the separate check kernel per tile.  On a
    ragged batch (runs of tiles that change pair, pairs smaller than a tile,
    one pair of many tiles) both take the same decisions at the same
    checks: equal iteration counts and statuses, the recorded residuals
    equal up to the order of the FP64 sums, and bitwise equal iterates.
    With max_groups = 8 every workgroup walks long runs of tiles (the
    persistent walk and the per-run accumulation of the fused check)."""
    shapes = SHAPES + [(300, 257)]
    pairs, src, dst, nx, ny, offs = batch_of(shapes, dev, seed0=40)
    out = []
    for ty in (4016, 16):
        s = G.Solver(G.Params(mode=mode, mu=1.1, rho=0.8, max_iter=600, check_every=20, tol=tol, tile_rows=ty,
                              flags=G.UOT_RECORD_HISTORY, max_groups=max_groups))
        st, reps = s.solve_batched(src, dst, nx, ny, offs)
        torch.cuda.synchronize()
        hist = [s.history(b) for b in range(len(shapes))]
        out.append((st, reps, hist))
        assert all(r["tile_rows"] == ty for r in reps)
    (sa, ra, ha), (sb, rb, hb) = out
    assert len({r["iters"] for r in ra}) > 1, "the pairs should stop at different checks"
    for b in range(len(shapes)):
        assert ra[b]["iters"] == rb[b]["iters"] and ra[b]["status"] == rb[b]["status"], b
        assert list(ha[b][0]) == list(hb[b][0]), b
        np.testing.assert_allclose(ha[b][1], hb[b][1], rtol=1e-9, atol=0)
    for k in planes(mode, False):
        assert torch.equal(sa[k], sb[k]), k


@pytest.mark.parametrize("mode,bc,norm,p", [(G.PROX_FIXED, 0, G.NORM_ISO, 1), (DIST, 1, G.NORM_ISO, 1),
                                             (DIST, 0, G.NORM_ANISO, 1), (PROX, 1, G.NORM_ISO, 2),
                                             (G.PROX_FIXED, 1, G.NORM_ANISO, 2)])
def test_fused_check_agrees_on_every_variant(dev, mode, bc, norm, p):
    """The fused check forms the stationarity residual from partial terms of
    the last step and the new dual's gradient, and the feasibility residual
    from the last step's K(z); the separate check kernel forms both from the
    two stored iterates.  On the one-argument-fixed mode, the free edges
    (bc = 1), the anisotropic norm and the squared source term, with a capped
    grid (long runs of tiles per workgroup), both give the same residual at
    every check (up to the order of the FP64 sums), the same decisions and
    bitwise equal iterates."""
    shapes = SHAPES + [(300, 257)]
    pairs, src, dst, nx, ny, offs = batch_of(shapes, dev, seed0=90)
    out = []
    for ty in (4016, 16):
        s = G.Solver(G.Params(mode=mode, bc=bc, norm=norm, residual_p=p, mu=1.1, rho=0.8, max_iter=400,
                              check_every=20, tol=1e-6, tile_rows=ty, flags=G.UOT_RECORD_HISTORY, max_groups=8))
        st, reps = s.solve_batched(src, dst, nx, ny, offs)
        torch.cuda.synchronize()
        out.append((st, reps, [s.history(b) for b in range(len(shapes))]))
        assert all(r["tile_rows"] == ty for r in reps)
    (sa, ra, ha), (sb, rb, hb) = out
    for b in range(len(shapes)):
        assert ra[b]["iters"] == rb[b]["iters"] and ra[b]["status"] == rb[b]["status"], b
        assert len(ha[b][0]) >= 1 and list(ha[b][0]) == list(hb[b][0]), b
        assert np.all(np.isfinite(ha[b][1])) and np.all(ha[b][1] > 0), b
        np.testing.assert_allclose(ha[b][1], hb[b][1], rtol=1e-9, atol=0)
    for k in planes(mode, False):
        assert torch.equal(sa[k], sb[k]), k


@pytest.mark.parametrize("ty", [4016, 4004, 116, 8])
def test_capped_grid_walks_the_tile_list(dev, ty):
    """max_groups = 8 gives each workgroup tens of tiles of several pairs
    (the persistent XCD-chunked walk, and for the blocked shape the fused
    check accumulated over runs of tiles of one pair).  Against the
    uncapped grid: the same decisions at the same checks and bitwise equal
    iterates.  Against the FP64 oracle, pair by pair on non-normalised
    inputs with a tolerance that stops pairs at different checks: the
    iterate after the GPU's iteration count matches element by element, and
    the oracle stops at the same check (or a neighbouring one, where the
    residual crosses tol within FP32 rounding)."""
    shapes = [(40, 70), (9, 130), (64, 64), (3, 5), (100, 33), (70, 70), (1, 90), (50, 1)]
    pairs, src, dst, nx, ny, offs = batch_of(shapes, dev, seed0=70, order=[3, 0, 5, 1, 7, 2, 6, 4], gap=5)
    tol, ce = 2e-4, 20
    runs = []
    for cap in (0, 8):
        s = G.Solver(G.Params(mode=DIST, mu=1.1, max_iter=3000, check_every=ce, tol=tol, tile_rows=ty,
                              max_groups=cap))
        st, reps = s.solve_batched(src, dst, nx, ny, offs)
        torch.cuda.synchronize()
        runs.append((st, reps))
    (s0, r0), (s8, r8) = runs
    rows = ty % 1000 if ty >= 1000 else ty % 100
    tiles = sum(-(-h // rows) * -(-w // 64) for h, w in shapes)
    assert tiles > 8 * 4, "every workgroup should walk several tiles"
    for b in range(len(shapes)):
        assert r0[b]["iters"] == r8[b]["iters"] and r0[b]["status"] == r8[b]["status"], b
        assert abs(r0[b]["rel_res"] - r8[b]["rel_res"]) <= 1e-9 * r0[b]["rel_res"], b
    for k in planes(DIST, False):
        assert torch.equal(s0[k], s8[k]), k
    assert len({r["iters"] for r in r8}) > 1, "the pairs should stop at different checks"
    for b, (p, q) in enumerate(pairs):
        if p.size > 5000:
            continue  # the oracle runs of the small pairs suffice
        prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), mu=1.1)
        t1, t2 = prob.default_steps()
        ref, _ = ora.solve(prob, tau1=np.float32(t1), tau2=np.float32(t2), max_iter=r8[b]["iters"], tol=0)
        o = offs[b]
        for k in planes(DIST, False):
            g = s8[k][o:o + p.size].double().cpu().numpy().reshape(p.shape)
            want = getattr(ref, k)
            assert np.abs(g - want).max() <= 1e-4 * max(1.0, np.abs(want).max()), (b, k)
        if r8[b]["status_name"] == "CONVERGED":
            _, orep = ora.solve(prob, tau1=np.float32(t1), tau2=np.float32(t2), max_iter=3000, tol=tol,
                                check_every=ce)
            assert abs(orep.iters - r8[b]["iters"]) <= ce, b
