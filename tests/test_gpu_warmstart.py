"""What the trained warm-start network gains over the method without it, on
held-out pairs (seeds never used in training), and the fallback path."""
import json
import os

import numpy as np
import pytest
import torch

from paper_1909_00149_amd import net as N
from paper_1909_00149_amd import uot as G
from paper_1909_00149_amd import warmstart as WS

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(WS.__file__), "data", "warmstart_256.npz")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "converged_values.json")


def certified_heldout():
    """Oracle-certified optimal values of held-out pairs: {seed: (dual, primal)}."""
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    return {c["seed"]: (c["dual"], c["primal"]) for c in cases
            if c["name"].startswith("heldout") and c["side"] == WS.SIDE and c["mu"] == WS.MU}


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def heldout(n, first=WS.EVAL_SEED0 + 5000):
    pairs = [WS._pair(s) for s in range(first, first + n)]
    return np.stack([p for p, _ in pairs]), np.stack([q for _, q in pairs])


def test_learned_start_beats_cold_start(dev):
    net = WS.load_net(WEIGHTS, dev, batch_max=16)
    src, dst = heldout(32)
    res = WS.evaluate(net, src, dst, dev, arms=("cold", "learned"))
    cold, learned = res["cold"], res["learned"]
    assert cold["converged"] == 32 and learned["converged"] == 32, res
    assert learned["iters_median"] <= 0.8 * cold["iters_median"], res
    # both arms reach the same optimal values (the stopping rule decides)
    assert abs(learned["primal_mean"] - cold["primal_mean"]) <= 1e-3 * cold["primal_mean"], res
    # and on the pairs whose optimum the FP64 oracle certified, each arm's
    # certified primal bound lies above the oracle's lower bound and within
    # 1e-3 relative of the optimum: the learned start converges to the
    # problem's solution, not merely to a small residual
    cert = certified_heldout()
    first = WS.EVAL_SEED0 + 5000
    assert len(cert) >= 2
    for seed, (lo, hi) in cert.items():
        i = seed - first
        assert 0 <= i < 32
        vstar = 0.5 * (lo + hi)
        for arm in (cold, learned):
            pr = arm["primal"][i]
            assert pr >= lo * (1 - 1e-5), (seed, pr, lo, hi)
            assert pr - vstar <= 1e-3 * vstar, (seed, pr, lo, hi)
        print(seed, "optimum", vstar, "cold", cold["primal"][i], "learned", learned["primal"][i])


def test_rejected_start_falls_back_to_cold(dev):
    """A network producing non-finite values gives a start the solver
    rejects; every pair of the learned arm falls back to the cold start and
    converges."""
    net = WS.load_net(WEIGHTS, dev, batch_max=16)
    bad = net.get_params()
    bad[:] = np.nan
    net.set_params(bad)
    src, dst = heldout(4, first=WS.EVAL_SEED0 + 9000)
    res = WS.evaluate(net, src, dst, dev, arms=("learned",))
    assert res["learned"]["converged"] == 4 and res["learned"]["fallback"] == 4
    # and the warm solve by itself reports the rejection
    S = torch.from_numpy(src.reshape(-1)).to(dev)
    D = torch.from_numpy(dst.reshape(-1)).to(dev)
    st = G.new_state(G.DIST, False, S.numel(), dev)
    net.warm_state(S, D, st, WS.IN_SCALE, WS.S_FLUX, WS.S_DUAL)
    s = G.Solver(G.Params(mu=WS.MU, tol=1e-4, max_iter=100, flags=G.UOT_WARM_START))
    with pytest.raises(G.UOTError) as e:
        s.solve_batched(S, D, [WS.SIDE] * 4, [WS.SIDE] * 4, [b * WS.NPX for b in range(4)], st)
    assert e.value.code == 4


def test_warm_fallback_per_pair(dev):
    """UOT_WARM_FALLBACK: in a batch whose second pair's warm state holds a
    NaN, that pair starts from zeros (cold_start in its report, iterates
    bitwise those of a cold solve) while the others start from their warm
    states (bitwise those of their own warm solves)."""
    src, dst = heldout(3, first=WS.EVAL_SEED0 + 9100)
    n = WS.NPX
    S = torch.from_numpy(src.reshape(-1)).to(dev)
    D = torch.from_numpy(dst.reshape(-1)).to(dev)
    rng = np.random.default_rng(5)
    warm = {k: torch.from_numpy((rng.standard_normal(3 * n) * 1e-4).astype(np.float32)).to(dev)
            for k in ("Mx", "My", "r", "a")}
    warm["a"].mul_(1e3)
    bad = {k: v.clone() for k, v in warm.items()}
    bad["a"][n + 17] = float("nan")
    sides, offs = [WS.SIDE] * 3, [0, n, 2 * n]
    kw = dict(mu=WS.MU, tol=1e-4, max_iter=400, check_every=20)
    st, reps = G.Solver(G.Params(flags=G.UOT_WARM_START | G.UOT_WARM_FALLBACK, **kw)).solve_batched(
        S, D, sides, sides, offs, {k: v.clone() for k, v in bad.items()})
    assert [r["cold_start"] for r in reps] == [0, 1, 0]
    cold, rc = G.Solver(G.Params(**kw)).solve_batched(S, D, sides, sides, offs)
    ref, rw = G.Solver(G.Params(flags=G.UOT_WARM_START, **kw)).solve_batched(
        S, D, sides, sides, offs, {k: v.clone() for k, v in warm.items()})
    torch.cuda.synchronize()
    for k in ("Mx", "My", "r", "a"):
        assert torch.equal(st[k][n:2 * n], cold[k][n:2 * n]), k
        assert torch.equal(st[k][:n], ref[k][:n]) and torch.equal(st[k][2 * n:], ref[k][2 * n:]), k
    assert reps[1]["iters"] == rc[1]["iters"] and reps[0]["iters"] == rw[0]["iters"]
