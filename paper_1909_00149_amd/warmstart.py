"""Learned warm start: solver-generated training data, training, evaluation.

    python -m paper_1909_00149_amd.warmstart --train 20000 --eval 1000 --epochs 20 \
        --out paper_1909_00149_amd/data/warmstart_256.npz

Pairs follow the 256x256 unbalanced blob recipe (centres at least 24 px
from the edge); training seeds 0..n-1, held-out seeds from 1,000,000.
Targets are the solver's own iterates (flux and dual) at rel_res <= 1e-5
(adaptive steps, capped iterations).  The network sees (in_scale p,
in_scale q) and predicts (s_flux Mx, s_flux My, s_dual a); the start it
gives is completed to a feasible one (r = D M + q - p) by the kernels.

Evaluation solves the held-out pairs in batched calls per arm to
rel_res <= 1e-4: cold (zeros), Poisson-flux start, learned start.  The
reported wall time of an arm includes building its start.  The learned
arm falls back to the cold start pair by pair: a pair whose start holds a
non-finite value starts from zeros (UOT_WARM_FALLBACK), and a pair whose
rel_res after the first check window (PROBE iterations) is worse than the
cold start's after the same iterations is restarted from zeros; the cold
solver's stopping rule decides convergence in every arm.  Each arm reports
the certified primal and dual bounds at stop and their relative gap.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import torch

from . import net as N
from . import synth
from . import uot as G

SIDE = 256
MU = 8.0
NPX = SIDE * SIDE
IN_SCALE = NPX / 16.0
S_FLUX = NPX / 8.0
S_DUAL = 1.0 / MU
CH = (32, 64, 128, 128)
EVAL_SEED0 = 1_000_000
PROBE = 20  # iterations of the first check window, where the learned start is compared with the cold one


def _pair(seed):
    return synth.unbalanced_pair(int(seed), side=SIDE, margin=24.0)


def gen_pairs(seeds, workers=None):
    """Seeded pairs as two float32 arrays (n, SIDE, SIDE)."""
    workers = workers or min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        out = list(ex.map(_pair, seeds, chunksize=64))
    return np.stack([p for p, _ in out]), np.stack([q for _, q in out])


def solve_targets(src, dst, dev, chunk=512, tol=1e-5, max_iter=40000, log=print):
    """Solver iterates (Mx, My, a) for every pair: device tensors (n*NPX,)."""
    n = src.shape[0]
    out = {k: torch.empty(n * NPX, dtype=torch.float32, device=dev) for k in ("Mx", "My", "a")}
    iters = []
    s = G.Solver(G.Params(mu=MU, tol=tol, max_iter=max_iter, check_every=20, flags=G.UOT_ADAPTIVE_STEPS))
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        B = c1 - c0
        S = torch.from_numpy(src[c0:c1].reshape(-1)).to(dev)
        D = torch.from_numpy(dst[c0:c1].reshape(-1)).to(dev)
        t = time.perf_counter()
        st, reps = s.solve_batched(S, D, [SIDE] * B, [SIDE] * B, [b * NPX for b in range(B)])
        torch.cuda.synchronize()
        for k in out:
            out[k][c0 * NPX:c1 * NPX].copy_(st[k])
        iters += [r["iters"] for r in reps]
        log(f"targets {c1}/{n}: {time.perf_counter() - t:.2f} s, median iters {int(np.median(iters[-B:]))}, "
            f"converged {sum(r['status'] == 0 for r in reps)}/{B}")
    return out, np.array(iters)


def train(net, src, dst, tgt, dev, epochs=4, batch=16, lr=1e-3, lr_min=2e-5, log=print):
    """Adam with cosine decay over all steps; shuffles pairs every epoch."""
    n = src.shape[0]
    S = torch.from_numpy(src.reshape(-1)).to(dev)
    D = torch.from_numpy(dst.reshape(-1)).to(dev)
    steps = epochs * (n // batch)
    rng = np.random.default_rng(0)
    k = 0
    hist = []
    bs = torch.empty(batch * NPX, dtype=torch.float32, device=dev)
    bd, bx, by, ba = (torch.empty_like(bs) for _ in range(4))
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(n)
        losses = []
        for i in range(n // batch):
            idx = torch.from_numpy(perm[i * batch:(i + 1) * batch]).to(dev)
            rows = (idx[:, None] * NPX + torch.arange(NPX, device=dev)[None, :]).reshape(-1)
            torch.index_select(S, 0, rows, out=bs)
            torch.index_select(D, 0, rows, out=bd)
            torch.index_select(tgt["Mx"], 0, rows, out=bx)
            torch.index_select(tgt["My"], 0, rows, out=by)
            torch.index_select(tgt["a"], 0, rows, out=ba)
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * k / max(1, steps)))
            losses.append(net.train_step(bs, bd, bx, by, ba, IN_SCALE, S_FLUX, S_DUAL, cur))
            k += 1
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.5f} (last batch {losses[-1]:.5f}), "
            f"{time.perf_counter() - t0:.1f} s")
    return hist, time.perf_counter() - t0


def _stats(reps, extra_iters=None):
    it = np.array([r["iters"] for r in reps]) + (0 if extra_iters is None else extra_iters)
    primal = np.array([r["primal"] for r in reps])
    dual = np.array([r["dual"] for r in reps])
    gap = np.array([r["rel_gap"] for r in reps])
    return {"iters_median": float(np.median(it)), "iters_p90": float(np.percentile(it, 90)),
            "iters_mean": float(it.mean()), "converged": int(sum(r["status"] == 0 for r in reps)),
            "pairs": len(reps), "primal_mean": float(primal.mean()), "dual_mean": float(dual.mean()),
            "rel_gap_mean": float(gap.mean()), "rel_gap_max": float(gap.max()),
            "primal": primal.tolist(), "dual": dual.tolist()}


def evaluate(net, src, dst, dev, tol=1e-4, max_iter=20000, arms=("cold", "poisson", "learned"), repeats=1):
    """Batched solve of all pairs per arm; returns per-arm statistics (the
    per-pair certified bounds included)."""
    n = src.shape[0]
    S = torch.from_numpy(src.reshape(-1)).to(dev)
    D = torch.from_numpy(dst.reshape(-1)).to(dev)
    nx = [SIDE] * n
    offs = [b * NPX for b in range(n)]
    prm = dict(mu=MU, check_every=20)
    res = {}
    for arm in arms:
        best = None
        for _ in range(repeats):
            st = G.new_state(G.DIST, False, n * NPX, dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fallback = 0
            if arm == "cold":
                s = G.Solver(G.Params(tol=tol, max_iter=max_iter, flags=G.UOT_ADAPTIVE_STEPS, **prm))
                _, reps = s.solve_batched(S, D, nx, nx, offs, st)
                t_start, pre = 0.0, None
            elif arm == "poisson":
                s = G.Solver(G.Params(tol=tol, max_iter=max_iter, flags=G.UOT_ADAPTIVE_STEPS | G.UOT_WARM_START, **prm))
                s.init_poisson(S, D, st, nx=nx, ny=nx, offset=offs)
                t_start = time.perf_counter() - t0
                _, reps = s.solve_batched(S, D, nx, nx, offs, st)
                pre = None
            else:
                for c0 in range(0, n, net.batch_max):
                    c1 = min(n, c0 + net.batch_max)
                    sub = {k: v[c0 * NPX:c1 * NPX] for k, v in st.items()}
                    net.warm_state(S[c0 * NPX:c1 * NPX], D[c0 * NPX:c1 * NPX], sub, IN_SCALE, S_FLUX, S_DUAL)
                t_start = time.perf_counter() - t0
                # the first window from the learned start (non-finite starts
                # begin from zeros) and from the cold start
                warm = G.Solver(G.Params(tol=0.0, max_iter=PROBE,
                                         flags=G.UOT_WARM_START | G.UOT_WARM_FALLBACK, **prm))
                _, r1 = warm.solve_batched(S, D, nx, nx, offs, st)
                cst = G.new_state(G.DIST, False, n * NPX, dev)
                _, rc = G.Solver(G.Params(tol=0.0, max_iter=PROBE, **prm)).solve_batched(S, D, nx, nx, offs, cst)
                del cst
                lose = [b for b in range(n)
                        if r1[b]["cold_start"] or not np.isfinite(r1[b]["rel_res"]) or r1[b]["rel_res"] > rc[b]["rel_res"]]
                fallback = len(lose)
                if lose:  # those pairs restart from zeros (a zero-iteration cold solve writes them)
                    G.Solver(G.Params(tol=0.0, max_iter=0, **prm)).solve_batched(
                        S, D, [SIDE] * len(lose), [SIDE] * len(lose), [offs[b] for b in lose], st)
                s = G.Solver(G.Params(tol=tol, max_iter=max_iter - PROBE,
                                      flags=G.UOT_ADAPTIVE_STEPS | G.UOT_WARM_START, **prm))
                _, reps = s.solve_batched(S, D, nx, nx, offs, st)
                pre = np.full(n, PROBE)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if best is None or wall < best[0]:
                best = (wall, t_start, reps, pre, fallback)
        wall, t_start, reps, pre, fallback = best
        res[arm] = {"wall_s": wall, "start_s": t_start, "fallback": fallback, **_stats(reps, pre)}
    return res


def save_params(net, path):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=net.get_params(), ch=np.array(CH), side=SIDE, in_scale=IN_SCALE, s_flux=S_FLUX,
             s_dual=S_DUAL, mu=MU)


def load_net(path, dev, batch_max=16):
    z = np.load(path, allow_pickle=False)
    net = N.WarmStartNet(int(z["side"]), int(z["side"]), ch=tuple(int(c) for c in z["ch"]), batch_max=batch_max)
    net.set_params(z["params"])
    return net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--eval", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--target-iters", type=int, default=40000)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "data", "warmstart_256.npz"))
    ap.add_argument("--report", default=None)
    ap.add_argument("--load", default=None, help="skip training, evaluate saved parameters")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)  # noqa: E731
    report = {"config": vars(args)}
    # every input is drawn by worker processes before this process touches the GPU
    t = time.perf_counter()
    esrc, edst = gen_pairs(range(EVAL_SEED0, EVAL_SEED0 + args.eval))
    if not args.load:
        src, dst = gen_pairs(range(args.train))
    log(f"generated {args.eval} held-out and {0 if args.load else args.train} training pairs in "
        f"{time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    if args.load:
        net = load_net(args.load, dev, args.batch)
    else:
        t = time.perf_counter()
        tgt, iters = solve_targets(src, dst, dev, max_iter=args.target_iters, log=log)
        report["targets"] = {"seconds": time.perf_counter() - t, "iters_median": float(np.median(iters)),
                             "iters_max": int(iters.max()), "tol": 1e-5, "cap": args.target_iters,
                             "rms_Mx": float(tgt["Mx"].float().pow(2).mean().sqrt()) * S_FLUX,
                             "rms_a": float(tgt["a"].float().pow(2).mean().sqrt()) * S_DUAL}
        log(json.dumps(report["targets"]))
        net = N.WarmStartNet(SIDE, SIDE, ch=CH, batch_max=args.batch, seed=0)
        hist, secs = train(net, src, dst, tgt, dev, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
        report["train"] = {"loss": hist, "seconds": secs,
                           "samples_per_s": args.epochs * (args.train // args.batch) * args.batch / secs}
        save_params(net, args.out)
        del tgt, src, dst
        torch.cuda.empty_cache()
    report["eval"] = evaluate(net, esrc, edst, dev)
    log(json.dumps({arm: {k: v for k, v in r.items() if k not in ("primal", "dual")}
                    for arm, r in report["eval"].items()}))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
