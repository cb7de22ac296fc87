"""Benchmark of the UOT prox iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete solve of the workload (setup, the fused iterations,
the device-side convergence checks) from a cold start, with every input
already resident in HBM.  The printed JSON line carries:
  value      pixel-iterations per second over the K timed steps
             (sum over pairs of pixels x iterations actually run)
  roofline   the fused iteration kernel against the 8 TB/s HBM peak:
             algorithmic bytes per pixel-iteration x pixel-iterations per
             launch / the kernel's average launch time, from HIP events on
             the solver's stream around graph-replayed back-to-back launches
             of the launch the step runs (a batch: every pair live).  A
             temporally blocked launch runs several iterations and moves the
             state once, so its fraction can pass 1: it beats the
             one-iteration-per-launch HBM bound.  `traffic` is the HBM bytes
             per launch from the profiler's FETCH_SIZE / WRITE_SIZE counters
             (calibrated on a device copy), or null when they were not taken
             for this workload and the current kernel sources.  `alu` is the
             same launch against the FP32 vector peak (algorithmic flops)
  warm_start time to rel_res <= 1e-4 on held-out 256x256 pairs, cold start
             against the trained network's start (inference included)
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample of
             the same workload: a batch's first 16 pairs at 200 iterations
             each over a process pool, or a fixed number of iterations of a
             single pair on one thread

Workloads (seeded synthetic inputs):
  ragged256 (default) 256 pairs with sides log-uniform in [32, 512] in
            one batched solve, rel_res <= 1e-4 or 20000 iterations per pair
            (batches are packed with rows padded to 256-byte boundaries);
            the tolerance workloads check every 40 iterations (--check-every)
  pair512   one unbalanced 512x512 blob pair, mu = 8, stop at
            rel_res <= 1e-4 or 2000 iterations, adaptive step balance
  balanced64  one balanced 64x64 pair, exactly 500 iterations
  video63   the 63 consecutive frame pairs of a 64-frame 256x256 video,
            prox mode (rho = 1, mu = 2), one batched solve
  sweepN    one NxN pair, exactly 200 iterations (the size sweep)
  uotdf     the run-time study of Algorithm 2 (UOT-DF ADMM, Sec. IV-A):
            ADMM iterations and time per iteration at sides 8..2048
  rpca      the prox-exactness study of Algorithm 3 (RPCA+UOT-DF ADMM,
            Sec. IV-B) on the 64-frame 256x256 video: ADMM iterations to
            1e-4 for 1..30 prox passes per iteration
  copy      a plain 1 GiB device-to-device copy (calibrates the HBM byte
            counters of the profiler and shows the attainable copy rate)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# algorithmic bytes per pixel-iteration of Algorithm 1: each state plane
# read once and written once, constants read once (FP32).  A temporally
# blocked launch runs several iterations of every pixel and moves the state
# once, so its algorithmic bytes are these times its iterations and its HBM
# traffic (the profiler's counters) is a fraction of them.
BYTES = {(0, False): 36, (0, True): 28, (1, False): 56, (1, True): 48, (2, False): 48, (2, True): 40}
# algorithmic FP32 operations per pixel-iteration (an FMA counts 2, rsqrt 1;
# compares and selects not counted): flux step 14, D M 3, residual prox 3,
# the x-steps 5 each, K and the dual step 4-6
FLOPS = {(0, False): 26, (0, True): 22, (1, False): 37, (1, True): 33, (2, False): 32, (2, True): 28}


# Counters of one launch of the fused kernel, from rocprofv3 --pmc passes
# over the graph-replayed timing launches of this script (the last 40
# dispatches, every pair of a batch live): FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch) scaled by what the same counters read for a 1 GiB device copy
# (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000), and the busy fractions of the
# vector ALUs and the LDS, the mean waves per CU and the VALU instructions
# issued.  Valid only for the kernel sources they were taken on: any change
# to them makes every counter figure unknown (null) until they are taken
# again.
TRAFFIC_SOURCES = ("paper_1909_00149_amd/csrc/uot_iter_impl.hpp", "paper_1909_00149_amd/csrc/uot_iter_mode.hip",
                   "paper_1909_00149_amd/csrc/uot_internal.hpp")
TRAFFIC_SHA256 = "c5d50bf0007c344fe1222539097d44a2af3e6d10fa00e059cd2620c80552e5e3"
FETCH_SCALE, WRITE_SCALE = 2.000, 1.000
# workload -> (tile_rows, FETCH_SIZE KiB, WRITE_SIZE KiB, VALUBusy %, LdsUtil %,
#              MeanOccupancyPerCU, SQ_INSTS_VALU, TCC hit rate) per dispatch
COUNTERS = {
    "ragged256": (4016, 180694.073, 231696.375, 63.63, 53.10, 15.26, 67279131, 0.542),
    "pair512": (4008, 2921.378, 4096.000, 17.82, 12.24, 3.10, 1897024, 0.674),
}
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every
# 4 cycles (16 lanes), 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 / 4 * 2.4e9


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_counters(name, shape):
    """The counter record of this workload's launch, or None when it was not
    taken for this kernel shape and the current kernel sources."""
    rec = COUNTERS.get(name)
    if rec is None or rec[0] != shape or kernel_sources_sha256() != TRAFFIC_SHA256:
        return None
    return {"traffic": int(round((rec[1] * FETCH_SCALE + rec[2] * WRITE_SCALE) * 1024)),
            "valu_busy": rec[3] / 100.0, "lds_util": rec[4] / 100.0, "waves_per_cu": rec[5],
            "valu_insts": rec[6], "l2_hit_rate": rec[7]}


def kernel_name(mode, balanced, shape, residual_p=1, norm=0):
    """Instantiated name of the fused kernel for a tile_rows code (the third
    template argument is the boundary code: bit 1 the anisotropic norm)."""
    resid = 0 if balanced else residual_p
    bcn = 2 * norm
    if shape >= 1000:
        return f"cp_iter_tb_kernel<{mode}, {resid}, {bcn}, {shape % 1000}, {shape // 1000}>"
    if shape >= 100:
        return f"cp_iter_vec_kernel<{mode}, {resid}, {bcn}, {shape % 100}, {'true' if shape >= 300 else 'false'}>"
    return f"cp_iter_kernel<{mode}, {resid}, {bcn}, {shape}>"

def workload(name):
    from paper_1909_00149_amd import synth
    if name == "pair512":
        p, q = synth.unbalanced_pair(0, side=512)
        return dict(desc="single unbalanced pair 512x512, 20 blobs, Poisson-noised target, mu=8, "
                         "stop at rel_res<=1e-4 or 2000 iterations",
                    pairs=[(p, q)], mode=0, balanced=False, mu=8.0, rho=1.0, tol=1e-4, max_iter=2000,
                    adaptive=True, check_every=40)
    if name == "pair512p2":
        p, q = synth.unbalanced_pair(0, side=512)
        return dict(desc="single unbalanced pair 512x512, 20 blobs, Poisson-noised target, mu=8, squared "
                         "l2 source term (p=2), stop at rel_res<=1e-4 or 2000 iterations",
                    pairs=[(p, q)], mode=0, balanced=False, mu=8.0, rho=1.0, tol=1e-4, max_iter=2000,
                    adaptive=True, residual_p=2, check_every=40)
    if name == "pair512aniso":
        p, q = synth.unbalanced_pair(0, side=512)
        return dict(desc="single unbalanced pair 512x512, 20 blobs, Poisson-noised target, mu=8, anisotropic "
                         "l1,1 flux norm, stop at rel_res<=1e-4 or 2000 iterations",
                    pairs=[(p, q)], mode=0, balanced=False, mu=8.0, rho=1.0, tol=1e-4, max_iter=2000,
                    adaptive=True, norm=1, check_every=40)
    if name == "balanced64":
        p, q = synth.balanced_pair(0)
        return dict(desc="single balanced pair 64x64, 3 blobs, exactly 500 iterations",
                    pairs=[(p, q)], mode=0, balanced=True, mu=1.0, rho=1.0, tol=0.0, max_iter=500,
                    adaptive=False)
    if name == "ragged256":
        sides, pairs = synth.ragged_batch(0, batch=256)
        return dict(desc="ragged batch of 256 unbalanced pairs, sides log-uniform 32..512, mu=8, "
                         "rel_res<=1e-4 (checked every 40 iterations) or 20000 iterations per pair",
                    pairs=pairs, mode=0, balanced=False, mu=8.0, rho=1.0, tol=1e-4, max_iter=20000,
                    adaptive=True, check_every=40)
    if name == "video63":
        S, _, _ = synth.video_frames(0)
        pairs = [(S[t], S[t + 1]) for t in range(S.shape[0] - 1)]
        return dict(desc="63 frame pairs of a 64-frame 256x256 video, prox mode rho=1 mu=2, "
                         "rel_res<=1e-4 or 2000 iterations",
                    pairs=pairs, mode=1, balanced=False, mu=2.0, rho=1.0, tol=1e-4, max_iter=2000,
                    adaptive=True, check_every=40)
    if name.startswith("sweep"):
        side = int(name[5:])
        p, q = synth.sweep_pair(0, side)
        return dict(desc=f"single unbalanced pair {side}x{side}, exactly 200 iterations",
                    pairs=[(p, q)], mode=0, balanced=False, mu=8.0, rho=1.0, tol=0.0, max_iter=200,
                    adaptive=False)
    raise SystemExit(f"unknown workload {name}")


def _oracle_pair_iters(args):
    """Worker of the batched CPU baseline: `iters` FP64 oracle iterations of
    one pair from zero on one thread; returns the seconds they took."""
    p, q, kw, iters = args
    from threadpoolctl import threadpool_limits
    from oracle import uot as ora
    with threadpool_limits(limits=1):
        prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), **kw)
        t1, t2 = prob.default_steps()
        st = ora.initial_state(prob)
        t0 = time.perf_counter()
        for _ in range(iters):
            st = ora.iterate(prob, st, t1, t2)
        return time.perf_counter() - t0


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "numpy": np.__version__}


def cpu_baseline_batched(W, n_pairs=16, iters=200, repeats=3):
    """The FP64 oracle over the first n_pairs pairs of a batch, one pair per
    process of a pool as wide as the host's cores (at most 16, the GPU machine's
    share), `iters` iterations each from zero; wall clock of the whole pool
    pass, median of `repeats`.  Must run before this process touches the
    GPU (the pool forks it)."""
    import multiprocessing as mp
    pairs = W["pairs"][:n_pairs]
    kw = dict(mode=W["mode"], balanced=W["balanced"], mu=W["mu"], rho=W["rho"],
              residual_p=W.get("residual_p", 1), norm=["iso", "aniso"][W.get("norm", 0)])
    work = [(p, q, kw, iters) for p, q in pairs]
    work.sort(key=lambda a: -a[0].size)  # largest first: the pool's tail is a small pair
    procs = max(1, min(len(work), os.cpu_count() or 1, 16))
    walls = []
    with mp.get_context("fork").Pool(procs) as pool:
        pool.map(_oracle_pair_iters, [(p[:8, :8], q[:8, :8], kw, 2) for p, q, kw, _ in work[:procs]])  # warm the workers
        for _ in range(repeats):
            t0 = time.perf_counter()
            pool.map(_oracle_pair_iters, work, chunksize=1)
            walls.append(time.perf_counter() - t0)
    wall = float(np.median(walls))
    px = sum(int(p.size) for p, _ in pairs)
    info = host_info()
    return {"value": px * iters / wall, "unit": "pixel-iters/s", "cores": procs, "kind": "oracle",
            "sample": f"subset: the first {len(pairs)} of the {len(W['pairs'])} pairs ({px} pixels), {iters} FP64 "
                      f"oracle iterations each from zero, one pair per process of a {procs}-process pool, one "
                      f"thread per process; wall clock of the pass, median of {repeats} ({wall:.2f} s)",
            **info}


def cpu_baseline(W, budget_s=20.0):
    """FP64 oracle on one host thread: as many iterations of the workload's
    first pair (from zero, the workload's own steps) as fit the budget."""
    from threadpoolctl import threadpool_limits
    from oracle import uot as ora
    p, q = W["pairs"][0]
    prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), mode=W["mode"],
                       balanced=W["balanced"], mu=W["mu"], rho=W["rho"], residual_p=W.get("residual_p", 1),
                       norm=["iso", "aniso"][W.get("norm", 0)])
    t1, t2 = prob.default_steps()
    with threadpool_limits(limits=1):
        st = ora.initial_state(prob)
        t0 = time.perf_counter()
        for _ in range(3):
            st = ora.iterate(prob, st, t1, t2)
        per = (time.perf_counter() - t0) / 3
        n = int(max(5, min(100000, budget_s / max(per, 1e-9))))
        t0 = time.perf_counter()
        for _ in range(n):
            st = ora.iterate(prob, st, t1, t2)
        secs = time.perf_counter() - t0
    return {"value": p.size * n / secs, "unit": "pixel-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} FP64 oracle iterations of the first pair ({p.shape[1]}x{p.shape[0]}) from zero, "
                      f"numpy with every thread pool limited to 1 thread, {secs:.1f} s", **host_info()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ragged256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=400)
    ap.add_argument("--check-every", type=int, default=None,
                    help="iterations between convergence checks (default: the workload's)")
    ap.add_argument("--warm-pairs", type=int, default=1000,
                    help="held-out 256x256 pairs for the warm-vs-cold time to 1e-4 (0: skip)")
    ap.add_argument("--prox-iters", default=None,
                    help="rpca, rpca_signed: comma-separated prox passes per ADMM iteration to study (default: all)")
    ap.add_argument("--tau-ratios", default=None,
                    help="rpca: comma-separated tau1/tau2 of the prox passes (default: 1,0.01)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"this benchmark runs on one GPU only (asked for {args.gpus}); the batched solver "
              f"shards by pairs across GPUs, which is not built here", file=sys.stderr)
        sys.exit(2)

    # the batched CPU baseline forks a process pool: it runs before anything
    # in this process touches the GPU
    early_cpu = None
    if not args.no_cpu_baseline and args.workload not in ("uotdf", "rpca", "rpca_signed", "dr512", "copy"):
        W0 = workload(args.workload)
        if len(W0["pairs"]) > 1:
            early_cpu = cpu_baseline_batched(W0)

    import torch
    from paper_1909_00149_amd import uot as G

    dev = torch.device("cuda:0")
    if args.workload == "uotdf":
        run_uotdf(args, dev)
        return
    if args.workload == "rpca":
        run_rpca(args, dev)
        return
    if args.workload == "rpca_signed":
        run_rpca_signed(args, dev)
        return
    if args.workload == "dr512":
        run_dr(args, dev)
        return
    if args.workload == "copy":
        n = (1 << 30) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
        print(json.dumps({"metric": "copy GB/s (read + write)", "value": gbs, "unit": "GB/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                          "higher_is_better": True, "bytes_read_per_copy": n * 4,
                          "bytes_written_per_copy": n * 4}), flush=True)
        return
    W = workload(args.workload)
    pairs = W["pairs"]
    imgs_p = [torch.from_numpy(np.ascontiguousarray(p)).to(dev) for p, _ in pairs]
    imgs_q = [torch.from_numpy(np.ascontiguousarray(q)).to(dev) for _, q in pairs]
    flags = G.UOT_ADAPTIVE_STEPS if W["adaptive"] else 0
    check_every = args.check_every or W.get("check_every", 20)
    batched = len(pairs) > 1
    if batched:
        # every row starts on a 256-byte boundary (one 64-pixel tile row), so
        # no cache line or HBM burst is shared between tiles or pairs; the
        # padding is never touched and not counted
        src, nx, ny, pitch, offs = G.pack_pitched(imgs_p, align=64)
        dst, _, _, _, _ = G.pack_pitched(imgs_q, align=64)
        prm = G.Params(mode=W["mode"], balanced=W["balanced"], mu=W["mu"], rho=W["rho"], tol=W["tol"],
                       max_iter=W["max_iter"], check_every=check_every, flags=flags, residual_p=W.get("residual_p", 1),
                       norm=W.get("norm", 0))
        state = G.new_state(W["mode"], W["balanced"], src.numel(), dev)
    else:
        src, dst = imgs_p[0], imgs_q[0]
        ny0, nx0 = src.shape
        prm = G.Params(nx=nx0, ny=ny0, mode=W["mode"], balanced=W["balanced"], mu=W["mu"], rho=W["rho"],
                       tol=W["tol"], max_iter=W["max_iter"], check_every=check_every, flags=flags,
                       residual_p=W.get("residual_p", 1), norm=W.get("norm", 0))
        state = G.new_state(W["mode"], W["balanced"], src.shape, dev)
    solver = G.Solver(prm)
    npx = [int(p.size) for p, _ in pairs]

    def step():
        if batched:
            _, reps = solver.solve_batched(src, dst, nx, ny, offs, state, pitch=pitch)
        else:
            _, rep = solver.solve(src, dst, state)
            reps = [rep]
        return reps

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pix_iters = 0
    reps = None
    for _ in range(args.steps):
        reps = step()
        pix_iters += sum(n * r["iters"] for n, r in zip(npx, reps))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    value = pix_iters / secs
    its = [int(r["iters"]) for r in reps]

    # fused-kernel timing on the solver's stream, on the launch the step runs
    # (a batch: every pair live; one pair: the pair itself)
    kstate = G.new_state(W["mode"], W["balanced"], src.shape if not batched else src.numel(), dev)
    ksolver = G.Solver(prm)
    if batched:
        ksolver.time_iterations_batched(src, dst, nx, ny, offs, kstate, 20, pitch=pitch)
        ms, shape = ksolver.time_iterations_batched(src, dst, nx, ny, offs, kstate, args.kernel_iters, pitch=pitch)
    else:
        ksolver.time_iterations(src, dst, kstate, 20)
        ms, shape = ksolver.time_iterations(src, dst, kstate, args.kernel_iters)
    bpp = BYTES[(W["mode"], W["balanced"])]
    px_launch = int(sum(npx))
    T = shape // 1000 if shape >= 1000 else 1  # iterations per launch
    secs_launch = ms * 1e-3
    fpp = FLOPS[(W["mode"], W["balanced"])]
    # effective: the per-iteration algorithmic bytes of every iteration the
    # launch runs (the metric's %HBM); a blocked launch can pass 1
    eff = bpp * px_launch * T / secs_launch / 1e9
    # physical: a launch must read and write the state once whatever T is
    once = bpp * px_launch / secs_launch / 1e9
    flops = fpp * px_launch * T / secs_launch / 1e12
    cnt = measured_counters(args.workload, shape)
    hbm_frac = (cnt["traffic"] / secs_launch / 1e9 / HBM_PEAK_GBS) if cnt else once / HBM_PEAK_GBS
    # the bound is the unit the counters show busiest: the vector ALUs
    # (issue) or HBM; without counters the one-iteration kernels are HBM
    # streams and the blocked ones are taken as issue-bound
    if cnt:
        bound = "alu" if cnt["valu_busy"] >= hbm_frac else "hbm"
    else:
        bound = "alu" if T > 1 else "hbm"
    if bound == "alu":
        head = {"bound": "alu", "achieved": round(flops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(flops / FP32_PEAK_TFLOPS, 4)}
    else:
        head = {"bound": "hbm", "achieved": round(once, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(once / HBM_PEAK_GBS, 4)}
    roofline = {**head, "traffic": cnt["traffic"] if cnt else None,
                "kernel": kernel_name(W["mode"], W["balanced"], shape, W.get("residual_p", 1), W.get("norm", 0)),
                "tile_rows": shape, "iterations_per_launch": T, "pixels_per_launch": px_launch,
                "kernel_ms": round(ms, 5), "flops_per_pixel_iter": fpp, "bytes_per_pixel_iter": bpp,
                "effective_hbm": {"achieved": round(eff, 1), "unit": "GB/s", "frac": round(eff / HBM_PEAK_GBS, 4),
                                  "bytes_per_launch": bpp * px_launch * T},
                "physical_hbm": {"achieved": round(cnt["traffic"] / secs_launch / 1e9, 1) if cnt else None,
                                 "unit": "GB/s", "frac": round(hbm_frac, 4) if cnt else None,
                                 "state_bytes_per_launch": bpp * px_launch,
                                 "traffic_vs_state": round(cnt["traffic"] / (bpp * px_launch), 4) if cnt else None},
                "counters": None if cnt is None else {
                    "valu_busy": cnt["valu_busy"], "lds_util": cnt["lds_util"], "waves_per_cu": cnt["waves_per_cu"],
                    "l2_hit_rate": cnt["l2_hit_rate"],
                    "valu_issue_frac": round(cnt["valu_insts"] / secs_launch / VALU_ISSUE_PEAK, 4)}}
    out = {
        "metric": "pixel-iters/s (%HBM peak); time-to-1e-4 residual, warm-start vs cold",
        "value": value,
        "unit": "pixel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * secs / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": W["desc"], "pairs": len(pairs),
                   "pixels": int(sum(npx)), "mode": ["DIST", "PROX", "PROX_FIXED"][W["mode"]],
                   "balanced": W["balanced"], "residual_p": W.get("residual_p", 1),
                   "flux_norm": ["l2,1", "l1,1"][W.get("norm", 0)], "check_every": check_every},
        "effective_hbm_frac_step": round(value * bpp / (HBM_PEAK_GBS * 1e9), 4),
        "tol": W["tol"], "max_iter": W["max_iter"],
        "iters_quantiles": {q: int(np.percentile(its, pq, method="nearest"))
                            for q, pq in (("min", 0), ("p50", 50), ("p90", 90), ("max", 100))},
        "not_converged": int(sum(r["status_name"] != "CONVERGED" for r in reps)) if W["tol"] > 0 else None,
        # the step's wall time counts as time to tol only when every pair met it
        "time_to_tol_ms": (round(1e3 * secs / args.steps, 3)
                           if W["tol"] > 0 and all(r["status_name"] == "CONVERGED" for r in reps) else None),
        "status": sorted({r["status_name"] for r in reps}),
        "max_rel_res": max(float(r["rel_res"]) for r in reps),
        "roofline": roofline,
    }
    if args.warm_pairs > 0:
        out["warm_start"] = warm_vs_cold(dev, args.warm_pairs)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = early_cpu if early_cpu is not None else cpu_baseline(W)
    print(json.dumps(out), flush=True)


UOTDF_SIDES = (8, 16, 32, 64, 128, 256, 512, 1024, 2048)
UOTDF_KW = dict(kappa=0.1, mu=1.0, rho=1.0)


def run_uotdf(args, dev):
    """The run-time study of Algorithm 2 (UOT-DF ADMM): denoising (Phi = I,
    no l1 term) of a synthetic frame at sides 8..2048, one warm-started prox
    pass per ADMM iteration, stop when both residuals are below 1e-3 (tested
    every 10 iterations).  Per side: ADMM iterations to converge and the
    device time per iteration (events around the replayed windows; median of
    the timed steps).  `value` is pixel-ADMM-iterations per second at 512^2."""
    import torch
    from paper_1909_00149_amd import admm as A
    from paper_1909_00149_amd import synth

    rows = []
    for side in UOTDF_SIDES:
        s0, y = synth.df_frame(0, side)
        ty, ts0 = torch.from_numpy(y).to(dev), torch.from_numpy(s0).to(dev)
        solver = A.UotDf(side, side, prox_iters=1, max_iter=5000, check_every=10, eps=1e-3, **UOTDF_KW)
        for _ in range(args.warmup):
            solver.solve(ty, ts0)
        reps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, rep = solver.solve(ty, ts0)
            reps.append(rep)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        it = reps[-1]["iters"]
        ms = float(np.median([r["ms_per_iter"] for r in reps]))
        rows.append({"side": side, "pixels": side * side, "iters": it, "converged": bool(reps[-1]["converged"]),
                     "ms_per_iter": round(ms, 5), "wall_ms": round(1e3 * wall, 3),
                     "us_per_iter_per_kpx": round(1e3 * ms / (side * side / 1e3), 5)})
        solver.close()
    r512 = next(r for r in rows if r["side"] == 512)
    value = 512 * 512 / (r512["ms_per_iter"] * 1e-3)
    # per ADMM iteration at 512^2 inside a check window: the multiplier step
    # fused with the next s/x/centre step streams 11 planes (reads x s z a b
    # y, writes a b s x p), the prox pass 48 bytes per pixel (one-argument-
    # fixed, unbalanced): 92 algorithmic bytes per pixel
    bpp = 92
    achieved = bpp * 512 * 512 / (r512["ms_per_iter"] * 1e-3) / 1e9
    out = {
        "metric": "UOT-DF ADMM pixel-iterations/s at 512^2 (Algorithm 2 run-time study)",
        "value": value, "unit": "pixel-ADMM-iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r512["wall_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uotdf", "description": "denoising, Phi = I, kappa 0.1, mu 1, rho 1, 1 prox pass "
                   "per ADMM iteration (warm-started), eps 1e-3, check every 10"},
        "sizes": rows,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "one ADMM iteration (df_absx_kernel + cp_iter_vec_kernel<2,1,0,16,false>)",
                     "bytes_per_pixel_iter": bpp},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = uotdf_cpu_baseline()
    print(json.dumps(out), flush=True)


def uotdf_cpu_baseline(budget_s=15.0):
    """The FP64 oracle of Algorithm 2 on one host thread, 64x64 frame: ADMM
    iterations (one prox pass each) for about budget_s seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import admm as ora
    from paper_1909_00149_amd import synth
    s0, y = synth.df_frame(0, 64)
    with threadpool_limits(limits=1):
        st = ora.df_initial_state(s0, **UOTDF_KW)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget_s:
            for _ in range(10):
                st = ora.df_iterate(y, s0, st, prox_iters=1, **UOTDF_KW)
            n += 10
        secs = time.perf_counter() - t0
    return {"value": 64 * 64 * n / secs, "unit": "pixel-ADMM-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} FP64 oracle ADMM iterations (one prox pass each) of a 64x64 frame, one thread, "
                      f"{secs:.1f} s"}


RPCA_KW = dict(lam=0.02, gam=8.0, kappa=0.02, mu=2.0, rho=1.0)
RPCA_PROX_ITERS = (1, 2, 3, 5, 10, 30)
RPCA_TAU_RATIOS = (1.0, 0.01)


def run_rpca(args, dev):
    """The prox-exactness study of Algorithm 3 (RPCA+UOT-DF ADMM, Sec. IV-B)
    on the 64-frame 256x256 synthetic video (Phi = I): for each number k of
    warm-started prox passes per ADMM iteration, the ADMM iterations b(k) to
    primal and dual residuals below 1e-4 (tested every 10 iterations) and the
    additional iterations |b(k) - b(30)| / b(30); the device time per ADMM
    iteration; the separation error against the generating S and L.  The
    study runs with equal prox steps and with tau1 / tau2 = 0.01 (the product
    fixed).  `value` is ADMM iterations per second with one prox pass."""
    import torch
    from paper_1909_00149_amd import admm as A
    from paper_1909_00149_amd import synth

    S0, L0, Y = synth.video_frames(0)
    T, ny, nx = Y.shape
    ty = torch.from_numpy(Y).to(dev)
    ks = RPCA_PROX_ITERS if args.prox_iters is None else tuple(int(v) for v in args.prox_iters.split(","))
    ratios = RPCA_TAU_RATIOS if args.tau_ratios is None else tuple(float(v) for v in args.tau_ratios.split(","))
    rows = []
    for ratio in ratios:
        part = []
        for k in ks:
            solver = A.Rpca(nx, ny, T, prox_iters=k, max_iter=5000, check_every=10, eps=1e-4,
                            prox_tau_ratio=ratio, **RPCA_KW)
            if k == 1 and not rows:
                for _ in range(args.warmup):
                    solver.solve(ty)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S, L, rep = solver.solve(ty)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            Sn, Ln = S.double().cpu().numpy(), L.double().cpu().numpy()
            part.append({"tau_ratio": ratio, "prox_iters": k, "admm_iters": rep["iters"],
                         "converged": bool(rep["converged"]), "ms_per_iter": round(rep["ms_per_iter"], 4),
                         "wall_s": round(wall, 3), "jacobi_sweeps_last": rep["jacobi_sweeps"],
                         "rmse_S": round(float(np.sum((Sn - S0) ** 2) / np.sum(S0.astype(np.float64) ** 2)), 5),
                         "rmse_L": round(float(np.sum((Ln - L0) ** 2) / np.sum(L0.astype(np.float64) ** 2)), 5)})
            solver.close()
            print(f"# rpca ratio {ratio} prox_iters {k}: {rep['iters']} ADMM iterations, "
                  f"{rep['ms_per_iter']:.3f} ms each", file=sys.stderr, flush=True)
        b30 = next((r["admm_iters"] for r in part if r["prox_iters"] == 30), None)
        for r in part:
            if b30:
                r["additional_pct"] = round(100.0 * abs(r["admm_iters"] - b30) / b30, 2)
        rows += part
    r1 = rows[0]
    out = {
        "metric": "RPCA+UOT-DF ADMM iterations/s, 64-frame 256^2 video, 1 prox pass (Algorithm 3)",
        "value": 1e3 / r1["ms_per_iter"], "unit": "ADMM-iters/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": r1["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rpca", "description": "64 frames of 256x256 (30 blobs at 0-3 px/frame over a "
                   "rank-3 background, noise 1e-3), Phi = I, lam 0.02, gam 8, kappa 0.02, mu 2, rho 1, "
                   "eps 1e-4, check every 10"},
        "prox_exactness": rows,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = rpca_cpu_baseline()
    print(json.dumps(out), flush=True)


RPCA_SIGNED_KW = dict(lam=0.02, gam=4.0, kappa=0.02, mu=2.0, rho=1.0, prox_tau_ratio=0.01)


def run_rpca_signed(args, dev):
    """The signed RPCA+UOT-DF (eq. RPCA_UOTDF_PN) at the size of the paper's
    video experiment (60 frames of 95x160) on a synthetic video whose
    foreground is lighter and darker than the background: ADMM iterations to
    1e-4 (checked every 10), device time per iteration and the separation
    error, with Phi = I and with a random half of the pixels observed (a
    diagonal stand-in for the paper's dense random projections, which this
    build does not support), for 1, 3 and 10 prox passes.  `value` is ADMM
    iterations per second with Phi = I and 3 prox passes."""
    import torch
    from paper_1909_00149_amd import admm as A
    from paper_1909_00149_amd import synth

    S0, L0, Y = synth.video_frames_signed(0)
    T, ny, nx = Y.shape
    rng = np.random.default_rng(1)
    mask = (rng.uniform(0, 1, Y.shape) < 0.5).astype(np.float32)
    ty = torch.from_numpy(Y).to(dev)
    tym = torch.from_numpy(Y * mask).to(dev)
    tmask = torch.from_numpy(mask).to(dev)
    ks = (1, 3, 10) if args.prox_iters is None else tuple(int(v) for v in args.prox_iters.split(","))
    rows = []
    for phi_name, yy, phi in (("identity", ty, None), ("half the pixels", tym, tmask)):
        for k in ks:
            solver = A.Rpca(nx, ny, T, prox_iters=k, max_iter=5000, check_every=10, eps=1e-4, signed=True,
                            **RPCA_SIGNED_KW)
            if not rows:
                for _ in range(args.warmup):
                    solver.solve(yy, phi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S, L, rep = solver.solve(yy, phi)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            Sn, Ln = S.double().cpu().numpy(), L.double().cpu().numpy()
            rows.append({"phi": phi_name, "prox_iters": k, "admm_iters": rep["iters"],
                         "converged": bool(rep["converged"]), "ms_per_iter": round(rep["ms_per_iter"], 4),
                         "wall_s": round(wall, 3),
                         "rmse_S": round(float(np.sum((Sn - S0) ** 2) / np.sum(S0.astype(np.float64) ** 2)), 5),
                         "rmse_L": round(float(np.sum((Ln - L0) ** 2) / np.sum(L0.astype(np.float64) ** 2)), 5),
                         "dark_recall": round(float(np.mean(Sn[S0 < -0.1] < -0.05)), 4)})
            solver.close()
            print(f"# rpca_signed phi {phi_name} prox_iters {k}: {rep['iters']} ADMM iterations, "
                  f"{rep['ms_per_iter']:.3f} ms each", file=sys.stderr, flush=True)
    head = next((r for r in rows if r["phi"] == "identity" and r["prox_iters"] == 3), rows[0])
    out = {
        "metric": "signed RPCA+UOT-DF ADMM iterations/s, 60 frames of 95x160 (eq. RPCA_UOTDF_PN)",
        "value": 1e3 / head["ms_per_iter"], "unit": "ADMM-iters/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": head["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rpca_signed", "description": "60 frames of 95x160, 12 blobs of either sign "
                   "(amplitude 0.3-0.8, 0-2 px/frame) over a rank-3 background, noise 1e-3; lam 0.02, gam 4, "
                   "kappa 0.02, mu 2, rho 1, prox tau1/tau2 0.01, eps 1e-4, check every 10"},
        "study": rows,
    }
    print(json.dumps(out), flush=True)


DR_GAMMAS = (1e-5, 1e-4, 1e-3)


def run_dr(args, dev):
    """The Douglas-Rachford splitting (uot_dr_solve: separable prox, then the
    exact projection onto the divergence constraint by the DCT Poisson
    solve) on the 512x512 unbalanced pair of the default workload, for a
    fixed budget of iterations at several DR steps gamma; the objective it
    reaches is compared with Algorithm 1's certified value on the same pair.
    `value` is DR pixel-iterations per second at the best gamma."""
    import torch
    from paper_1909_00149_amd import uot as G

    W = workload("pair512")
    p, q = W["pairs"][0]
    ny, nx = p.shape
    tp, tq = torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev)
    cp = G.Solver(G.Params(nx=nx, ny=ny, mode=0, mu=W["mu"], tol=1e-6, max_iter=20000, check_every=20,
                           flags=G.UOT_ADAPTIVE_STEPS))
    _, crep = cp.solve(tp, tq)
    vstar = crep["primal"]
    iters = 1000 if args.kernel_iters == 400 else args.kernel_iters
    rows = []
    for gam in DR_GAMMAS:
        s = G.Solver(G.Params(nx=nx, ny=ny, mode=0, mu=W["mu"], max_iter=iters, check_every=50, tol=0.0))
        for _ in range(args.warmup):
            s.dr_solve(tp, tq, gamma=gam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = s.dr_solve(tp, tq, gamma=gam)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        rows.append({"gamma": gam, "iters": rep["iters"], "ms_per_iter": round(rep["ms_per_iter"], 4),
                     "wall_s": round(wall, 4), "fixed_point_res": rep["fixed_point_res"],
                     "objective": rep["objective"], "infeasibility": rep["infeasibility"],
                     "rel_to_cp_value": (rep["objective"] - vstar) / vstar})
        print(f"# dr gamma {gam}: {rep['ms_per_iter']:.4f} ms/iter, objective {rep['objective']:.6g} "
              f"(cp {vstar:.6g}), infeasibility {rep['infeasibility']:.3g}", file=sys.stderr, flush=True)
    best = min(rows, key=lambda r: abs(r["rel_to_cp_value"]) + r["infeasibility"] / max(vstar, 1e-30))
    out = {
        "metric": "Douglas-Rachford pixel-iters/s, 512^2 unbalanced pair (DCT projection)",
        "value": nx * ny / (best["ms_per_iter"] * 1e-3), "unit": "pixel-iters/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": best["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "dr512", "description": f"the pair512 problem (DIST, mu 8) by Douglas-Rachford, "
                   f"{iters} iterations per gamma, w from zero; Algorithm 1's value to rel_res 1e-6 for reference"},
        "cp_value": vstar, "cp_iters": crep["iters"], "study": rows,
    }
    print(json.dumps(out), flush=True)


def rpca_cpu_baseline(budget_s=15.0):
    """The FP64 oracle of Algorithm 3 on one host thread: ADMM iterations
    (one prox pass each) of the first 8 frames of the video cropped to
    64x64, for about budget_s seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import admm as ora
    from paper_1909_00149_amd import synth
    _, _, Y = synth.video_frames(0)
    Y = Y[:8, :64, :64].astype(np.float64)
    with threadpool_limits(limits=1):
        st = ora.rpca_initial_state(Y.shape, RPCA_KW["kappa"], RPCA_KW["mu"], RPCA_KW["rho"])
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget_s:
            st = ora.rpca_iterate(Y, st, prox_iters=1, **RPCA_KW)
            n += 1
        secs = time.perf_counter() - t0
    return {"value": n / secs, "unit": "ADMM-iters/s (8 frames of 64x64)", "cores": 1, "kind": "oracle",
            "sample": f"{n} FP64 oracle ADMM iterations of 8 frames of 64x64 (the video cropped), one thread, "
                      f"{secs:.1f} s"}


def warm_vs_cold(dev, n):
    """Time to rel_res <= 1e-4 on n held-out 256x256 pairs, one batched solve
    per arm (best of 3): cold start vs the trained network's start
    (inference included)."""
    from paper_1909_00149_amd import warmstart as WS
    path = os.path.join(ROOT, "paper_1909_00149_amd", "data", "warmstart_256.npz")
    pairs = [WS._pair(s) for s in range(WS.EVAL_SEED0, WS.EVAL_SEED0 + n)]
    src = np.stack([p for p, _ in pairs])
    dst = np.stack([q for _, q in pairs])
    net = WS.load_net(path, dev, batch_max=64)  # inference in chunks of 64 pairs
    res = WS.evaluate(net, src, dst, dev, arms=("cold", "learned"), repeats=3)
    c, l = res["cold"], res["learned"]
    cp, lp = np.array(c["primal"]), np.array(l["primal"])
    return {"pairs": n, "side": WS.SIDE, "tol": 1e-4,
            "cold_ms": round(1e3 * c["wall_s"], 3), "learned_ms": round(1e3 * l["wall_s"], 3),
            "learned_start_ms": round(1e3 * l["start_s"], 3),
            "cold_iters_median": c["iters_median"], "learned_iters_median": l["iters_median"],
            "converged": [c["converged"], l["converged"]], "learned_fell_back": l["fallback"],
            "rel_gap_mean": [round(c["rel_gap_mean"], 5), round(l["rel_gap_mean"], 5)],
            "learned_primal_above_cold_mean": float(np.mean((lp - cp) / cp)),
            "speedup": round(c["wall_s"] / l["wall_s"], 3)}


if __name__ == "__main__":
    main()
