"""Host-side parts of bench.py that need no GPU: the workload definitions,
the counter table and its source digest, the refusal of several GPUs, and
the CPU baseline's arithmetic on a tiny sample."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_default_workload_is_the_ragged_batch():
    W = bench.workload("ragged256")
    sides = [p.shape[0] for p, _ in W["pairs"]]
    assert len(W["pairs"]) == 256 and min(sides) >= 32 and max(sides) <= 512
    assert all(p.shape[0] == p.shape[1] for p, _ in W["pairs"])
    assert W["tol"] == 1e-4 and W["max_iter"] == 20000 and W["adaptive"] and W["check_every"] == 40
    assert W["mode"] == 0 and not W["balanced"] and W["mu"] == 8.0


def test_counters_belong_to_the_committed_kernels():
    """The counter table was taken on the kernel sources as committed: a
    change to them must come with counters taken again (the bench reports
    no traffic meanwhile)."""
    assert bench.kernel_sources_sha256() == bench.TRAFFIC_SHA256
    for wl, rec in bench.COUNTERS.items():
        c = bench.measured_counters(wl, rec[0])
        assert c is not None and c["traffic"] > 0 and 0.0 < c["valu_busy"] <= 1.0
        assert bench.measured_counters(wl, rec[0] + 1) is None  # another shape: no counters
    # the traffic of one launch covers at least one read and one write of the state
    W = bench.workload("ragged256")
    npx = sum(p.size for p, _ in W["pairs"])
    state = bench.BYTES[(0, False)] * npx
    assert bench.measured_counters("ragged256", 4016)["traffic"] >= state


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout.strip() == ""


def test_cpu_baseline_worker_and_host_info():
    """The batched CPU baseline's worker times the oracle's iterations of
    one pair on one thread; the host description is plain JSON."""
    rng = np.random.default_rng(2)
    p = rng.uniform(0, 1, (12, 9)).astype(np.float32)
    q = rng.uniform(0, 1, (12, 9)).astype(np.float32)
    kw = dict(mode=0, balanced=False, mu=8.0)
    assert bench._oracle_pair_iters((p, q, kw, 5)) > 0.0
    info = json.loads(json.dumps(bench.host_info()))
    assert info["cpu_count"] >= 1 and "numpy" in info
