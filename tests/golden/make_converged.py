"""Writes converged_values.json: the optimal value of seeded unbalanced
blob pairs (the 512 x 512 workload and its 128 x 128 cut-down) certified by
the FP64 oracle's primal and dual bounds.  Calls only the oracle and the
seeded input generator; run from the repository root:
    python tests/golden/make_converged.py
Each case stores the certified interval [dual, primal] that contains the
optimal value; its width is the recorded rel_gap.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import uot as ora  # noqa: E402
from paper_1909_00149_amd import synth  # noqa: E402

# (name, seed, side, blobs, mu): the 512^2 pair and a 128^2 cut-down with
# the blob density of the 512^2 recipe scaled up to keep it non-trivial
CASES = [("pair128", 7, 128, 6, 8.0), ("pair512", 0, 512, 20, 8.0),
         # two held-out pairs of the learned-start evaluation (256^2 recipe)
         ("heldout256a", 1005000, 256, 20, 8.0), ("heldout256b", 1005001, 256, 20, 8.0)]


def main(names=None, max_iter=300000, gap_tol=1e-10, out=None):
    path = out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "converged_values.json")
    old = {}
    if os.path.exists(path):
        with open(path) as f:
            old = {c["name"]: c for c in json.load(f)["cases"]}
    for name, seed, side, nb, mu in CASES:
        if names and name not in names:
            continue
        p, q = synth.unbalanced_pair(seed, side=side, nblobs=nb, margin=min(24.0, side / 4))
        prob = ora.Problem(p.astype(np.float64), q.astype(np.float64), mu=mu)
        t0 = time.time()
        st, rep = ora.solve(prob, max_iter=max_iter, check_every=50, tol=1e-14, adaptive=True,
                            gap_tol=gap_tol, gap_every=1000)
        g = ora.certified_gap(prob, st)
        old[name] = dict(name=name, seed=seed, side=side, blobs=nb, mu=mu, primal=g.primal, dual=g.dual,
                         rel_gap=g.rel_gap, iters=rep.iters, rel_res=rep.rel_res,
                         seconds=round(time.time() - t0, 1))
        print(old[name], flush=True)
        with open(path, "w") as f:
            json.dump({"source": "oracle.uot.solve (FP64, adaptive steps) and oracle.uot.certified_gap; "
                                 "inputs from paper_1909_00149_amd.synth.unbalanced_pair",
                       "cases": [old[k] for k in sorted(old)]}, f, indent=1)


if __name__ == "__main__":
    # python tests/golden/make_converged.py [names...] [--out file.json] [--iters N]
    argv = sys.argv[1:]
    kw = {}
    for flag, key, conv in (("--out", "out", str), ("--iters", "max_iter", int)):
        if flag in argv:
            i = argv.index(flag)
            kw[key] = conv(argv[i + 1])
            del argv[i:i + 2]
    main(argv or None, **kw)
