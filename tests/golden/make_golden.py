"""Writes lp_values.json: anisotropic Beckmann values of small seeded
instances from the two LP routes of ``oracle.lp`` (HiGHS).  Calls only the
oracle and the seeded input generator; run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lp  # noqa: E402


def instance(seed, ny, nx):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, (ny, nx)) * (rng.uniform(0, 1, (ny, nx)) < 0.35)
    q = rng.uniform(0, 1, (ny, nx)) * (rng.uniform(0, 1, (ny, nx)) < 0.35)
    p[0, 0] += 0.1
    q[-1, -1] += 0.1
    return p, q


def main():
    out = []
    for seed, (ny, nx) in [(11, (6, 6)), (12, (5, 8)), (13, (8, 3)), (14, (7, 7))]:
        p, q = instance(seed, ny, nx)
        for mu in (0.8, 2.5):
            for bc in (0, 1):
                row = dict(seed=seed, ny=ny, nx=nx, mu=mu, bc=bc, balanced=False,
                           beckmann=lp.beckmann_aniso(p, q, mu, bc, False))
                if bc == 0:
                    row["kantorovich"] = lp.kantorovich(p, q, mu, False, lp.manhattan_cost(nx, ny))
                out.append(row)
        qb = q * (p.sum() / q.sum())
        for bc in (0, 1):
            row = dict(seed=seed, ny=ny, nx=nx, mu=None, bc=bc, balanced=True,
                       beckmann=lp.beckmann_aniso(p, qb, None, bc, True))
            if bc == 0:
                row["kantorovich"] = lp.kantorovich(p, qb, None, True, lp.manhattan_cost(nx, ny))
            out.append(row)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lp_values.json")
    with open(path, "w") as f:
        json.dump({"source": "oracle.lp (scipy HiGHS); instances from make_golden.instance",
                   "cases": out}, f, indent=1)
    print("wrote", path, len(out))


if __name__ == "__main__":
    main()
