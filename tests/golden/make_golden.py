"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

Usage: python tests/golden/make_golden.py [medium]
Each record names the instance (generator preset and seed), the oracle options, and
the oracle's objective and KKT residuals at a tight tolerance.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_10891_amd import scuc  # noqa: E402


def record(preset, seed, tol):
    _, lp = scuc.make_instance(preset, seed)
    t = time.time()
    r = oracle.solve(lp, oracle.Options(tol=tol, max_iter=2_000_000))
    ev = oracle.kkt(lp, r.x, r.y, r.z)
    return dict(preset=preset, seed=seed, m=lp.m, n=lp.n, nnz=lp.nnz, tol=tol, term=r.term,
                iters=r.iters, restarts=r.restarts, pobj=r.pobj, dobj=r.dobj,
                rel_kkt=ev["rel_kkt"], seconds=round(time.time() - t, 1),
                source="oracle.solve (CPU FP64)")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "medium"
    out = os.path.join(HERE, f"oracle_{which}_seed0.json")
    rec = record(which, 0, 1e-8)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
