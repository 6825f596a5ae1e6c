"""Writes the Algorithm 1 fixings of the reduced-LP batches under tests/golden/ from solved
relaxations, without the GPU path.

Usage: python tests/golden/make_fixing_masks.py mixed|medium [first last]

Member i of a batch has parent seed 100 + i and a target share 0.2 + 0.7 i / 63 of its u
variables fixed; its parent is the 2,000-bus preset ("medium") or size class i mod 5 of the
mixed parents (30 to 1,000 buses). For each member the parent's LP relaxation is solved by the
oracle (FP64, rel_kkt 1e-4), and Algorithm 1 (the oracle's) is run on the relaxed binaries for
every tau of a grid; the member keeps the tau whose share of fixed unit-hours is nearest its
target (the smaller tau on a tie). Stored per member: parent, seed, target, tau, the share
reached, the oracle's iterations and rel_kkt, and the fixing itself as zlib-compressed,
base64-encoded bit planes over [G][T]: which unit-hours are fixed, and the rounded u, v, w of
the fixed ones. With "first last" only members first..last-1 are (re)computed and merged into
the existing file.
"""
import base64
import json
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import fixing as ofix  # noqa: E402
from paper_2510_10891_amd import scuc  # noqa: E402

TAUS = (0.0, 1e-6, 1e-4, 1e-3, 0.01, 0.03, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.45)
COUNT = 64


def plane(bits: np.ndarray) -> str:
    return base64.b64encode(zlib.compress(np.packbits(bits.astype(np.uint8).ravel()).tobytes(), 9)).decode()


def member(parent: scuc.SCUCConfig, seed: int, target: float) -> dict:
    _, lp = scuc.make_instance(parent, seed)
    G, T = parent.n_gen, parent.T
    t, g = np.arange(T)[None, :], np.arange(G)[:, None]
    cols = np.stack([scuc.col_index(G, t, var, g) for var in (scuc.U, scuc.V, scuc.W)], -1).tolist()
    t0 = time.time()
    r = oracle.solve(lp, oracle.Options(tol=1e-4, max_iter=400000))
    best = None
    for tau in TAUS:
        fixed, rounded = ofix.algorithm1(r.x, cols, tau)
        share = float(fixed.mean())
        if best is None or abs(share - target) < abs(best[1] - target):
            best = (tau, share, fixed, rounded)
    tau, share, fixed, rounded = best
    on = fixed == 1
    return dict(parent=parent.name, seed=seed, target=target, tau=tau, fixed_u=share, G=G, T=T,
                oracle_term=r.term, oracle_iters=r.iters, oracle_rel_kkt=r.rel_kkt,
                oracle_seconds=round(time.time() - t0, 1),
                fixed=plane(on), u=plane(on & (rounded[:, :, 0] == 1)), v=plane(on & (rounded[:, :, 1] == 1)),
                w=plane(on & (rounded[:, :, 2] == 1)))


def parents(which: str):
    if which == "medium":
        return [scuc.MEDIUM] * COUNT
    return [scuc.BATCH_PARENTS[i % len(scuc.BATCH_PARENTS)] for i in range(COUNT)]


if __name__ == "__main__":
    which = sys.argv[1]
    first, last = (int(sys.argv[2]), int(sys.argv[3])) if len(sys.argv) > 3 else (0, COUNT)
    path = os.path.join(HERE, f"fixing_masks_{which}.json")
    rec = json.load(open(path)) if os.path.exists(path) else dict(
        batch=which, source="oracle.solve (FP64, tol 1e-4) of each parent relaxation, then oracle.fixing.algorithm1",
        taus=list(TAUS), members=[None] * COUNT)
    par = parents(which)
    for i in range(first, last):
        rec["members"][i] = member(par[i], 100 + i, 0.2 + 0.7 * i / (COUNT - 1))
        m = rec["members"][i]
        print(f"{i}: {m['parent']} seed {m['seed']} tau {m['tau']} share {m['fixed_u']:.3f} "
              f"(target {m['target']:.3f}) {m['oracle_term']} {m['oracle_iters']} its {m['oracle_seconds']} s",
              flush=True)
        with open(path, "w") as f:
            json.dump(rec, f, indent=0)
