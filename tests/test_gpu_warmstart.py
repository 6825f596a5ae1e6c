"""Learned warm start: networks trained on the GPU (the library's own kernels) on solutions
the solver produced for training instances, evaluated on held-out reduced LPs.

Checked: the trained networks' losses fall; every warm-started solve reaches 1e-4 relative
KKT as judged by the oracle's FP64 evaluator; an LP whose prediction the fallback rejects runs
exactly the cold solve. The iteration gain over cold starts is printed and recorded, whatever
it is."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2510_10891_amd import fixing, hprlp, warmstart

pytestmark = pytest.mark.gpu



def _train_lps(n):
    return [fixing.reduced_lp(fixing.BATCH_PARENTS[i % 2], 10000 + i, 0.2 + 0.7 * ((i * 37) % 64) / 63).lp
            for i in range(n)]


def test_learned_warm_start_against_cold_start():
    lps = _train_lps(400)
    opts = hprlp.Options(tol=1e-4, max_iter=100000, unroll=4)
    sols = []
    for k in range(0, len(lps), 200):
        sols += [(x, y) for (_, x, y, _) in hprlp.batch_solve(lps[k:k + 200], opts)]
    Xg, Tg, Xl, Tl = warmstart.training_set(lps, sols)
    gen_net, lg = warmstart.train(warmstart.GEN_SIZES, Xg, Tg, steps=1500, batch=8192, lr=1e-3)
    line_net, ll = warmstart.train(warmstart.LINE_SIZES, Xl, Tl, steps=1500, batch=8192, lr=1e-3)
    assert np.mean(lg[-50:]) < 0.5 * np.mean(lg[:5])
    assert np.mean(ll[-50:]) <= np.mean(ll[:5])

    ev = [fixing.reduced_lp(fixing.BATCH_PARENTS[i % 3], 100 + i, 0.2 + 0.7 * i / 15).lp for i in range(16)]
    cold = hprlp.batch_solve(ev, opts)
    starts = [warmstart.predict_start(gen_net, line_net, lp) for lp in ev]
    warm = hprlp.batch_solve(ev, opts, starts=starts)
    rows = []
    for lp, (ic, xc, yc, zc), (iw, xw, yw, zw) in zip(ev, cold, warm):
        assert ic.term == "solved" and iw.term == "solved"
        assert oracle.kkt(lp, xw, yw, zw)["rel_kkt"] <= 1e-4 * (1 + 1e-6)
        if not iw.warm_start:
            assert iw.iters == ic.iters and np.array_equal(xw, xc)
        rows.append(dict(parent=lp.meta["parent"], n=lp.n, cold=ic.iters, warm=iw.iters, used=iw.warm_start))
    cold_total = sum(r["cold"] for r in rows)
    warm_total = sum(r["warm"] for r in rows)
    summary = dict(train_lps=len(lps), eval_lps=len(ev), cold_iters=cold_total, warm_iters=warm_total,
                   ratio=warm_total / cold_total, used=sum(r["used"] for r in rows), per_lp=rows,
                   gen_loss=[float(np.mean(lg[:5])), float(np.mean(lg[-50:]))],
                   line_loss=[float(np.mean(ll[:5])), float(np.mean(ll[-50:]))])
    print(json.dumps(summary))
    out = os.environ.get("HPR_TEST_OUTPUT_DIR")   # optional: where to keep the per-LP record
    if out and os.path.isdir(out):
        with open(os.path.join(out, "warmstart_eval.json"), "w") as f:
            json.dump(summary, f, indent=1)
