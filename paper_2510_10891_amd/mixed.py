"""FP32 storage with an FP64 continuation of stalled LPs.

FP32 storage (the FP32 variant of the GPU solver in Section III-B) rounds the scaled matrix and
the iterates to 24 bits. That puts a floor under the residuals (of the order of
2^-24 ||A~^T |y~| || / ||c~|| for the dual one), and an FP32 run can also settle on a plateau above
the tolerance that FP64 storage leaves (seen on a reduced LP at rel_kkt 1e-3, far above its rounding
floor). With hpr_opts.stall_iters set the library ends a solve whose residuals stop falling as
"stalled" (a plateau that FP32 would leave later ends that way too: its continuation costs FP64
iterations, not accuracy); the functions here continue those LPs with FP64 storage from the point
the FP32 run returned (a warm start that skips the start-point race: that point is the FP32 run's
best estimate), so that every LP ends at the requested tolerance or at a genuine iteration or time
limit. All arithmetic runs in the library.
"""
from __future__ import annotations

import time
from dataclasses import replace

from . import hprlp


STALL_ITERS = 8192   # stall-test span used when the caller's options leave the test off


def fp32_options(opts: hprlp.Options) -> hprlp.Options:
    """The FP32 run's options: the caller's, with the stall test on."""
    return replace(opts, stall_iters=opts.stall_iters or STALL_ITERS)


def fp64_options(opts: hprlp.Options, iters_done: int) -> hprlp.Options:
    """The continuation's options: FP64 storage, the caller's point kept, the iterations left."""
    return replace(opts, precision=hprlp.HPR_FP64, warm_fallback=0,
                   max_iter=max(opts.max_iter - iters_done, opts.check_every))


def merge(first: hprlp.Info, second: hprlp.Info, offset_s: float) -> hprlp.Info:
    """Info of an FP32 run continued in FP64: the continuation's outcome, the iterations and
    restarts of both runs, and the time to the continuation's stop counted from the start of
    the FP32 run (`offset_s` = seconds from that start to the continuation's solve call, which
    includes the continuation's setup)."""
    return replace(second, iters=first.iters + second.iters, restarts=first.restarts + second.restarts,
                   setup_s=first.setup_s, solve_s=offset_s + second.solve_s, warm_start=first.warm_start)


def continue_stalled(lps, opts: hprlp.Options, infos, get_solution, t_start: float | None = None):
    """Continue the members of an FP32 solve that ended "stalled" as one FP64 batch.

    lps: the LPs of the solve; infos: their Info; get_solution(i) -> (x, y, z) of LP i as the
    FP32 run left it; t_start: perf_counter() at the start of that run, for the stop times of
    the continued members (without it each is counted as if its continuation had started
    when its FP32 run stopped). Returns (infos with the continued members merged in,
    {i: (x, y, z)} of those members)."""
    idx = [i for i, inf in enumerate(infos) if inf.term == "stalled"]
    if not idx:
        return list(infos), {}
    t_cont = time.perf_counter()
    o = fp64_options(opts, max(infos[i].iters for i in idx))
    b = hprlp.hpr_batch_create([lps[i] for i in idx], o)
    try:
        for k, i in enumerate(idx):
            x, y, _ = get_solution(i)
            hprlp.hpr_batch_set_start(b, k, x, y)
        t_call = time.perf_counter()
        more = hprlp.hpr_batch_solve(b)
        sols = {i: hprlp.hpr_batch_get_solution(b, k) for k, i in enumerate(idx)}
    finally:
        hprlp.hpr_batch_destroy(b)
    out = list(infos)
    for k, i in enumerate(idx):
        offset = t_call - t_start if t_start is not None else infos[i].solve_s + (t_call - t_cont)
        out[i] = merge(infos[i], more[k], offset)
    return out, sols


def solve(lp, opts: hprlp.Options | None = None, x0=None, y0=None):
    """hprlp.solve with the FP64 continuation: returns (info, x, y, z, continued); info.solve_s
    runs from the FP32 solve call to the continuation's stop (the continuation's setup
    included)."""
    opts = fp32_options(opts or hprlp.Options(precision=hprlp.HPR_FP32))
    h = hprlp.hpr_create(lp, opts)
    try:
        if x0 is not None or y0 is not None:
            hprlp.hpr_set_start(h, x0, y0)
        t0 = time.perf_counter()
        info = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
    finally:
        hprlp.hpr_destroy(h)
    if info.term != "stalled":
        return info, x, y, z, False
    h = hprlp.hpr_create(lp, fp64_options(opts, info.iters))
    try:
        hprlp.hpr_set_start(h, x, y)
        offset = time.perf_counter() - t0
        more = hprlp.hpr_solve(h)
        x, y, z = hprlp.hpr_get_solution(h)
    finally:
        hprlp.hpr_destroy(h)
    return merge(info, more, offset), x, y, z, True
