"""Benchmark: time to 1e-4 relative KKT of the LP relaxation of a synthetic 2,000-bus SCUC
instance (500 units, 48 h, 300 monitored lines x (1 + 10 outages)) on one MI355X.

A step is one cold-start solve (hpr_solve) of the instance already resident in HBM: the
whole iteration with its FP64 checks, restarts and sigma updates, until the first check
with rel_kkt <= 1e-4 (FP64-verified). The headline runs with FP32 storage of A and the
iterates (FP64 reductions); the plain FP64 solve of the same instance is timed beside it.

Printed: one JSON line with the metric, iterations/s, the roofline of the dominant fused
kernel (algorithmic bytes / event-timed duration against 8 TB/s), and the CPU oracle
timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` measured by rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, each scaled by the ratio a plain copy kernel of known size gives)
    as recorded under profiles/, or None when no record exists or the kernel or schedule source
    has changed since (the record holds sources_sha256() of the sources it was measured with)."""
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = sources_sha256()
    m_sha = re.search(r"sources_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != sha:
        return None
    return float(m_val.group(1))


KERNEL_SOURCES = ("csr.h", "kernels_dual32.hip", "kernels_primal32.hip", "solver.hip", "setup.hip")


def sources_sha256():
    """SHA-256 of the sources that decide what the fused FP32 steps move: the kernel template,
    their instantiations, the runtime that builds the layouts and schedules, and the instance
    generator (its row and column order shapes the layouts)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2510_10891_amd", "csrc", name), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_2510_10891_amd", "scuc.py"), "rb").read())
    return h.hexdigest()


def write_traffic_record(fetch_dir, write_dir, kernel="dual_step_fp32", workload="scuc-2000bus-500gen-T48",
                         config="medium"):
    """The record recorded_traffic reads, from two rocprofv3 --pmc runs of this bench (FETCH_SIZE,
    then WRITE_SIZE, `--max-iter 129 --precision fp32 --config <config>`): per-launch mean of the
    fused FP32 step `kernel` over the solve's own last 64 launches (the schedule tuner's timing
    launches come before the solve), each counter scaled by the ratio it gives for the stream
    probe's copy kernel (1 GiB read and written per dispatch)."""
    import csv
    import glob
    import re

    op = "DualOp<float>" if kernel.startswith("dual") else "PrimalOp<float>"

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("(anonymous namespace)::", ""))
                    name = name.replace("void ", "").replace("hpr::", "")
                    rows.append((int(r["Dispatch_Id"]), name, float(r["Counter_Value"])))
        rows.sort()
        return rows

    def solve_mean(rows):
        mine = [r for r in rows if r[1].startswith((f"csr_kernel<{op}", f"csr_kernel<Packed<{op}"))][-64:]
        names = sorted({r[1] for r in mine})
        return sum(r[2] for r in mine) / len(mine), names, len(mine)

    def copy_mean(rows):
        v = [r[2] for r in rows if r[1].startswith("stream_copy_kernel")]
        return sum(v) / len(v)

    fr, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    fetch_dir, write_dir = (os.path.relpath(os.path.abspath(d), ROOT) for d in (fetch_dir, write_dir))
    known = float(1 << 20)   # KiB in 1 GiB
    cfk, cwk = copy_mean(fr), copy_mean(wr)
    cf, cw = known / cfk, known / cwk
    fk, fnames, fn = solve_mean(fr)
    wk, wnames, wn = solve_mean(wr)
    traffic = (fk * cf + wk * cw) * 1024
    what = "dual half-iteration over A~" if op.startswith("Dual") else "primal half-iteration over A~^T"
    text = f"""# HBM traffic of the fused FP32 {kernel.split('_')[0]} step on {workload}

Kernel: `csr_kernel<{op}, ...>`, one launch = one {what}; the solve's last {fn} / {wn} launches in the
FETCH / WRITE runs (variants {", ".join(f"`{x}`" for x in fnames)} / {", ".join(f"`{x}`" for x in wnames)}).

Commands (R = the repository root; each counter in a run of its own, then this record from the
repository root):

```
cd /tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/{fetch_dir} -o run -- python3 $R/bench.py --steps 1 --warmup 0 --no-cpu --batch 0 --successive 0 --large-steps 0 --max-iter 129 --precision fp32 --config {config}
cd /tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d $R/{write_dir} -o run -- python3 $R/bench.py --steps 1 --warmup 0 --no-cpu --batch 0 --successive 0 --large-steps 0 --max-iter 129 --precision fp32 --config {config}
python bench.py --traffic-record {fetch_dir} {write_dir} --traffic-kernel {kernel} --config {config}
```

Calibration: the stream probe's copy kernel reads and writes 1,048,576 KiB per dispatch; FETCH_SIZE
reports {cfk:,.1f} KiB for it (factor {cf:.4f}), WRITE_SIZE {cwk:,.1f} KiB (factor {cw:.4f}).

| counter | raw KiB per launch | calibrated bytes per launch |
|---|---|---|
| FETCH_SIZE | {fk:,.1f} | {fk * cf * 1024:,.0f} |
| WRITE_SIZE | {wk:,.1f} | {wk * cw * 1024:,.0f} |

traffic_bytes_per_launch: {traffic:.0f}
sources_sha256: {sources_sha256()}   (SHA-256 of {", ".join(KERNEL_SOURCES)} under paper_2510_10891_amd/csrc, in that order, then paper_2510_10891_amd/scuc.py)
"""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    with open(path, "w") as fh:
        fh.write(text)
    print(text)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(lp, fp32: bool):
    """Bytes one launch of each fused kernel must move with 4-byte column indices and row offsets
    (the count of the iteration of eq.(hpr) for a plain CSR matrix).

    Dual step (rows of A): nnz values + nnz column indices + row offsets, reads y, y0, lo, hi,
    writes y, gathers each entry of xhat once.  Primal step (rows of A^T): nnz values + indices
    + offsets, reads x, x0, c, l, u, writes xhat and x, gathers each entry of y once.
    Value width 4 (FP32 storage) or 8 (FP64).
    """
    sv = 4 if fp32 else 8
    nnz, m, n = lp.nnz, lp.m, lp.n
    dual = nnz * (sv + 4) + 4 * m + sv * (5 * m) + sv * n
    primal = nnz * (sv + 4) + 4 * n + sv * (7 * n) + sv * m
    return primal, dual


def layout_bytes(lp, fp32: bool, ks=None):
    """Bytes one launch of each fused kernel must move in the layout the library streams (the
    figure the roofline fraction is computed from): every row padded to a multiple of 4 entries,
    each stored entry a value; per quad (4 entries) of a row spanning fewer than 65,536 columns
    either its four 16-bit offsets or, when the matrix reads packed words (kernel stats `ks`), a
    4-byte word (13-bit offset of the first entry and three 6-bit gaps) plus the 16-bit offsets of the
    quads whose gaps do not fit; 4-byte indices for
    wider rows; one 16-byte row descriptor per row; and the same vector traffic as
    algorithmic_bytes (each gathered entry read once). Returns (primal, dual)."""
    import numpy as np
    sv = 4 if fp32 else 8
    A = lp.to_scipy().tocsr()

    def matrix_bytes(M, narrow_quads, packed_quads, used):
        M = M.tocsr()
        M.sort_indices()
        lens = np.diff(M.indptr)
        padded = (lens + 3) // 4 * 4
        lo = np.full(M.shape[0], 0, np.int64)
        hi = np.full(M.shape[0], 0, np.int64)
        nz = lens > 0
        lo[nz] = M.indices[M.indptr[:-1][nz]]
        hi[nz] = M.indices[M.indptr[1:][nz] - 1]
        wide = (hi - lo) >= 65536
        narrow = int(padded[~wide].sum()) // 4
        if used and narrow_quads == narrow:
            narrow_idx = 4 * packed_quads + 12 * (narrow - packed_quads)
        else:                             # 16-bit offsets only
            narrow_idx = 8 * narrow
        idx = 16 * (int(padded[wide].sum()) // 4) + narrow_idx
        return int(padded.sum() * sv + idx + 16 * M.shape[0])

    ks = ks or {}
    m, n = lp.m, lp.n
    dual = (matrix_bytes(A, ks.get("narrow_quads_a"), ks.get("packed_quads_a"), ks.get("packed_a"))
            + sv * (5 * m) + sv * n)
    primal = (matrix_bytes(A.T, ks.get("narrow_quads_at"), ks.get("packed_quads_at"), ks.get("packed_at"))
              + sv * (7 * n) + sv * m)
    return primal, dual


def run_solves(hprlp, h, steps, warmup, torch):
    infos = []
    for _ in range(warmup):
        hprlp.hpr_set_start(h, None, None)
        hprlp.hpr_solve(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hprlp.hpr_set_start(h, None, None)
        infos.append(hprlp.hpr_solve(h))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return infos, (t1 - t0) / steps


def cpu_baseline(lp, gpu_fp64_iters, limit_s, gpu_objs):
    """The oracle (plain C, FP64, OpenMP row loops) on the same instance: a full solve to 1e-4
    bounded by `limit_s` seconds of wall time. If it reaches the tolerance, its own time is the
    value and the GPU objectives are compared with its objective (the error against the FP64
    oracle); if it stops at the limit, the time to 1e-4 is extrapolated from its measured rate
    to the iteration count of the FP64 GPU solve (same algorithm, same iterations)."""
    import oracle
    oracle.build()
    r = oracle.solve(lp, oracle.Options(tol=1e-4, max_iter=1000000, time_limit=limit_s))
    its_per_s = r.iters / max(r.solve_s, 1e-9)
    out = dict(unit="s", cores=oracle.num_threads(), kind="oracle", iters=r.iters,
               iters_per_s=round(its_per_s, 3), setup_s=round(r.setup_s, 3), host=host_info())
    if r.term == "solved":
        out["value"] = round(r.setup_s + r.solve_s, 3)
        out["sample"] = (f"full oracle solve of the same instance to 1e-4: {r.iters} iterations, "
                         f"{r.solve_s:.1f} s + setup {r.setup_s:.1f} s")
        out["oracle_pobj"] = r.pobj
        out["gpu_obj_rel_err_vs_oracle"] = {k: abs(v - r.pobj) / max(1.0, abs(r.pobj)) for k, v in gpu_objs.items()}
        # the same instance on one core: a short sample, extrapolated to the full solve
        nt = oracle.num_threads()
        oracle.set_num_threads(1)
        k = 64
        r1 = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=k))
        oracle.set_num_threads(nt)
        out["single_thread"] = dict(value=round(r1.setup_s + r.iters * r1.solve_s / r1.iters, 3), cores=1,
                                    sample=f"{r1.iters} iterations on one core in {r1.solve_s:.1f} s plus setup "
                                           f"{r1.setup_s:.1f} s, extrapolated to the {r.iters} iterations above")
    else:
        out["value"] = round(r.setup_s + gpu_fp64_iters / its_per_s, 3)
        out["sample"] = (f"{r.iters} oracle iterations of the same instance in {r.solve_s:.1f} s (stopped at "
                         f"the {limit_s:.0f} s bound) plus setup {r.setup_s:.1f} s; time to 1e-4 extrapolated "
                         f"to the {gpu_fp64_iters} iterations the FP64 GPU solve takes")
    return out


TAU_GRID = (0.0, 1e-6, 1e-4, 1e-3, 0.01, 0.03, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.45)


def reduced_batch(count, big, stream):
    """The batch's reduced LPs: member i has parent seed 100 + i and Algorithm 1's fixing of its
    parent's solved relaxation at the tau (of TAU_GRID) whose share of fixed unit-hours is
    nearest 0.2 + 0.7 i / (count - 1). Mixed parents (30 to 1,000 buses): the fixings stored
    under tests/golden (relaxations solved by the oracle); 2,000-bus parents: relaxations solved
    here by the GPU solver (FP32, 1e-4), Algorithm 1 on the device."""
    from paper_2510_10891_amd import fixing, hprlp, scuc, successive

    if not big:
        path = os.path.join(ROOT, "tests", "golden", "fixing_masks_mixed.json")
        fx = fixing.load_fixings(path) if count <= 64 and os.path.exists(path) else None
        return [p.lp for p in fixing.make_reduced_batch(count=count, seed0=100, fixings=fx[:count] if fx else None)]
    opts = hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=200000, stream=stream)
    lps = []
    for i in range(count):
        target = 0.2 + 0.7 * i / max(count - 1, 1)
        data, lp = scuc.make_instance(scuc.MEDIUM, 100 + i)
        fx = successive.solved_fixing(data, lp, target, TAU_GRID, opts)
        if fx is None:
            raise RuntimeError(f"parent relaxation of member {i} was not solved")
        fixed, ur, vr, wr, tau, info = fx
        pre = fixing.apply_fixing(scuc.MEDIUM, 100 + i, target, data, lp, fixed, ur, vr, wr,
                                  f"solved relaxation (GPU, {info.iters} iterations), tau {tau}")
        lps.append(pre.lp)
        log(f"reduced LP {i + 1}/{count}: tau {tau}, {pre.lp.meta['fixed_u']:.3f} of u fixed (target {target:.3f}), "
            f"n {pre.lp.n}, nnz {pre.lp.nnz}")
    return lps


def batch_leg(count, stream, parent="mixed", sequential=True, max_iter=100000, detail=None, stall_iters=-1):
    """The reduced LPs of successive-fixing rounds (uneven sizes) solved as one batch with FP32
    storage, against the same LPs solved one after another with the same options. `parent`:
    "mixed" = parents of 30 to 1,000 buses; "medium" = 2,000-bus parents (seeds 100 + i), each
    member filling the GPU on its own (no warm-up solves there: one batch solve takes minutes
    and its graph capture is a negligible share)."""
    import numpy as np
    import torch

    from paper_2510_10891_amd import fixing, hprlp, mixed, scuc

    big = parent == "medium"
    t = time.perf_counter()
    lps = reduced_batch(count, big, stream)
    log(f"batch: {count} reduced LPs, n {min(lp.n for lp in lps)}..{max(lp.n for lp in lps)}, "
        f"nnz total {sum(lp.nnz for lp in lps)} ({time.perf_counter() - t:.1f} s)")
    # the 2,000-bus batch is one long library call: a time limit bounds it (members still running
    # then end as time_limit and are counted as unsolved)
    if stall_iters < 0:
        stall_iters = 8192 if big else 0
    opts = hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=max_iter, stream=stream,
                         time_limit_s=400.0 if big else 0.0, stall_iters=stall_iters)
    t = time.perf_counter()
    b = hprlp.hpr_batch_create(lps, opts)
    log(f"batch engine created in {time.perf_counter() - t:.1f} s")
    if not big:
        hprlp.hpr_batch_solve(b)                 # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = hprlp.hpr_batch_solve(b)
    # members whose FP32 run stalled above the tolerance go on in FP64 from their points
    infos, cont = mixed.continue_stalled(lps, opts, infos, lambda i: hprlp.hpr_batch_get_solution(b, i), t0)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batch solve {t_batch:.2f} s")
    worst = max(i.rel_kkt for i in infos)       # FP64 evaluation by the library
    setup = infos[0].setup_s
    hprlp.hpr_batch_destroy(b)
    seq, t_seq, seq_cont = [], 0.0, 0
    for k in range(0, count if sequential else 0, 16 if big else count):   # big members: 16 handles at a time
        handles = [hprlp.hpr_create(lp, opts) for lp in lps[k:k + (16 if big else count)]]
        if not big:
            for h in handles:
                hprlp.hpr_solve(h)               # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        part = [hprlp.hpr_solve(h) for h in handles]
        part, c = mixed.continue_stalled(lps[k:k + len(handles)], opts, part,
                                         lambda i: hprlp.hpr_get_solution(handles[i]))
        seq += part
        seq_cont += len(c)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        for h in handles:
            hprlp.hpr_destroy(h)
        log(f"sequential: {len(seq)}/{count} solved one by one ({t_seq:.1f} s)")
    iters = np.array([i.iters for i in infos])
    name = "2,000-bus parents" if big else "parents of 30-1,000 buses"
    shares = [float(lp.meta.get("fixed_u", 0.0)) for lp in lps]
    out = dict(workload=f"{count} reduced SCUC LPs ({name}; Algorithm 1 fixings of the solved relaxations, "
                        f"{min(shares):.0%}-{max(shares):.0%} of u fixed, presolved)",
               fixings=lps[0].meta.get("fixing_source", "").split(",")[0] if lps else None,
               lps=count, nnz_total=int(sum(lp.nnz for lp in lps)),
               n_min=int(min(lp.n for lp in lps)), n_max=int(max(lp.n for lp in lps)),
               batch_s=round(t_batch, 4), lps_per_s=round(count / t_batch, 2),
               sequential_s=round(t_seq, 4) if sequential else None,
               speedup_vs_sequential=round(t_seq / t_batch, 3) if sequential else None,
               solved=int(sum(i.term == "solved" for i in infos)),
               seq_solved=int(sum(i.term == "solved" for i in seq)),
               stall_iters=stall_iters, continued_in_fp64=sorted(cont), seq_continued_in_fp64=seq_cont,
               worst_rel_kkt_fp64_eval=worst, setup_s=round(setup, 2),
               iters_min=int(iters.min()), iters_median=int(np.median(iters)), iters_max=int(iters.max()),
               lp_time_to_stop_s=[round(float(q), 4) for q in np.percentile([i.solve_s for i in infos],
                                                                            [0, 50, 90, 100])],
               iters_total=int(iters.sum()), warmed_up=not big,
               unsolved=[dict(index=i, parent=lps[i].meta.get("parent"), seed=lps[i].meta.get("seed"),
                              fixed_u=round(float(lps[i].meta.get("fixed_u", 0.0)), 4), n=lps[i].n, m=lps[i].m,
                              nnz=int(lps[i].nnz), term=infos[i].term, iters=infos[i].iters,
                              rel_kkt=infos[i].rel_kkt, rel_p=infos[i].rel_p, rel_d=infos[i].rel_d,
                              rel_gap=infos[i].rel_gap, restarts=infos[i].restarts, sigma=infos[i].sigma)
                         for i in range(count) if infos[i].term != "solved"])
    if detail:   # per-LP record: size, iterations and time to stop, batched and one by one
        with open(detail, "w") as fh:
            json.dump([dict(index=i, parent=lps[i].meta.get("parent"), n=lps[i].n, m=lps[i].m, nnz=int(lps[i].nnz),
                            iters=infos[i].iters, stop_s=infos[i].solve_s, term=infos[i].term,
                            seq_s=(seq[i].solve_s if i < len(seq) else None)) for i in range(count)], fh)
    log(f"batch: {out}")
    return out


def mlp_leg(steps, stream, rows=8192):
    """Training-step throughput of the warm-start network (the unit-hour network's shape,
    BF16 MFMA products with FP32 accumulation): `steps` Adam steps on `rows` synthetic rows,
    timed after one warm-up step; FLOPs = 2 rows (sum K N) for the forward products and twice
    that for the backward ones (dW and, except for the first layer, dh)."""
    import numpy as np
    import torch

    from paper_2510_10891_amd import mlp, warmstart

    sizes = warmstart.GEN_SIZES
    rng = np.random.default_rng(0)
    X = rng.standard_normal((rows, sizes[0])).astype(np.float32)
    T = rng.standard_normal((rows, sizes[-1])).astype(np.float32)
    net = mlp.MLP(sizes, mlp.init_params(sizes, 0), stream=stream)
    net.train_step(X, T, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(X, T, 1e-3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kn = [sizes[i] * sizes[i + 1] for i in range(len(sizes) - 1)]
    flops = 2.0 * rows * (sum(kn) + sum(kn) + sum(kn[1:]))
    out = dict(workload=f"Adam steps of the unit-hour network {sizes} on {rows} rows (BF16 MFMA, FP32 accumulation)",
               ms_per_step=round(dt * 1e3, 3), tflops=round(flops / dt / 1e12, 2),
               frac_of_bf16_peak=round(flops / dt / 2.5e15, 5),
               note="host-staged inputs: each step copies its rows to the device and reads the loss back")
    log(f"mlp: {out}")
    return out


def warmstart_leg(n_train, n_eval, stream):
    """Learned warm start: train the two networks on the GPU on solver-produced solutions of
    `n_train` training LPs, then solve the evaluation batch (the batch leg's reduced LPs)
    cold and warm-started, FP32 storage, to 1e-4; inference time counts on the warm side."""
    import numpy as np
    import torch

    from paper_2510_10891_amd import fixing, hprlp, warmstart

    t0 = time.perf_counter()
    lps = []
    for k in range(0, n_train, 200):
        lps += warmstart.training_lps_range(k, min(k + 200, n_train), workers=min(16, os.cpu_count() or 1))
        log(f"warm start: {len(lps)} of {n_train} training LPs generated")
    t_gen = time.perf_counter() - t0
    opts = hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=100000, stream=stream)
    t0 = time.perf_counter()
    sols, ok = warmstart.label(lps, opts, log=log)
    t_label = time.perf_counter() - t0
    keep = [i for i in range(len(lps)) if ok[i]]
    Xg, Tg, Xl, Tl = warmstart.training_set([lps[i] for i in keep], [sols[i] for i in keep])
    t0 = time.perf_counter()
    gen_net, lg = warmstart.train(warmstart.GEN_SIZES, Xg, Tg, steps=1500, batch=8192, lr=1e-3, stream=stream)
    line_net, ll = warmstart.train(warmstart.LINE_SIZES, Xl, Tl, steps=1500, batch=8192, lr=1e-3, stream=stream)
    t_train = time.perf_counter() - t0
    log(f"warm start: {len(keep)} labelled LPs ({t_gen:.1f} s gen, {t_label:.1f} s solves), "
        f"train {t_train:.1f} s, gen loss {np.mean(lg[:5]):.3g}->{np.mean(lg[-50:]):.3g}, "
        f"line loss {np.mean(ll[:5]):.3g}->{np.mean(ll[-50:]):.3g}")
    ev = [p.lp for p in fixing.make_reduced_batch(count=n_eval, seed0=100)]
    b = hprlp.hpr_batch_create(ev, opts)
    hprlp.hpr_batch_solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold = hprlp.hpr_batch_solve(b)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    t0 = time.perf_counter()
    starts = [warmstart.predict_start(gen_net, line_net, lp) for lp in ev]
    t_inf = time.perf_counter() - t0
    for i, (x0, y0) in enumerate(starts):
        hprlp.hpr_batch_set_start(b, i, x0, y0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm = hprlp.hpr_batch_solve(b)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    hprlp.hpr_batch_destroy(b)
    # the plain solver on the same LPs: FP64, cold, one LP after another
    opts64 = hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP64, max_iter=100000, stream=stream)
    handles = [hprlp.hpr_create(lp, opts64) for lp in ev]
    for h in handles:
        hprlp.hpr_solve(h)                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [hprlp.hpr_solve(h) for h in handles]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for h in handles:
        hprlp.hpr_destroy(h)
    ci = np.array([i.iters for i in cold])
    wi = np.array([i.iters for i in warm])
    out = dict(train_lps=len(keep), eval_lps=len(ev), train_s=round(t_train, 2),
               gen_loss=[float(np.mean(lg[:5])), float(np.mean(lg[-50:]))],
               line_loss=[float(np.mean(ll[:5])), float(np.mean(ll[-50:]))],
               cold_iters_total=int(ci.sum()), warm_iters_total=int(wi.sum()),
               iters_ratio=round(float(wi.sum() / ci.sum()), 4),
               median_lp_ratio=round(float(np.median(wi / ci)), 4),
               warm_used=int(sum(i.warm_start for i in warm)),
               cold_batch_s=round(t_cold, 3), warm_batch_s=round(t_warm + t_inf, 3), inference_s=round(t_inf, 3),
               plain_fp64_sequential_s=round(t_plain, 3),
               speedup_fp32_batched_warm_vs_plain_fp64=round(t_plain / (t_warm + t_inf), 3),
               all_solved=bool(all(i.term == "solved" for i in cold + warm + plain)),
               worst_rel_kkt_fp64_eval=float(max(i.rel_kkt for i in warm)))
    log(f"warm start: {out}")
    return out


def ablation_leg(data, rounds, stream, formulation="compact"):
    """LP-side analogue of the paper's ablation (Section V): successive fixing with `rounds`
    rounds on the bench instance under three solver configurations, LP time only (creation
    with scaling and lambda, plus the rounds' solves). SF(FOM): Ruiz (10 passes) + Pock-
    Chambolle + b/c normalisation, no instance-aware scaling, FP64. SF(FOM+FP32): the same
    with FP32 storage. SF: instance-aware scaling (Section III-A), Ruiz off, FP32. A fourth run,
    not in the paper, keeps Ruiz and instance-aware scaling off (FP32): what the instance-aware
    scaling buys when it replaces Ruiz. On the full formulation every LP is first presolved
    (cost variables substituted). Each solve is bounded by 150 s."""
    import torch

    from paper_2510_10891_amd import hprlp, scuc, successive

    full = hprlp.HPR_SCALE_PC | hprlp.HPR_SCALE_RUIZ | hprlp.HPR_SCALE_BC
    runs = [("SF(FOM)", False, full, hprlp.HPR_FP64), ("SF(FOM+FP32)", False, full, hprlp.HPR_FP32),
            ("SF", True, hprlp.HPR_SCALE_PC | hprlp.HPR_SCALE_BC, hprlp.HPR_FP32),
            ("PC only (FP32)", False, hprlp.HPR_SCALE_PC | hprlp.HPR_SCALE_BC, hprlp.HPR_FP32)]
    out = []
    for name, inst, scaling, prec in runs:
        if formulation == "full":
            from paper_2510_10891_amd import fixing
            lp = fixing.presolve_free_singletons(scuc.build_full_lp(data, instance_scaling=inst)).lp
        else:
            lp = scuc.build_lp(data, instance_scaling=inst)
        eta_c = lp.meta["eta_c"]
        opts = hprlp.Options(tol=1e-4, precision=prec, scaling=scaling, ruiz_iters=10, max_iter=200000,
                             stream=stream, time_limit_s=150.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = successive.run(data, lp, rounds=rounds, tau=0.1, opts=opts, log=lambda m: log(f"  {name} {m}"))
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        rec = dict(method=name, instance_scaling=inst, ruiz=bool(scaling & hprlp.HPR_SCALE_RUIZ),
                   precision="fp32" if prec == hprlp.HPR_FP32 else "fp64", lp_time_s=round(total, 3),
                   solve_s=round(sum(x.solve_s for x in r.rounds), 3),
                   iters=[x.iters for x in r.rounds], terms=[x.term for x in r.rounds],
                   objective=[x.objective * eta_c for x in r.rounds],
                   fixed_u=[round(x.fixed_u, 4) for x in r.rounds])
        log(f"ablation: {rec}")
        out.append(rec)
    return out


def host_info():
    """CPU model, logical cores and memory of the host (for the CPU baseline's context)."""
    model, mem_gb = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return dict(cpu_model=model, logical_cpus=os.cpu_count(), mem_gib=mem_gb)


def large_leg(steps, stream, read_gbs, copy_gbs):
    """The 13,500-bus instance (1,000 monitored lines x (1 + 20 outages), T = 36): FP32 storage
    against the plain FP64 solve of the same instance, `steps` timed cold solves each after one
    warm-up, every solve to 1e-4 (FP64-evaluated), with the roofline of FP32's dominant kernel."""
    from paper_2510_10891_amd import hprlp, scuc
    import numpy as np
    import torch

    t = time.perf_counter()
    data, lp = scuc.make_instance("large", 0)
    gen_s = time.perf_counter() - t
    log(f"large instance: m={lp.m} n={lp.n} nnz={lp.nnz} ({gen_s:.1f} s)")
    out = dict(workload=data.cfg.name, m=lp.m, n=lp.n, nnz=lp.nnz, steps=steps)
    res = {}
    for name, prec in (("fp32", hprlp.HPR_FP32), ("fp64", hprlp.HPR_FP64)):
        opts = hprlp.Options(tol=1e-4, precision=prec, max_iter=200000, profile=1, stream=stream,
                             time_limit_s=60.0)
        h = hprlp.hpr_create(lp, opts)
        infos, sec = run_solves(hprlp, h, steps, 1, torch)
        ks = hprlp.hpr_get_kernel_stats(h)
        x, _, _ = hprlp.hpr_get_solution(h)
        hprlp.hpr_destroy(h)
        info = infos[-1]
        res[name] = (info, sec, ks, x)
        out[name] = dict(value=round(sec, 4), iters=info.iters, iters_per_s=round(info.iters / sec, 1),
                         setup_s=round(info.setup_s, 3), setup_phases_s=ks["setup_phases_s"],
                         solved=info.term == "solved", rel_kkt_fp64_eval=info.rel_kkt,
                         primal_us=round(ks["primal_ms"] * 1e3, 2), dual_us=round(ks["dual_ms"] * 1e3, 2),
                         schedule={"unroll_A": ks["unroll_a"], "unroll_At": ks["unroll_at"],
                                   "window_mode_A": ks["win_mode_a"], "window_mode_At": ks["win_mode_at"],
                                   "sliced_blocks_At": ks["sliced_blocks_at"],
                                   "blocks_in_rounds_A": ks["round_blocks_a"]})
        log(f"large {name}: {info.term} iters={info.iters} solve={sec:.3f}s setup={info.setup_s:.2f}s "
            f"primal={ks['primal_ms'] * 1e3:.1f}us dual={ks['dual_ms'] * 1e3:.1f}us {ks['setup_phases_s']}")
    (i32, s32, k32, x32), (i64, s64, k64, x64) = res["fp32"], res["fp64"]
    out["fp32_vs_fp64"] = dict(speedup=round(s64 / s32, 3),
                               obj_rel_diff=abs(i32.pobj - i64.pobj) / max(1.0, abs(i64.pobj)),
                               x_rel_diff=float(np.linalg.norm(x32 - x64) / max(1e-30, np.linalg.norm(x64))))
    out["roofline"] = roofline(lp, k32, data.cfg.name, read_gbs, copy_gbs)
    return out


def roofline(lp, ks, workload, read_gbs, copy_gbs, fp32=True):
    """Roofline record of the dominant fused kernel (the slower of the two steps, event-timed):
    the bytes its layout makes it move per launch (layout_bytes) over its average launch time,
    against 8 TB/s; the plain-CSR count (4-byte indices and offsets) beside it."""
    pb, db = layout_bytes(lp, fp32, ks)
    pa, da = algorithmic_bytes(lp, fp32)
    tag = "fp32" if fp32 else "fp64"
    if ks["dual_ms"] >= ks["primal_ms"]:
        kname, kbytes, kalg, kms, other = f"dual_step_{tag}", db, da, ks["dual_ms"], ks["primal_ms"]
    else:
        kname, kbytes, kalg, kms, other = f"primal_step_{tag}", pb, pa, ks["primal_ms"], ks["dual_ms"]
    if not kms > 0:      # no sampled launch (a run shorter than the sampling interval)
        return None
    achieved = kbytes / (kms * 1e-3) / 1e9
    return dict(bound="hbm", kernel=kname, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=recorded_traffic(kname, workload),
                bytes_per_launch=int(kbytes), launch_us=round(kms * 1e3, 2),
                other_kernel_us=round(other * 1e3, 2),
                packed_quads={"share_A": round(ks["packed_quads_a"] / max(1, ks["narrow_quads_a"]), 4),
                              "share_At": round(ks["packed_quads_at"] / max(1, ks["narrow_quads_at"]), 4),
                              "read_A": ks["packed_a"], "read_At": ks["packed_at"]},
                plain_csr_bytes_per_launch=int(kalg),
                plain_csr_gbs=round(kalg / (kms * 1e-3) / 1e9, 1),
                schedule={"unroll_A": ks["unroll_a"], "unroll_At": ks["unroll_at"],
                          "nontemporal_A": ks["nt_a"], "nontemporal_At": ks["nt_at"],
                          "window_mode_A": ks["win_mode_a"], "window_mode_At": ks["win_mode_at"],
                          "blocks_A": ks["blocks_a"], "blocks_At": ks["blocks_at"],
                          "blocks_in_rounds_A": ks["round_blocks_a"], "blocks_in_rounds_At": ks["round_blocks_at"]},
                stream_probe_gbs={"read": round(read_gbs, 1), "copy": round(copy_gbs, 1)},
                frac_of_stream_read=round(achieved / read_gbs, 4))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="medium")
    ap.add_argument("--formulation", choices=["compact", "full"], default="compact",
                    help="SCUC model: u, v, w, p per unit-hour, or the full one with cost segments, "
                         "no-load cost and unserved demand")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-limit", type=float, default=40.0,
                    help="wall-time bound (s) of the oracle solve in the cpu_baseline leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch", type=int, default=64, help="LPs in the batch leg (0: skip)")
    ap.add_argument("--batch-parent", choices=["mixed", "medium"], default="mixed",
                    help="parents of the batch's reduced LPs: 30-1,000 buses, or the 2,000-bus preset")
    ap.add_argument("--batch-no-seq", action="store_true",
                    help="skip the one-by-one solves of the batch's LPs")
    ap.add_argument("--batch-max-iter", type=int, default=100000)
    ap.add_argument("--batch-detail", default=None, help="write per-LP batch results to this JSON file")
    ap.add_argument("--stall-iters", type=int, default=-1,
                    help="FP32 stall-test span of the batch leg (stalled members continue in FP64; 0: off; "
                         "default: 8192 for 2,000-bus parents, off for the mixed parents, whose members all "
                         "converge in FP32 and where the continuation, run after the batch, only adds time)")
    ap.add_argument("--successive", type=int, default=4,
                    help="rounds of the successive-fixing leg on the bench instance (0: skip)")
    ap.add_argument("--large-steps", type=int, default=2,
                    help="timed solves per precision of the 13,500-bus leg (0: skip the leg)")
    ap.add_argument("--ablation", type=int, default=0,
                    help="rounds of the scaling/precision ablation leg (successive fixing; 0: skip)")
    ap.add_argument("--warmstart", type=int, default=0,
                    help="training LPs of the learned warm-start leg (0: skip)")
    ap.add_argument("--mlp-steps", type=int, default=0,
                    help="timed training steps of the warm-start network's throughput leg (0: skip)")
    ap.add_argument("--max-iter", type=int, default=200000,
                    help="iteration cap (lower it only for profiler runs; the line is then not a tolerance time)")
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--time-limit", type=float, default=0.0,
                    help="wall-time bound (s) of each timed solve (0: none); a solve that hits it "
                         "ends as time_limit and the line reports all_solved false")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM traffic record under profiles/ from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--traffic-kernel", choices=["dual_step_fp32", "primal_step_fp32"], default="dual_step_fp32")
    args = ap.parse_args()
    if args.traffic_record:
        from paper_2510_10891_amd import scuc
        write_traffic_record(*args.traffic_record, kernel=args.traffic_kernel,
                             workload=scuc.PRESETS[args.config].name, config=args.config)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_10891_amd import hprlp, scuc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream

    t = time.perf_counter()
    data, lp = scuc.make_instance(args.config, args.seed, formulation=args.formulation)
    workload = data.cfg.name + ("-full" if args.formulation == "full" else "")
    log(f"instance {workload}: m={lp.m} n={lp.n} nnz={lp.nnz} ({time.perf_counter() - t:.1f} s)")
    presolve = None
    if args.formulation == "full":
        from paper_2510_10891_amd import fixing
        t = time.perf_counter()
        sub = fixing.presolve_free_singletons(lp)
        presolve = dict(step="implied-free column singletons substituted (cost variables)",
                        removed_cols=int(len(sub.sub_c)), removed_rows=int(len(sub.sub_r)),
                        host_s=round(time.perf_counter() - t, 2), m=lp.m, n=lp.n, nnz=lp.nnz)
        lp = sub.lp
        del sub
        log(f"presolve: {presolve}; reduced m={lp.m} n={lp.n} nnz={lp.nnz}")

    res = {}
    legs = [("fp32", hprlp.HPR_FP32), ("fp64", hprlp.HPR_FP64)]
    if args.precision != "both":
        legs = [l for l in legs if l[0] == args.precision]
    for name, prec in legs:
        opts = hprlp.Options(tol=1e-4, precision=prec, max_iter=args.max_iter, profile=1, stream=stream,
                             time_limit_s=args.time_limit)
        h = hprlp.hpr_create(lp, opts)
        infos, sec = run_solves(hprlp, h, args.steps, args.warmup, torch)
        ks = hprlp.hpr_get_kernel_stats(h)
        x, y, z = hprlp.hpr_get_solution(h)
        info = infos[-1]
        res[name] = dict(sec=sec, info=info, ks=ks, x=x)
        log(f"{name}: {info.term} iters={info.iters} restarts={info.restarts} solve={sec:.4f}s "
            f"setup={info.setup_s:.2f}s it/s={info.iters / sec:.0f} rel_kkt(fp64)={info.rel_kkt:.2e} "
            f"pobj={info.pobj:.8g} primal={ks['primal_ms'] * 1e3:.1f}us dual={ks['dual_ms'] * 1e3:.1f}us "
            f"U(A)={ks['unroll_a']} U(At)={ks['unroll_at']}")
        hprlp.hpr_destroy(h)

    read_gbs, copy_gbs = hprlp.hpr_probe_stream(1 << 30, 20)
    log(f"stream probe: read {read_gbs:.0f} GB/s, copy {copy_gbs:.0f} GB/s")
    if args.precision != "both":
        log("single-precision leg only (profiler run): no JSON line")
        return
    f32, f64 = res["fp32"], res["fp64"]
    roof = roofline(lp, f32["ks"], workload, read_gbs, copy_gbs)


    batch = (batch_leg(args.batch, stream, args.batch_parent, not args.batch_no_seq, args.batch_max_iter,
                       args.batch_detail, args.stall_iters) if args.batch > 0 else None)
    warm = warmstart_leg(args.warmstart, max(args.batch, 16), stream) if args.warmstart > 0 else None
    mlp_out = mlp_leg(args.mlp_steps, stream) if args.mlp_steps > 0 else None
    sf = None
    if args.successive > 0 and args.formulation == "compact":
        from paper_2510_10891_amd import successive
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = successive.run(data, lp, rounds=args.successive, tau=0.1,
                           opts=hprlp.Options(tol=1e-4, precision=hprlp.HPR_FP32, max_iter=200000, stream=stream),
                           log=lambda m: log(f"successive fixing {m}"))
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        sf = dict(workload=f"{workload}: {args.successive} rounds of solve, Algorithm 1 on the device, Fix and "
                           f"LP-Presolve (fixed columns substituted), warm-started re-solves, tau 0.1, FP32",
                  total_s=round(total, 3),
                  rounds=[dict(round=x.index, term=x.term, iters=x.iters, solve_s=round(x.solve_s, 3),
                               setup_s=round(x.setup_s, 3), n=x.n, m=x.m, nnz=x.nnz, objective=x.objective,
                               fixed_u=round(x.fixed_u, 4), newly_fixed=x.newly_fixed) for x in r.rounds])
        log(f"successive fixing: {sf}")
    large = large_leg(args.large_steps, stream, read_gbs, copy_gbs) if args.large_steps > 0 else None

    abl = ablation_leg(data, args.ablation, stream, args.formulation) if args.ablation > 0 else None

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(lp, f64["info"].iters, args.cpu_limit,
                           {"fp32": f32["info"].pobj, "fp64": f64["info"].pobj})
        log(f"cpu baseline: {cpu}")

    rel_obj = abs(f32["info"].pobj - f64["info"].pobj) / max(1.0, abs(f64["info"].pobj))
    exact = None
    gold = os.path.join(ROOT, "tests", "golden", f"highs_{args.config}_seed{args.seed}.json")
    if os.path.exists(gold) and args.formulation == "compact":
        g = json.load(open(gold))
        if (g["m"], g["n"], g["nnz"]) == (lp.m, lp.n, lp.nnz):
            exact = dict(objective=g["objective"], source="HiGHS interior point (tests/golden)",
                         fp32_rel_err=abs(f32["info"].pobj - g["objective"]) / abs(g["objective"]),
                         fp64_rel_err=abs(f64["info"].pobj - g["objective"]) / abs(g["objective"]))
    out = {
        "metric": "time-to-1e-4 rel KKT (s)",
        "value": round(f32["sec"], 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["sec"] * 1e3, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 reductions",
        "data": "synthetic",
        "config": {"workload": workload, "m": lp.m, "n": lp.n, "nnz": lp.nnz, "tol": 1e-4,
                   "seed": args.seed, **({"presolve": presolve} if presolve else {})},
        "iters": f32["info"].iters,
        "iters_per_s": round(f32["info"].iters / f32["sec"], 1),
        "setup_s": round(f32["info"].setup_s, 3),
        "setup_phases_s": f32["ks"]["setup_phases_s"],
        "setup_plus_solve_s": round(f32["info"].setup_s + f32["sec"], 3),
        "rel_kkt_fp64_eval": f32["info"].rel_kkt,
        "all_solved": all(i.term == "solved" for i in (f32["info"], f64["info"])),
        "fp64": {"value": round(f64["sec"], 5), "iters": f64["info"].iters,
                 "iters_per_s": round(f64["info"].iters / f64["sec"], 1),
                 "rel_kkt_fp64_eval": f64["info"].rel_kkt,
                 "dual_us": round(f64["ks"]["dual_ms"] * 1e3, 2),
                 "primal_us": round(f64["ks"]["primal_ms"] * 1e3, 2)},
        "objective_vs_exact": exact,
        "fp32_vs_fp64": {"speedup": round(f64["sec"] / f32["sec"], 3), "obj_rel_diff": rel_obj,
                         "x_rel_diff": float(np.linalg.norm(f32["x"] - f64["x"]) /
                                             max(1e-30, np.linalg.norm(f64["x"])))},
        "roofline": roof,
        "batch": batch,
        "warm_start": warm,
        "mlp": mlp_out,
        "successive_fixing": sf,
        "large": large,
        "ablation": abl,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
