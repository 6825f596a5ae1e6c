// gfx950 kernels of the LP iteration that are not matrix products: fixed-order sums of the
// check partials, the per-LP control of the checks (restart, sigma, termination), segmented
// vector kernels of the power method, and the instantiations of the bookkeeping operations
// (restart copies, unscaling, casts). The fused matrix-product kernels are in
// csr.h, instantiated in the kernels_*.hip files.
#include "csr.h"

namespace hpr {

// ---------------------------------------------------------------- sums and control

// block (q, l): fixed-order sum of partials[q][seg[l] .. seg[l+1])
__global__ __launch_bounds__(kBlock) void finish_sums_kernel(const double* partials, int nb, const int32_t* seg,
                                                             double* out, int off) {
    __shared__ double sh[kBlock];
    const int q = blockIdx.x, l = blockIdx.y;
    const double* p = partials + (size_t)q * nb;
    double s = 0.0;
    for (int i = seg[l] + threadIdx.x; i < seg[l + 1]; i += kBlock) s += p[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)l * kSumStride + off + q] = sh[0];
}

struct CheckValues {
    double rel_p, rel_d, rel_gap, rel_kkt, pobj, dobj, merit, move_x, move_y;
    bool bad;
    bool infeasible;   // ybar is a primal infeasibility certificate
    bool unbounded;    // the step's primal move is a ray: the LP has no finite optimum
};

// The relative KKT residuals of the original problem and the merit from the check sums
// (see CheckRowsOp / CheckColsOp). Written without FMA contraction so that the device
// takes the same decisions as an IEEE host evaluation of the same formulas.
__device__ CheckValues check_values(const double* s, const Ctrl& c, const LpState& S, double ray_tol) {
#pragma clang fp contract(off)
    const double* r = s;
    const double* k = s + kColOff;
    CheckValues v;
    const double bb = c.beta_b * c.beta_c;
    v.rel_p = sqrt(r[0]) / (1.0 + S.norm_b);
    v.rel_d = sqrt(k[0]) / (1.0 + S.norm_c);
    v.pobj = bb * k[1] + S.obj_offset;
    v.dobj = bb * (r[3] + k[2]) + S.obj_offset;
    v.rel_gap = fabs(v.pobj - v.dobj) / (1.0 + fabs(v.pobj) + fabs(v.dobj));
    v.rel_kkt = fmax(v.rel_p, fmax(v.rel_d, v.rel_gap));
    const double r2 = k[3] / c.sigma + c.lambda * c.sigma * r[1] + 2.0 * r[2];
    v.merit = sqrt(r2 > 0.0 ? r2 : 0.0);
    v.move_x = sqrt(k[4]);
    v.move_y = sqrt(r[4]);
    v.bad = (r[5] + k[5]) > 0.0 || isnan(v.rel_p) || isnan(v.rel_d) || isnan(v.rel_gap) ||
            !isfinite(v.rel_kkt) || !isfinite(v.pobj) || !isfinite(v.merit);
    // For a feasible LP, h(y) = sum lo_i y_i+ - hi_i y_i- + sum l_j dz_j+ - u_j dz_j- with
    // dz = -A^T y is <= 0 for every sign-feasible y (it is bounded by y'Ax - y'Ax = 0), so
    // h(ybar) > 0 certifies primal infeasibility; margins relative to the terms' magnitude.
    const double h = r[3] + k[6], mag = r[6] + k[7];
    v.infeasible = h > kInfeasTol * mag && k[8] <= kInfeasTol * r[7];
    // A direction d with c~'d < 0 inside the rows' and columns' recession cones shows that the
    // dual has no feasible point; d = the step's primal move, accepted when its cone violations
    // are at most ray_tol of the cost decrease in units of d.
    const double g = k[9], vr = sqrt(r[8]), vc = sqrt(k[10]), nc = sqrt(k[11]);
    v.unbounded = g < 0.0 && nc > 0.0 && vr + vc <= ray_tol * (-g / nc);
    return v;
}

__device__ void store_values(LpState& S, const CheckValues& v) {
    S.rel_p = v.rel_p;
    S.rel_d = v.rel_d;
    S.rel_gap = v.rel_gap;
    S.rel_kkt = v.rel_kkt;
    S.pobj = v.pobj;
    S.dobj = v.dobj;
    S.merit = v.merit;
}

// After a check that did not terminate: iteration limit, then the restart rule:
// restart when r <= 0.2 r0, or r <= 0.8 r0 while rising (r > r_prev), or when the
// iterations since the last restart are >= 0.2 of all iterations. At a restart
// log sigma <- (1 - w) log sigma + w log sigma* (w = sigma_smoothing, or sigma_smoothing_warm for
// an LP started from the caller's point; w = 1 is sigma <- sigma*, w = 1/2 is sigma <- sqrt(sigma
// sigma*)), sigma* = ||dx|| / (sqrt(lambda) ||dy||) from the anchor
// move (skipped below 1e-12), clamped to [1e-4, 1e4]; anchor = iterate = bar point, k = 0.
__device__ void decide(LpState& S, Ctrl& c, const ControlArgs& a, double r, double move_x, double move_y) {
#pragma clang fp contract(off)
    if (S.it >= a.max_iter) {
        S.term = 2;   // HPR_ITER_LIMIT
        c.active = 0;
        return;
    }
    if (S.it == 1) {
        S.r0 = r;
        S.r_prev = r;
        c.k_base = S.k;
        return;
    }
    bool do_restart = false;
    if (a.restart_rule) {
        if (r <= 0.2 * S.r0) do_restart = true;
        else if (r <= 0.8 * S.r0 && r > S.r_prev) do_restart = true;
        else if ((double)S.k >= 0.2 * (double)S.it) do_restart = true;
    }
    if (do_restart) {
        double sigma = c.sigma;
        if (a.sigma_update && move_x > 1e-12 && move_y > 1e-12) {
            const double star = move_x / (sqrt(c.lambda) * move_y);
            const double w = S.warm ? a.sigma_smoothing_warm : a.sigma_smoothing;
            sigma = (w == 1.0)   ? star
                  : (w == 0.5) ? sqrt(sigma * star)
                               : exp((1.0 - w) * log(sigma) + w * log(star));
            sigma = sigma < 1e-4 ? 1e-4 : (sigma > 1e4 ? 1e4 : sigma);
        }
        c.sigma = sigma;
        c.s = 1.0 / (c.lambda * sigma);
        c.restart = 1;
        S.k = 0;
        S.restarts += 1;
        S.r0 = r;
    }
    S.r_prev = r;
    c.k_base = S.k;
}

// FP32 storage only: an LP has stalled when its check rel_kkt has not fallen to half the value
// it had at the last such halving while the iteration count since then reached the count at
// that halving (and at least stall_iters): FP32 rounding of A~ and of the iterates sets a floor
// on the residuals that FP64 storage does not have.
__device__ bool stalled(LpState& S, double rel_kkt, int64_t stall_iters) {
    if (rel_kkt <= 0.5 * S.mark_kkt) {
        S.mark_kkt = rel_kkt;
        S.mark_it = S.it;
        return false;
    }
    const int64_t since = S.it - S.mark_it;
    return since >= stall_iters && since >= S.mark_it;
}

__global__ __launch_bounds__(kMaxBatch) void control_kernel(ControlArgs a) {
    __shared__ int n_run, n_cand;
    if (threadIdx.x == 0) {
        n_run = 0;
        n_cand = 0;
    }
    __syncthreads();
    const int l = threadIdx.x;
    // the ray of the dual infeasibility test is a difference of iterates that grow along it: in
    // FP32 storage it carries their rounding (2^-24 of their size), so it is judged at 1e-3
    const double ray_tol = a.fp32 ? kRayTol32 : kInfeasTol;
    if (l < a.nlp) {
        Ctrl c = a.ctrl[l];
        LpState S = a.st[l];
        if (a.phase == 1) {
            c.restart = 0;
            if (c.active) {
                S.it += a.nb;
                S.k += a.nb;
                const CheckValues v = check_values(a.sums + (size_t)l * kSumStride, c, S, ray_tol);
                store_values(S, v);
                if (v.bad) {
                    S.term = 4;   // HPR_NUMERIC_FAIL
                    c.active = 0;
                } else if (v.rel_kkt <= a.tol || v.infeasible || v.unbounded) {
                    if (!a.fp32) {   // HPR_SOLVED, HPR_PRIMAL_INFEASIBLE, HPR_DUAL_INFEASIBLE
                        S.term = v.rel_kkt <= a.tol ? 1 : (v.infeasible ? 5 : 6);
                        c.active = 0;
                    } else {   // FP32 storage: confirmed (or not) by the FP64 re-evaluation
                        S.candidate = 1;
                        S.p32[0] = v.merit;
                        S.p32[1] = v.move_x;
                        S.p32[2] = v.move_y;
                    }
                } else if (a.fp32 && a.stall_iters > 0 && S.it < a.max_iter && stalled(S, v.rel_kkt, a.stall_iters)) {
                    S.term = 7;   // HPR_STALLED
                    c.active = 0;
                } else {
                    decide(S, c, a, v.merit, v.move_x, v.move_y);
                }
            }
        } else if (a.phase == 2) {
            c.restart = 0;
            if (c.active && S.candidate) {
                S.candidate = 0;
                const CheckValues v = check_values(a.sums64 + (size_t)l * kSumStride, c, S, ray_tol);
                if (!v.bad && (v.rel_kkt <= a.tol || v.infeasible || v.unbounded)) {
                    store_values(S, v);
                    S.term = v.rel_kkt <= a.tol ? 1 : (v.infeasible ? 5 : 6);
                    c.active = 0;
                } else if (!v.bad && a.stall_iters > 0 && S.it < a.max_iter && stalled(S, v.rel_kkt, a.stall_iters)) {
                    S.term = 7;   // HPR_STALLED
                    c.active = 0;
                } else {
                    decide(S, c, a, S.p32[0], S.p32[1], S.p32[2]);
                }
            }
        } else if (a.phase == 3) {
            if (S.term != 4) {
                const CheckValues v = check_values(a.sums64 + (size_t)l * kSumStride, c, S, ray_tol);
                S.rel_p = v.rel_p;
                S.rel_d = v.rel_d;
                S.rel_gap = v.rel_gap;
                S.rel_kkt = v.rel_kkt;
                S.pobj = v.pobj;
                S.dobj = v.dobj;
            }
        } else if (a.phase == 4) {
            c.restart = 0;
            if (c.active) {
                S.term = 3;   // HPR_TIME_LIMIT
                c.active = 0;
                S.candidate = 0;
            }
        }
        a.ctrl[l] = c;
        a.st[l] = S;
        if (c.active) atomicAdd(&n_run, 1);
        if (S.candidate) atomicAdd(&n_cand, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.stat[0] = n_run;
        a.stat[1] = n_cand;
    }
}

// ---------------------------------------------------------------- segmented vector kernels

__device__ __forceinline__ uint64_t splitmix64_draw(uint64_t seed, uint64_t i) {
    // SplitMix64 (Steele, Lea and Flood 2014) as a counter-based generator: draw i is the
    // finaliser applied to seed + (i + 1) * 0x9E3779B97F4A7C15.
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// grid (max_chunks, nlp): block (c, l) covers entries seg[l] + c*kChunk .. of LP l
__global__ __launch_bounds__(kBlock) void seg_sumsq_kernel(const double* v, const int64_t* seg, int max_chunks,
                                                           double* partials) {
    const int c = blockIdx.x, l = blockIdx.y;
    const int64_t b = seg[l] + (int64_t)c * kChunk;
    const int64_t e = b + kChunk < seg[l + 1] ? b + kChunk : seg[l + 1];
    double s = 0.0;
    for (int64_t i = b + threadIdx.x; i < e; i += kBlock) s += v[i] * v[i];
    __shared__ double sh[kBlock / 64];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
        partials[(size_t)l * max_chunks + c] = t;
    }
}

__global__ __launch_bounds__(kBlock) void seg_start_kernel(double* v, const int64_t* seg, uint64_t seed) {
    const int c = blockIdx.x, l = blockIdx.y;
    const int64_t b = seg[l] + (int64_t)c * kChunk;
    const int64_t e = b + kChunk < seg[l + 1] ? b + kChunk : seg[l + 1];
    for (int64_t i = b + threadIdx.x; i < e; i += kBlock) {
        const uint64_t r = splitmix64_draw(seed, (uint64_t)(i - seg[l]));
        v[i] = 2.0 * (double(r >> 11) * 0x1.0p-53) - 1.0;
    }
}

__global__ __launch_bounds__(kBlock) void seg_scale_kernel(double* v, const int64_t* seg, const double* f) {
    const int c = blockIdx.x, l = blockIdx.y;
    const int64_t b = seg[l] + (int64_t)c * kChunk;
    const int64_t e = b + kChunk < seg[l + 1] ? b + kChunk : seg[l + 1];
    const double s = f[l];
    for (int64_t i = b + threadIdx.x; i < e; i += kBlock) v[i] *= s;
}

void launch_finish_sums(const double* partials, int nq, int nblocks, const int32_t* seg, int nlp, double* out,
                        int off, hipStream_t st) {
    if (nq <= 0 || nlp <= 0) return;
    hipLaunchKernelGGL(finish_sums_kernel, dim3(nq, nlp), dim3(kBlock), 0, st, partials, nblocks, seg, out, off);
}

void launch_control(const ControlArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(control_kernel, dim3(1), dim3(kMaxBatch), 0, st, a);
}

void launch_seg_sumsq(const double* v, const int64_t* seg, int nlp, int max_chunks, double* partials,
                      hipStream_t st) {
    if (nlp <= 0 || max_chunks <= 0) return;
    hipLaunchKernelGGL(seg_sumsq_kernel, dim3(max_chunks, nlp), dim3(kBlock), 0, st, v, seg, max_chunks, partials);
}

void launch_seg_start_vector(double* v, const int64_t* seg, int nlp, int max_chunks, uint64_t seed,
                             hipStream_t st) {
    if (nlp <= 0 || max_chunks <= 0) return;
    hipLaunchKernelGGL(seg_start_kernel, dim3(max_chunks, nlp), dim3(kBlock), 0, st, v, seg, seed);
}

// ---------------------------------------------------------------- fixing (Section IV)

// Round (Section IV-A) and the Fixing-Strategy of Algorithm 1, one thread per unit g. Each
// hour's (u, v, w) value, x[col] for a column of the LP or fixval[entry] for one that a presolve
// removed (col < 0), is rounded with threshold tau: 1 if s >= 1 - tau, 0 if 0 <= s <= tau, else
// -1. Then, from the second hour on, an hour is fixed while the four rounded values it reads
// (u_t, u_{t-1}, v_t, w_t) are all confident and satisfy u_t - u_{t-1} = v_t - w_t and
// v_t + w_t <= 1; the first hour that fails ends the unit's loop (the first hour is never fixed).
// Layout: cols, fixval and rounded [G][T][3], fixed [G][T].
__device__ __forceinline__ int8_t round_tau(double s, double tau) {
    if (s >= 1.0 - tau) return 1;
    if (s >= 0.0 && s <= tau) return 0;
    return -1;
}

__global__ __launch_bounds__(kBlock) void fix_strategy_kernel(const double* x, const int32_t* cols,
                                                              const double* fixval, int G, int T, double tau,
                                                              int8_t* fixed, int8_t* rounded) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int64_t base = (int64_t)g * T;
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < 3; ++k) {
            const int64_t e = (base + t) * 3 + k;
            const int32_t c = cols[e];
            rounded[e] = round_tau(c >= 0 ? x[c] : fixval[e], tau);
        }
    fixed[base] = 0;
    bool on = true;
    for (int t = 1; t < T; ++t) {
        const int8_t* r = rounded + (base + t) * 3;
        const int u = r[0], v = r[1], w = r[2], u_prev = rounded[(base + t - 1) * 3];
        on = on && u >= 0 && u_prev >= 0 && v >= 0 && w >= 0 && u - u_prev == v - w && v + w <= 1;
        fixed[base + t] = on ? 1 : 0;
    }
}

void launch_fix_strategy(const double* x, const int32_t* cols, const double* fixval, int G, int T, double tau,
                         int8_t* fixed, int8_t* rounded, hipStream_t st) {
    if (G <= 0 || T <= 0) return;
    hipLaunchKernelGGL(fix_strategy_kernel, dim3((unsigned)((G + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, x,
                       cols, fixval, G, T, tau, fixed, rounded);
}

// power method: per LP, the norm s = sqrt(sums[l * kSumStride]) into hist[l] and the factor 1 / s
// (1 when s = 0) that normalises the vector, without a round trip to the host
__global__ __launch_bounds__(kMaxBatch) void power_norms_kernel(const double* sums, int nlp, double* hist,
                                                                double* fac) {
    const int l = threadIdx.x;
    if (l >= nlp) return;
    const double s = sqrt(sums[(size_t)l * kSumStride]);
    hist[l] = s;
    fac[l] = s > 0.0 ? 1.0 / s : 1.0;
}

void launch_power_norms(const double* sums, int nlp, double* hist, double* fac, hipStream_t st) {
    if (nlp <= 0) return;
    hipLaunchKernelGGL(power_norms_kernel, dim3(1), dim3(kMaxBatch), 0, st, sums, nlp, hist, fac);
}

void launch_seg_scale(double* v, const int64_t* seg, int nlp, int max_chunks, const double* factor,
                      hipStream_t st) {
    if (nlp <= 0 || max_chunks <= 0) return;
    hipLaunchKernelGGL(seg_scale_kernel, dim3(max_chunks, nlp), dim3(kBlock), 0, st, v, seg, factor);
}

// Packed quads: quad q (entries 4q..4q+3) of a narrow row, whose entries are in column order,
// gets bit 31, its first offset (13 bits) and the three gaps to the next entries (6 bits each)
// when they fit; quads of wide rows and the others get 0 (read from col16). The row of a quad is
// found by bisection of the row starts. count[0] += narrow quads, count[1] += packed.
__global__ __launch_bounds__(kBlock) void pack_quads_kernel(const uint16_t* col16, const int64_t* start,
                                                            const uint8_t* wide, int32_t rows, int64_t nquads,
                                                            uint32_t* qpack, unsigned long long* count) {
    __shared__ unsigned n_narrow, n_packed;
    if (threadIdx.x == 0) n_narrow = n_packed = 0;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned narrow = 0, packed = 0;
    if (q < nquads) {
        const int64_t k = 4 * q;
        int32_t lo = 0, hi = rows - 1;                 // last row with start <= k
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (start[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        uint32_t w = 0;
        if (!wide[lo] && k < start[lo + 1]) {
            narrow = 1;
            const uint32_t c0 = col16[k], c1 = col16[k + 1], c2 = col16[k + 2], c3 = col16[k + 3];
            if (c0 < 8192u && c1 >= c0 && c2 >= c1 && c3 >= c2 && c1 - c0 < 64u && c2 - c1 < 64u && c3 - c2 < 64u) {
                w = 0x80000000u | c0 | ((c1 - c0) << 13) | ((c2 - c1) << 19) | ((c3 - c2) << 25);
                packed = 1;
            }
        }
        qpack[q] = w;
    }
    if (narrow) atomicAdd(&n_narrow, narrow);
    if (packed) atomicAdd(&n_packed, packed);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (n_narrow) atomicAdd(count, (unsigned long long)n_narrow);
        if (n_packed) atomicAdd(count + 1, (unsigned long long)n_packed);
    }
}

void launch_pack_quads(const uint16_t* col16, const int64_t* start, const uint8_t* wide, int32_t rows,
                       int64_t nquads, uint32_t* qpack, unsigned long long* count, hipStream_t st) {
    if (nquads <= 0 || rows <= 0) return;
    hipLaunchKernelGGL(pack_quads_kernel, dim3((unsigned)((nquads + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       col16, start, wide, rows, nquads, qpack, count);
}

// ---------------------------------------------------------------- instantiations

#define HPR_INST(T)                                                                                          \
    template void launch_restart<T>(const DevCsr<T>&, const DevCsr<T>&, const DevIter<T>&, const Ctrl*,      \
                                    hipStream_t);                                                            \
    template void launch_unscale<T>(const DevCsr<T>&, const DevCsr<T>&, const DevIter<T>&, const double*,    \
                                    const double*, const Ctrl*, double*, double*, double*, hipStream_t);     \
    template void launch_cast<T>(const double*, T*, int64_t, hipStream_t);

HPR_INST(double)
HPR_INST(float)

}  // namespace hpr
