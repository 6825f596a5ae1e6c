// gfx950 kernels of the LP iteration: binned CSR products fused with the primal and
// dual projection steps of eq.(hpr), FP64 check reductions, and small helpers.
//
// Every matrix product walks one stored row per group of G lanes (G = 1..64 by row
// length). A lane loads quads of 4 values and 4 column indices with 16-byte loads, U
// quads at a time, gathers the vector entries, and the G partial sums are combined with
// cross-lane shuffles in a fixed order, so results are bitwise repeatable for a given
// schedule (G per row and U per matrix).
#include "internal.h"

#include <math.h>

namespace hpr {

// ---------------------------------------------------------------- loads

template <typename T>
struct Quad;

template <>
struct Quad<float> {
    float a[4];
    __device__ __forceinline__ static Quad load(const float* p) {
        float4 v = *reinterpret_cast<const float4*>(p);
        return Quad{{v.x, v.y, v.z, v.w}};
    }
};

template <>
struct Quad<double> {
    double a[4];
    __device__ __forceinline__ static Quad load(const double* p) {
        double2 v0 = *reinterpret_cast<const double2*>(p);
        double2 v1 = *reinterpret_cast<const double2*>(p + 2);
        return Quad{{v0.x, v0.y, v1.x, v1.y}};
    }
};

__device__ __forceinline__ int4 load_idx(const int32_t* p) { return *reinterpret_cast<const int4*>(p); }

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Dot products of stored row [b, e) with one or two gathered vectors. Lane `lane` of a
// group of G lanes takes quads b + 4*(lane + G*t); each pass issues the loads of U quads
// before any gather so U 16-byte loads per array are in flight per lane.
template <int G, int U, int NV, typename Tm, typename Tx, typename Acc>
__device__ __forceinline__ void group_dot(const DevCsr<Tm>& A, int64_t b, int64_t e, int lane,
                                          const Tx* __restrict__ g0, const Tx* __restrict__ g1,
                                          Acc& s0, Acc& s1) {
    s0 = Acc(0);
    s1 = Acc(0);
    for (int64_t p = b + kVec * lane; p < e; p += (int64_t)kVec * G * U) {
        int4 c[U];
        Quad<Tm> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + (int64_t)kVec * G * u;
            if (q < e) {
                c[u] = load_idx(A.col + q);
                v[u] = Quad<Tm>::load(A.val + q);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + (int64_t)kVec * G * u;
            if (q < e) {
                s0 += Acc(v[u].a[0]) * Acc(g0[c[u].x]) + Acc(v[u].a[1]) * Acc(g0[c[u].y]) +
                      Acc(v[u].a[2]) * Acc(g0[c[u].z]) + Acc(v[u].a[3]) * Acc(g0[c[u].w]);
                if constexpr (NV == 2) {
                    s1 += Acc(v[u].a[0]) * Acc(g1[c[u].x]) + Acc(v[u].a[1]) * Acc(g1[c[u].y]) +
                          Acc(v[u].a[2]) * Acc(g1[c[u].z]) + Acc(v[u].a[3]) * Acc(g1[c[u].w]);
                }
            }
        }
    }
}

// One block of bin `bin`: each group of G lanes takes one row of the bin's row list.
template <int G, int U, typename Op>
__device__ __forceinline__ void run_bin(const DevCsr<typename Op::Tm>& A, Op& op, int bin, int lb) {
    using Acc = typename Op::Acc;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int r = lb * (kBlock / G) + grp;
    const bool active = r < A.bins.nrows[bin];
    const int row = active ? A.rows[A.bins.row_off[bin] + r] : 0;
    const int64_t b = active ? A.start[row] : 0;
    const int64_t e = active ? A.start[row + 1] : 0;
    Acc s0, s1;
    group_dot<G, U, Op::NV>(A, b, e, lane, op.g0, op.g1, s0, s1);
    s0 = group_sum<G>(s0);
    if constexpr (Op::NV == 2) s1 = group_sum<G>(s1);
    if (active && lane == 0) op.epi(row, s0, s1);
}

template <int NQ>
__device__ __forceinline__ void block_reduce_store(double (&q)[NQ], double* partials) {
    __shared__ double sh[kBlock / 64][NQ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        double v = wave_sum(q[k]);
        if (lane == 0) sh[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
        partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

template <typename Op, int U>
__global__ __launch_bounds__(kBlock) void csr_kernel(DevCsr<typename Op::Tm> A, Op op_in) {
    Op op = op_in;
    op.init();
    const int blk = blockIdx.x;
    int bin = 0;
#pragma unroll
    for (int b = 1; b < kNumBins; ++b)
        if (blk >= A.bins.block_off[b]) bin = b;
    const int lb = blk - A.bins.block_off[bin];
    switch (bin) {
        case 0: run_bin<1, U>(A, op, bin, lb); break;
        case 1: run_bin<2, U>(A, op, bin, lb); break;
        case 2: run_bin<4, U>(A, op, bin, lb); break;
        case 3: run_bin<8, U>(A, op, bin, lb); break;
        case 4: run_bin<16, U>(A, op, bin, lb); break;
        case 5: run_bin<32, U>(A, op, bin, lb); break;
        default: run_bin<64, U>(A, op, bin, lb); break;
    }
    if constexpr (Op::NQ > 0) block_reduce_store(op.q, op.partials);
}

template <typename Op>
static void launch_csr(const DevCsr<typename Op::Tm>& A, const Op& op, hipStream_t st) {
    const int nb = A.bins.block_off[kNumBins];
    if (nb <= 0) return;
    switch (A.unroll) {
        case 1: hipLaunchKernelGGL((csr_kernel<Op, 1>), dim3(nb), dim3(kBlock), 0, st, A, op); break;
        case 2: hipLaunchKernelGGL((csr_kernel<Op, 2>), dim3(nb), dim3(kBlock), 0, st, A, op); break;
        case 8: hipLaunchKernelGGL((csr_kernel<Op, 8>), dim3(nb), dim3(kBlock), 0, st, A, op); break;
        default: hipLaunchKernelGGL((csr_kernel<Op, 4>), dim3(nb), dim3(kBlock), 0, st, A, op); break;
    }
}

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------- eq.(hpr), primal half

// Over the rows of A^T (= columns of A): with g = (A^T y)_j,
//   w = x_j + sigma (g - c_j),  xbar = Pi_[l,u](w),  xhat = 2 xbar - x_j,
//   x_j <- x0_j / (k+2) + (k+1)/(k+2) xhat;  at a check also xbar, zbar = (xbar - w)/sigma,
//   and x_j - xbar are stored.
template <typename T>
struct PrimalOp {
    using Tm = T;
    using Acc = T;
    static constexpr int NV = 1, NQ = 0;
    const T* g0;
    const T* g1;
    DevProb<T> p;
    DevIter<T> v;
    const Ctrl* ctrl;
    int j;
    int check;
    T sigma, a0, a1;
    double q[1];
    double* partials;
    __device__ __forceinline__ void init() {
        const int64_t k = ctrl->k_base + j;
        sigma = T(ctrl->sigma);
        a0 = T(1.0 / double(k + 2));
        a1 = T(double(k + 1) / double(k + 2));
    }
    __device__ __forceinline__ void epi(int col, T aty, T) {
        const T xk = v.x[col];
        const T w = xk + sigma * (aty - p.c[col]);
        const T xb = clampv(w, p.l[col], p.u[col]);
        const T xh = T(2) * xb - xk;
        v.xh[col] = xh;
        v.x[col] = a0 * v.x0[col] + a1 * xh;
        if (check) {
            v.xb[col] = xb;
            v.zb[col] = (xb - w) / sigma;
            v.dx[col] = xk - xb;
        }
    }
};

// ---------------------------------------------------------------- eq.(hpr), dual half

// Over the rows of A: with g = (A xhat)_i and s = 1/(lambda sigma), vv = y_i - s g,
//   ybar = vv + s lo_i if > 0;  vv + s hi_i if < 0;  else 0
// (for hi = +inf this is Pi_+(y + s(theta - A xhat)) of eq.(hpr)),
//   y_i <- y0_i / (k+2) + (k+1)/(k+2) (2 ybar - y_i);  at a check ybar and y_i - ybar are stored.
template <typename T>
struct DualOp {
    using Tm = T;
    using Acc = T;
    static constexpr int NV = 1, NQ = 0;
    const T* g0;
    const T* g1;
    DevProb<T> p;
    DevIter<T> v;
    const Ctrl* ctrl;
    int j;
    int check;
    T s, a0, a1;
    double q[1];
    double* partials;
    __device__ __forceinline__ void init() {
        const int64_t k = ctrl->k_base + j;
        s = T(ctrl->s);
        a0 = T(1.0 / double(k + 2));
        a1 = T(double(k + 1) / double(k + 2));
    }
    __device__ __forceinline__ void epi(int row, T ax, T) {
        const T yk = v.y[row];
        const T vv = yk - s * ax;
        const T up = vv + s * p.lo[row];
        const T dn = vv + s * p.hi[row];
        const T yb = up > T(0) ? up : (dn < T(0) ? dn : T(0));
        const T yh = T(2) * yb - yk;
        v.y[row] = a0 * v.y0[row] + a1 * yh;
        if (check) {
            v.yb[row] = yb;
            v.dy[row] = yk - yb;
        }
    }
};

// ---------------------------------------------------------------- FP64 checks

// Row side, over the rows of A with (A xbar)_i and (A dx)_i:
//   q0 = sum (beta_b/dr_i * max(lo_i - a, 0, a - hi_i))^2   (unscaled primal residual)
//   q1 = sum dy_i^2, q2 = sum dy_i (A dx)_i                 (merit terms)
//   q3 = sum lo_i ybar_i+ - hi_i ybar_i-                      (scaled dual objective, rows)
//   q4 = sum (ybar_i - y0_i)^2                                (anchor move)
//   q5 = number of non-finite values
template <typename M, typename P, typename V>
struct CheckRowsOp {
    using Tm = M;
    using Acc = M;
    static constexpr int NV = 2, NQ = kRowQ;
    const V* g0;
    const V* g1;
    DevProb<P> p;
    DevIter<V> v;
    double beta_b;
    double q[NQ];
    double* partials;
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[k] = 0.0;
    }
    __device__ __forceinline__ void epi(int row, M ax, M adx) {
        const double a = double(ax);
        const double lo = double(p.lo[row]), hi = double(p.hi[row]);
        double r = 0.0;
        if (lo - a > r) r = lo - a;
        if (a - hi > r) r = a - hi;
        const double ru = r * beta_b / p.dr[row];
        q[0] += ru * ru;
        const double dy = double(v.dy[row]);
        q[1] += dy * dy;
        q[2] += dy * double(adx);
        const double yb = double(v.yb[row]);
        if (yb > 0.0) q[3] += lo * yb;
        else if (yb < 0.0) q[3] += hi * yb;
        const double d0 = yb - double(v.y0[row]);
        q[4] += d0 * d0;
        if (!isfinite(a) || !isfinite(yb) || !isfinite(double(adx)) || !isfinite(dy)) q[5] += 1.0;
    }
};

// Column side, over the rows of A^T with (A^T ybar)_j:
//   q0 = sum (beta_c/dc_j * (c_j - (A^T ybar)_j - zbar_j))^2   (unscaled dual residual)
//   q1 = sum c_j xbar_j                                        (scaled primal objective)
//   q2 = sum l_j zbar_j+ - u_j zbar_j-                          (scaled dual objective, columns)
//   q3 = sum dx_j^2,  q4 = sum (xbar_j - x0_j)^2,  q5 = non-finite count
template <typename M, typename P, typename V>
struct CheckColsOp {
    using Tm = M;
    using Acc = M;
    static constexpr int NV = 1, NQ = kColQ;
    const V* g0;
    const V* g1;
    DevProb<P> p;
    DevIter<V> v;
    double beta_c;
    double q[NQ];
    double* partials;
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[k] = 0.0;
    }
    __device__ __forceinline__ void epi(int col, M aty, M) {
        const double c = double(p.c[col]);
        const double zb = double(v.zb[col]);
        const double rd = c - double(aty) - zb;
        const double rdu = rd * beta_c / p.dc[col];
        q[0] += rdu * rdu;
        const double xb = double(v.xb[col]);
        q[1] += c * xb;
        if (zb > 0.0) q[2] += double(p.l[col]) * zb;
        else if (zb < 0.0) q[2] += double(p.u[col]) * zb;
        const double dx = double(v.dx[col]);
        q[3] += dx * dx;
        const double d0 = xb - double(v.x0[col]);
        q[4] += d0 * d0;
        if (!isfinite(double(aty)) || !isfinite(xb) || !isfinite(zb)) q[5] += 1.0;
    }
};

// ---------------------------------------------------------------- plain product

template <typename T>
struct SpmvOp {
    using Tm = T;
    using Acc = T;
    static constexpr int NV = 1, NQ = 0;
    const T* g0;
    const T* g1;
    T* out;
    double q[1];
    double* partials;
    __device__ __forceinline__ void init() {}
    __device__ __forceinline__ void epi(int row, T s, T) { out[row] = s; }
};

// ---------------------------------------------------------------- small kernels

// Fixed-order sum of partials[k][0..nb) for k = blockIdx.x.
__global__ __launch_bounds__(kBlock) void finish_sums_kernel(const double* partials, int nb, double* out) {
    __shared__ double sh[kBlock];
    const double* p = partials + (size_t)blockIdx.x * nb;
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) s += p[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

constexpr int kSumsqItems = 8192;   // entries per block of the sum-of-squares kernel

template <typename T>
__global__ __launch_bounds__(kBlock) void sumsq_kernel(const T* v, int64_t n, double* partials) {
    double q[1] = {0.0};
    const int64_t b = (int64_t)blockIdx.x * kSumsqItems;
    const int64_t e = b + kSumsqItems < n ? b + kSumsqItems : n;
    for (int64_t i = b + threadIdx.x; i < e; i += kBlock) {
        const double a = double(v[i]);
        q[0] += a * a;
    }
    block_reduce_store(q, partials);
}

template <typename T>
__global__ void scale_kernel(T* v, int64_t n, double f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = T(double(v[i]) * f);
}

// SplitMix64 (Steele, Lea and Flood 2014) as a counter-based generator: draw i is the
// finaliser applied to seed + (i + 1) * 0x9E3779B97F4A7C15; mapped to [-1, 1) from its top 53 bits.
__device__ __forceinline__ uint64_t splitmix64_draw(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void start_vector_kernel(T* v, int64_t n, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = T(2.0 * (double(splitmix64_draw(seed, (uint64_t)i) >> 11) * 0x1.0p-53) - 1.0);
}

template <typename T>
__global__ void restart_kernel(T* x0, T* x, const T* xb, int n, T* y0, T* y, const T* yb, int m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const T a = xb[i];
        x0[i] = a;
        x[i] = a;
    }
    if (i < m) {
        const T b = yb[i];
        y0[i] = b;
        y[i] = b;
    }
}

template <typename T>
__global__ void unscale_kernel(const T* xb, const T* zb, const T* yb, const double* dr, const double* dc, int n,
                               int m, double beta_b, double beta_c, double* x, double* y, double* z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        x[i] = beta_b * dc[i] * double(xb[i]);
        z[i] = beta_c * double(zb[i]) / dc[i];
    }
    if (i < m) y[i] = beta_c * dr[i] * double(yb[i]);
}

template <typename T>
__global__ void cast_kernel(const double* s, T* d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = T(s[i]);
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------- launchers

template <typename T>
void launch_primal_step(const DevCsr<T>& At, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                        int j, bool check, hipStream_t st) {
    PrimalOp<T> op{};
    op.g0 = v.y;
    op.p = p;
    op.v = v;
    op.ctrl = ctrl;
    op.j = j;
    op.check = check ? 1 : 0;
    launch_csr(At, op, st);
}

template <typename T>
void launch_dual_step(const DevCsr<T>& A, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                      int j, bool check, hipStream_t st) {
    DualOp<T> op{};
    op.g0 = v.xh;
    op.p = p;
    op.v = v;
    op.ctrl = ctrl;
    op.j = j;
    op.check = check ? 1 : 0;
    launch_csr(A, op, st);
}

template <typename Tm, typename Tp, typename Tv>
void launch_check_rows(const DevCsr<Tm>& A, const DevProb<Tp>& p, const DevIter<Tv>& v, double beta_b,
                       double* partials, hipStream_t st) {
    CheckRowsOp<Tm, Tp, Tv> op{};
    op.g0 = v.xb;
    op.g1 = v.dx;
    op.p = p;
    op.v = v;
    op.beta_b = beta_b;
    op.partials = partials;
    launch_csr(A, op, st);
}

template <typename Tm, typename Tp, typename Tv>
void launch_check_cols(const DevCsr<Tm>& At, const DevProb<Tp>& p, const DevIter<Tv>& v, double beta_c,
                       double* partials, hipStream_t st) {
    CheckColsOp<Tm, Tp, Tv> op{};
    op.g0 = v.yb;
    op.p = p;
    op.v = v;
    op.beta_c = beta_c;
    op.partials = partials;
    launch_csr(At, op, st);
}

void launch_finish_sums(const double* partials, int nq, int nblocks, double* out, hipStream_t st) {
    if (nq <= 0) return;
    hipLaunchKernelGGL(finish_sums_kernel, dim3(nq), dim3(kBlock), 0, st, partials, nblocks, out);
}

template <typename T>
void launch_spmv(const DevCsr<T>& A, const T* x, T* y, hipStream_t st) {
    SpmvOp<T> op{};
    op.g0 = x;
    op.out = y;
    launch_csr(A, op, st);
}

int sumsq_blocks(int64_t n) { return (int)((n + kSumsqItems - 1) / kSumsqItems); }

template <typename T>
void launch_sumsq(const T* v, int64_t n, double* partials, hipStream_t st) {
    const int nb = sumsq_blocks(n);
    if (nb <= 0) return;
    hipLaunchKernelGGL(sumsq_kernel<T>, dim3(nb), dim3(kBlock), 0, st, v, n, partials);
}

template <typename T>
void launch_scale(T* v, int64_t n, double factor, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_kernel<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, v, n, factor);
}

template <typename T>
void launch_start_vector(T* v, int64_t n, uint64_t seed, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(start_vector_kernel<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, v, n, seed);
}

template <typename T>
void launch_restart(const DevIter<T>& v, int n, int m, hipStream_t st) {
    const int len = n > m ? n : m;
    if (len <= 0) return;
    hipLaunchKernelGGL(restart_kernel<T>, dim3(grid_for(len)), dim3(kBlock), 0, st, v.x0, v.x, v.xb, n, v.y0,
                       v.y, v.yb, m);
}

template <typename T>
void launch_unscale(const DevIter<T>& v, const double* dr, const double* dc, int n, int m, double beta_b,
                    double beta_c, double* x, double* y, double* z, hipStream_t st) {
    const int len = n > m ? n : m;
    if (len <= 0) return;
    hipLaunchKernelGGL(unscale_kernel<T>, dim3(grid_for(len)), dim3(kBlock), 0, st, v.xb, v.zb, v.yb, dr, dc,
                       n, m, beta_b, beta_c, x, y, z);
}

template <typename T>
void launch_cast(const double* src, T* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(cast_kernel<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, src, dst, n);
}

// ---------------------------------------------------------------- instantiations

#define HPR_INST(T)                                                                                          \
    template void launch_primal_step<T>(const DevCsr<T>&, const DevProb<T>&, const DevIter<T>&, const Ctrl*, \
                                        int, bool, hipStream_t);                                             \
    template void launch_dual_step<T>(const DevCsr<T>&, const DevProb<T>&, const DevIter<T>&, const Ctrl*,   \
                                      int, bool, hipStream_t);                                               \
    template void launch_spmv<T>(const DevCsr<T>&, const T*, T*, hipStream_t);                              \
    template void launch_sumsq<T>(const T*, int64_t, double*, hipStream_t);                                  \
    template void launch_scale<T>(T*, int64_t, double, hipStream_t);                                         \
    template void launch_start_vector<T>(T*, int64_t, uint64_t, hipStream_t);                                \
    template void launch_restart<T>(const DevIter<T>&, int, int, hipStream_t);                               \
    template void launch_unscale<T>(const DevIter<T>&, const double*, const double*, int, int, double,       \
                                    double, double*, double*, double*, hipStream_t);                         \
    template void launch_cast<T>(const double*, T*, int64_t, hipStream_t);

HPR_INST(double)
HPR_INST(float)

#define HPR_INST_CHECK(M, P, V)                                                                             \
    template void launch_check_rows<M, P, V>(const DevCsr<M>&, const DevProb<P>&, const DevIter<V>&, double, \
                                             double*, hipStream_t);                                         \
    template void launch_check_cols<M, P, V>(const DevCsr<M>&, const DevProb<P>&, const DevIter<V>&, double, \
                                             double*, hipStream_t);

HPR_INST_CHECK(double, double, double)
HPR_INST_CHECK(float, float, float)
HPR_INST_CHECK(double, double, float)

}  // namespace hpr
