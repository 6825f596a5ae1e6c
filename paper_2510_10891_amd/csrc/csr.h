// Shared device code of the LP kernels: quad loads, lane-group sums, LDS windows of the
// gathered vector, the binned CSR kernel template and the fused operations run over it
// (primal and dual halves of eq.(hpr), FP64 check reductions, restart copies, unscaling,
// plain products), with their launchers. The explicit instantiations are spread over
// several translation units so that they compile in parallel.
//
// Every matrix product walks one stored row per group of G lanes (G = 1..64 by row
// length). A lane loads quads of 4 values (one 16-byte load) and their column indices
// (16-bit offsets from the row's smallest column, or 32-bit indices for rows spanning
// 65,536 columns or more), U quads at a time, gathers the vector entries (from an LDS
// window of the vector where the block has one, else from global memory), and the G
// partial sums are combined with cross-lane moves in a fixed order, so results are bitwise
// repeatable for a given schedule (G per row, U per matrix, window mode per block).
#ifndef HPR_CSR_H
#define HPR_CSR_H

#include "internal.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <type_traits>

namespace hpr {

// ---------------------------------------------------------------- loads

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// 16-byte loads of the matrix stream; NT = non-temporal (the stream is read once per
// iteration and is larger than the caches, so it need not displace the gathered vectors)
template <bool NT, typename V>
__device__ __forceinline__ V ld16(const V* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T>
struct Quad;

template <>
struct Quad<float> {
    float a[4];
    template <bool NT>
    __device__ __forceinline__ static Quad load(const float* p) {
        const f32x4 v = ld16<NT>(reinterpret_cast<const f32x4*>(p));
        return Quad{{v.x, v.y, v.z, v.w}};
    }
};

template <>
struct Quad<double> {
    double a[4];
    template <bool NT>
    __device__ __forceinline__ static Quad load(const double* p) {
        const f64x2 v0 = ld16<NT>(reinterpret_cast<const f64x2*>(p));
        const f64x2 v1 = ld16<NT>(reinterpret_cast<const f64x2*>(p + 2));
        return Quad{{v0.x, v0.y, v1.x, v1.y}};
    }
};

template <bool NT>
__device__ __forceinline__ int4 load_idx(const int32_t* p) {
    const i32x4 v = ld16<NT>(reinterpret_cast<const i32x4*>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// 4 column offsets of 16 bits (one 8-byte load) plus the row's base column
template <bool NT>
__device__ __forceinline__ int4 load_idx16(const uint16_t* p, int base) {
    u32x2 v;
    if constexpr (NT) v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    else v = *reinterpret_cast<const u32x2*>(p);
    return make_int4(base + (int)(v.x & 0xFFFFu), base + (int)(v.x >> 16), base + (int)(v.y & 0xFFFFu),
                     base + (int)(v.y >> 16));
}

// A packed quad (DevCsr::qpack, bit 31 set): the first entry's 13-bit offset and the three 6-bit
// gaps to the entries after it.
__device__ __forceinline__ int4 unpack_quad(uint32_t w, int base) {
    const int c0 = base + (int)(w & 0x1FFFu);
    const int c1 = c0 + (int)((w >> 13) & 63u);
    const int c2 = c1 + (int)((w >> 19) & 63u);
    return make_int4(c0, c1, c2, c2 + (int)((w >> 25) & 63u));
}

template <bool NT>
__device__ __forceinline__ uint32_t load_pack(const uint32_t* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Lane moves within rows of 16 lanes (DPP): each lane reads the value of the lane that the
// control word names (quad permutations, half-row and row mirrors).
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- lane 7 - i within each 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <- lane 15 - i within each 16 lanes

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xFFFFFFFFull), CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over each aligned group of G lanes, left in every lane of the group. Pairs first
// (lanes i and i^1, then quads, half-rows of 8, rows of 16 by DPP moves, which are exact
// because after each step every lane of a block holds the same value), then rows of 16 and
// 32 by cross-lane shuffles; a fixed tree, so the result is the same in every run.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (G >= 2) v += dpp_move<kDppXor1>(v);
    if constexpr (G >= 4) v += dpp_move<kDppXor2>(v);
    if constexpr (G >= 8) v += dpp_move<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_move<kDppMirror>(v);
    if constexpr (G >= 32) v += __shfl_xor(v, 16, G);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, G);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Where a gathered entry comes from. Global: g[c]. Window: w[c] (c already relative to the
// block's LDS window). Split: the LDS window for columns in [lo, lo + len), g elsewhere.
template <typename Tx>
struct FromGlobal {
    const Tx* __restrict__ g;
    __device__ __forceinline__ Tx operator()(int c) const { return g[c]; }
};
template <typename Tx>
using LdsPtr = const __attribute__((address_space(3))) Tx*;
template <typename Tx>
struct FromWindow {
    LdsPtr<Tx> w;
    __device__ __forceinline__ Tx operator()(int c) const { return w[c]; }
};
template <typename Tx>
struct FromSplit {
    LdsPtr<Tx> w;
    const Tx* __restrict__ g;
    int lo, len;
    __device__ __forceinline__ Tx operator()(int c) const {
        // an LDS read for every entry (clamped index) and a global read only outside the
        // window: two separate loads, which the compiler cannot merge into one flat load
        const unsigned r = (unsigned)(c - lo);
        const bool in = r < (unsigned)len;
        Tx x = w[in ? r : 0u];
        if (!in) x = g[c];
        return x;
    }
};

// Copies src[lo, lo + len) into the block's LDS window (16-byte copies when lo allows it; the
// vector's base is 256-byte aligned).
template <typename Tx>
__device__ __forceinline__ void copy_window(Tx* win, const Tx* src, int lo, int len) {
    constexpr int kPer = 16 / (int)sizeof(Tx);   // entries per 16-byte load
    int t0 = 0;
    if (lo % kPer == 0) {
        const int n16 = len / kPer;
        const int4* s16 = reinterpret_cast<const int4*>(src + lo);
        int4* d16 = reinterpret_cast<int4*>(win);
        for (int t = threadIdx.x; t < n16; t += kBlock) d16[t] = s16[t];
        t0 = n16 * kPer;
    }
    for (int t = t0 + threadIdx.x; t < len; t += kBlock) win[t] = src[lo + t];
}

// Sliced blocks: one window [lo, lo + len) in LDS, entries of other columns count 0 in this
// pass; and the pass over the entries outside all windows, read from global memory.
template <typename Tx>
struct FromSlice {
    LdsPtr<Tx> w;
    int lo, len;
    __device__ __forceinline__ Tx operator()(int c) const {
        const unsigned r = (unsigned)(c - lo);
        const bool in = r < (unsigned)len;
        const Tx x = w[in ? r : 0u];
        return in ? x : Tx(0);
    }
};
template <typename Tx>
struct FromOutside {
    const Tx* __restrict__ g;
    int lo, hi;
    __device__ __forceinline__ Tx operator()(int c) const {
        Tx x = Tx(0);
        if (c < lo || c >= hi) x = g[c];
        return x;
    }
};

// Dot products of stored row [b, e) with one or two gathered vectors. Lane `lane` of a
// group of G lanes takes quads b + 4*(lane + G*t); each pass issues the loads of U quads
// before any gather so U 16-byte loads per array are in flight per lane.
// PK (narrow rows of a matrix that reads packed words): each quad's index comes from its packed
// word, or from its 16-bit offsets when the word is not packed.
template <int G, int U, bool NT, bool WIDE, int NV, bool PK, typename Tm, typename S0, typename S1, typename Acc>
__device__ __forceinline__ void group_dot(const DevCsr<Tm>& A, int64_t b, int64_t e, int base, int lane,
                                          const S0& g0, const S1& g1, Acc& s0, Acc& s1) {
    s0 = Acc(0);
    s1 = Acc(0);
    for (int64_t p = b + kVec * lane; p < e; p += (int64_t)kVec * G * U) {
        int4 c[U];
        Quad<Tm> v[U];
        uint32_t w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + (int64_t)kVec * G * u;
            if (q < e) {
                if constexpr (WIDE) c[u] = load_idx<NT>(A.col + q);
                else if constexpr (PK) w[u] = load_pack<NT>(A.qpack + (q >> 2));
                else c[u] = load_idx16<NT>(A.col16 + q, base);
                v[u] = Quad<Tm>::template load<NT>(A.val + q);
            }
        }
        if constexpr (!WIDE && PK) {
            // a packed quad costs 4 bytes of index stream instead of 8; the others (an offset of
            // 8192 or more, or a gap of 64 or more) read their 16-bit offsets as well
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = p + (int64_t)kVec * G * u;
                if (q < e) c[u] = (w[u] >> 31) ? unpack_quad(w[u], base) : load_idx16<NT>(A.col16 + q, base);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + (int64_t)kVec * G * u;
            if (q < e) {
                s0 += Acc(v[u].a[0]) * Acc(g0(c[u].x)) + Acc(v[u].a[1]) * Acc(g0(c[u].y)) +
                      Acc(v[u].a[2]) * Acc(g0(c[u].z)) + Acc(v[u].a[3]) * Acc(g0(c[u].w));
                if constexpr (NV == 2) {
                    s1 += Acc(v[u].a[0]) * Acc(g1(c[u].x)) + Acc(v[u].a[1]) * Acc(g1(c[u].y)) +
                          Acc(v[u].a[2]) * Acc(g1(c[u].z)) + Acc(v[u].a[3]) * Acc(g1(c[u].w));
                }
            }
        }
    }
}

// A fused step on a matrix that reads packed words (DevCsr::qpack): the same op, instantiated
// apart so that matrices without them keep the plain offset path.
template <typename Base>
struct Packed : Base {};
template <typename Op>
struct PackOf { static constexpr bool value = false; };
template <typename Base>
struct PackOf<Packed<Base>> { static constexpr bool value = true; };

// One round of a block: each group of G lanes takes one row of rows r0 .. r0 + kBlock / G of the
// block's slice of the row list.
// MODE 0: the gathered vector is read from global memory; 1: from the block's LDS window
// `win`, which holds every column the block uses (columns relative to d.wlo; no wide rows in
// such a block); 2: from the window for the columns it holds, global memory for the rest.
template <int G, int U, bool NT, int MODE, typename Op, typename Tx>
__device__ __forceinline__ void run_round(const DevCsr<typename Op::Tm>& A, Op& op, const BlockDesc& d,
                                          const Tx* win, int r0) {
    using Acc = typename Op::Acc;
    const int lane = threadIdx.x & (G - 1);
    const int grp = r0 + (int)(threadIdx.x / G);
    const bool active = grp < d.count;
    const RowRef rr = active ? A.rows[d.first + grp] : RowRef{0, 0, 0, 0};
    const int row = rr.row;
    if (active && lane == 0) op.pre(row);   // epilogue operands, loaded while the row streams
    Acc s0 = Acc(0), s1 = Acc(0);
    if constexpr (Op::NV > 0) {
        const int64_t b = (int64_t)kVec * rr.start4;
        const int64_t e = b + (int64_t)kVec * (rr.quads & ~kWide);
        if constexpr (MODE == 1) {
            const FromWindow<Tx> w{(LdsPtr<Tx>)win};
            group_dot<G, U, NT, false, 1, PackOf<Op>::value>(A, b, e, rr.base - d.wlo, lane, w, w, s0, s1);
        } else if constexpr (MODE == 2) {
            const FromSplit<Tx> w{(LdsPtr<Tx>)win, op.g0, d.wlo, -d.wlen};
            if (rr.quads & kWide) group_dot<G, U, NT, true, 1, false>(A, b, e, rr.base, lane, w, w, s0, s1);
            else group_dot<G, U, NT, false, 1, PackOf<Op>::value>(A, b, e, rr.base, lane, w, w, s0, s1);
        } else {
            const FromGlobal<Tx> g0{op.g0}, g1{op.g1};
            if (rr.quads & kWide) group_dot<G, U, NT, true, Op::NV, false>(A, b, e, rr.base, lane, g0, g1, s0, s1);
            else group_dot<G, U, NT, false, Op::NV, PackOf<Op>::value>(A, b, e, rr.base, lane, g0, g1, s0, s1);
        }
        s0 = group_sum<G>(s0);
        if constexpr (Op::NV == 2) s1 = group_sum<G>(s1);
    }
    if (active && lane == 0) op.epi(row, s0, s1);
}

// One block. RD (the schedule has blocks in rounds): a block of rows with 8 or more lanes each may
// hold more than kBlock / G rows (the schedule gives such blocks a full window), which every op
// takes in rounds; with the window in LDS (MODE 1) all rounds gather from the one window copy.
template <int G, int U, bool NT, int MODE, bool RD, typename Op, typename Tx>
__device__ __forceinline__ void run_bin(const DevCsr<typename Op::Tm>& A, Op& op, const BlockDesc& d,
                                        const Tx* win) {
    if constexpr (RD && G >= 8 && MODE != 2) {   // blocks in rounds have full windows, never split
        for (int r0 = 0; r0 < d.count; r0 += kBlock / G)   // uniform over the block
            run_round<G, U, NT, MODE>(A, op, d, win, r0);
    } else {
        run_round<G, U, NT, MODE>(A, op, d, win, 0);
    }
}

// Sliced block (BlockDesc.ns > 0): the block walks its windows one at a time (copy into LDS,
// every row's entries of that window, which are a contiguous range of quads since the row is
// in column order; a quad that straddles two windows is read in both passes and each entry
// counted in its own), then one pass over the quads before and after all windows with the
// entries outside them read from global memory.
template <int G, int U, bool NT, typename Op, typename Tx>
__device__ __forceinline__ void run_bin_sliced(const DevCsr<typename Op::Tm>& A, Op& op, const BlockDesc& d,
                                               Tx* win) {
    using Acc = typename Op::Acc;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const bool active = grp < d.count;
    const RowRef rr = active ? A.rows[d.first + grp] : RowRef{0, 0, 0, 0};
    const int row = rr.row;
    const bool wide = (rr.quads & kWide) != 0;
    const int quads = rr.quads & ~kWide;
    const int64_t b = (int64_t)kVec * rr.start4;
    const int32_t* cum = A.slice_cum + d.cum_first + (active ? grp : 0) * (d.ns + 1);
    if (active && lane == 0) op.pre(row);
    Acc s0 = Acc(0), part = Acc(0), unused = Acc(0);
    const int W = A.slice_w;
    for (int k = 0; k < d.ns; ++k) {
        const int lo = d.wlo + k * W;
        const int len = max(0, min(W, A.ncols - lo));
        __syncthreads();                       // the previous window is no longer read
        copy_window(win, op.g0, lo, len);
        __syncthreads();
        if (active) {
            const int qa = cum[k] >> 2, qb = min(quads, (cum[k + 1] + 3) >> 2);
            if (qb > qa) {
                const FromSlice<Tx> src{(LdsPtr<Tx>)win, lo, len};
                if (wide) group_dot<G, U, NT, true, 1, false>(A, b + kVec * qa, b + kVec * qb, rr.base, lane, src, src, part, unused);
                else group_dot<G, U, NT, false, 1, PackOf<Op>::value>(A, b + kVec * qa, b + kVec * qb, rr.base, lane, src, src, part, unused);
                s0 += part;
            }
        }
    }
    if (active) {
        const FromOutside<Tx> src{op.g0, d.wlo, d.wlo + d.ns * W};
        const int q_low = min(quads, (cum[0] + 3) >> 2), q_high = cum[d.ns] >> 2;
        if (q_low > 0) {
            if (wide) group_dot<G, U, NT, true, 1, false>(A, b, b + kVec * q_low, rr.base, lane, src, src, part, unused);
            else group_dot<G, U, NT, false, 1, PackOf<Op>::value>(A, b, b + kVec * q_low, rr.base, lane, src, src, part, unused);
            s0 += part;
        }
        if (q_high < quads) {
            const int qa = max(q_high, q_low);   // a quad below every window is not read twice
            if (wide) group_dot<G, U, NT, true, 1, false>(A, b + kVec * qa, b + kVec * quads, rr.base, lane, src, src, part, unused);
            else group_dot<G, U, NT, false, 1, PackOf<Op>::value>(A, b + kVec * qa, b + kVec * quads, rr.base, lane, src, src, part, unused);
            s0 += part;
        }
    }
    s0 = group_sum<G>(s0);
    if (active && lane == 0) op.epi(row, s0, Acc(0));
}

template <int U, bool NT, typename Op, typename Tx>
__device__ __forceinline__ void run_block_sliced(const DevCsr<typename Op::Tm>& A, Op& op, const BlockDesc& d,
                                                 Tx* win) {
    switch (d.bin) {
        case 0: run_bin_sliced<1, U, NT>(A, op, d, win); break;
        case 1: run_bin_sliced<2, U, NT>(A, op, d, win); break;
        case 2: run_bin_sliced<4, U, NT>(A, op, d, win); break;
        case 3: run_bin_sliced<8, U, NT>(A, op, d, win); break;
        case 4: run_bin_sliced<16, U, NT>(A, op, d, win); break;
        case 5: run_bin_sliced<32, U, NT>(A, op, d, win); break;
        default: run_bin_sliced<64, U, NT>(A, op, d, win); break;
    }
}

template <int U, bool NT, int MODE, bool RD, typename Op, typename Tx>
__device__ __forceinline__ void run_block(const DevCsr<typename Op::Tm>& A, Op& op, const BlockDesc& d,
                                          const Tx* win) {
    switch (d.bin) {
        case 0: run_bin<1, U, NT, MODE, RD>(A, op, d, win); break;
        case 1: run_bin<2, U, NT, MODE, RD>(A, op, d, win); break;
        case 2: run_bin<4, U, NT, MODE, RD>(A, op, d, win); break;
        case 3: run_bin<8, U, NT, MODE, RD>(A, op, d, win); break;
        case 4: run_bin<16, U, NT, MODE, RD>(A, op, d, win); break;
        case 5: run_bin<32, U, NT, MODE, RD>(A, op, d, win); break;
        default: run_bin<64, U, NT, MODE, RD>(A, op, d, win); break;
    }
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

// Ops with NQ > 0 (reductions) never skip a block: every block writes its partials. A block
// with a window (wlen > 0: every column it uses; wlen < 0: a window of -wlen columns holding
// most of them), for an op with one gathered vector and a window that fits kWinBytes, copies
// the window into LDS with coalesced loads and gathers from there: the same values in the same
// order, so the result does not depend on which path a block takes.
// SL: the schedule has sliced blocks; RD: it has blocks in rounds. Separate instantiations, so
// that schedules without them keep the register budget (and occupancy) and the code of the
// simpler paths.
template <typename Op, int U, bool NT, bool SL, bool RD>
__global__ __launch_bounds__(kBlock) void csr_kernel(DevCsr<typename Op::Tm> A, Op op_in) {
    using Tx = typename std::remove_cv<typename std::remove_pointer<decltype(op_in.g0)>::type>::type;
    const BlockDesc d = A.sched[blockIdx.x];
    Op op = op_in;
    if (!op.init(d)) return;    // uniform over the block
    bool done = false;
    if constexpr (Op::NV == 1) {
        constexpr int kWinElems = kWinBytes / (int)sizeof(Tx);
        __shared__ __align__(16) Tx win[kWinElems];
        const int len = d.wlen < 0 ? -d.wlen : d.wlen;
        bool sliced = false;
        if constexpr (SL) {
            if (d.ns > 0 && A.slice_w <= kWinElems) {
                run_block_sliced<U, NT>(A, op, d, win);
                sliced = true;
            }
        }
        if (sliced) {
            done = true;
        } else if (len > 0 && len <= kWinElems) {
            copy_window(win, op.g0, d.wlo, len);
            __syncthreads();
            if (d.wlen > 0) run_block<U, NT, 1, RD>(A, op, d, win);
            else run_block<U, NT, 2, RD>(A, op, d, win);
            done = true;
        }
    }
    if (!done) run_block<U, NT, 0, RD>(A, op, d, static_cast<const Tx*>(nullptr));
    if constexpr (Op::NQ > 0) block_reduce_store(op.q, op.partials);
}

// With start/stop events (timing runs only, never under capture) the kernel is launched through
// hipExtLaunchKernelGGL, which stamps the events at the dispatch's own start and end.
template <typename Op, int U, bool NT, bool SL, bool RD>
static void launch_csr_kernel(const DevCsr<typename Op::Tm>& A, const Op& op, hipStream_t st, hipEvent_t start,
                              hipEvent_t stop) {
    if (start) hipExtLaunchKernelGGL((csr_kernel<Op, U, NT, SL, RD>), dim3(A.nblocks), dim3(kBlock), 0, st, start, stop, 0, A, op);
    else hipLaunchKernelGGL((csr_kernel<Op, U, NT, SL, RD>), dim3(A.nblocks), dim3(kBlock), 0, st, A, op);
}

template <typename Op, int U, bool NT, bool SL>
static void launch_csr_rounds(const DevCsr<typename Op::Tm>& A, const Op& op, hipStream_t st, hipEvent_t start,
                              hipEvent_t stop) {
    if (A.has_rounds) launch_csr_kernel<Op, U, NT, SL, true>(A, op, st, start, stop);
    else launch_csr_kernel<Op, U, NT, SL, false>(A, op, st, start, stop);
}

template <typename Op, int U, bool NT>
static void launch_csr_variant(const DevCsr<typename Op::Tm>& A, const Op& op, hipStream_t st, hipEvent_t start,
                               hipEvent_t stop) {
    if constexpr (Op::NV == 1) {
        if (A.has_sliced) {
            launch_csr_rounds<Op, U, NT, true>(A, op, st, start, stop);
            return;
        }
    }
    launch_csr_rounds<Op, U, NT, false>(A, op, st, start, stop);
}

// Op::STREAM: the op is one of the iteration's fused steps, the only ones whose schedule may ask
// for non-temporal matrix loads (a cache policy; the values and their order are the same).
template <typename Op>
static void launch_csr(const DevCsr<typename Op::Tm>& A, const Op& op, hipStream_t st, hipEvent_t start = nullptr,
                       hipEvent_t stop = nullptr) {
    if (A.nblocks <= 0) return;
    if constexpr (Op::NV == 0) {   // no matrix stream: one variant per row layout (rounds or not)
        if (A.has_rounds) launch_csr_kernel<Op, 1, false, false, true>(A, op, st, start, stop);
        else launch_csr_kernel<Op, 1, false, false, false>(A, op, st, start, stop);
        return;
    }
    if constexpr (Op::STREAM && !PackOf<Op>::value) {   // the fused steps read packed words when there are
        if (A.qpack) {                                    // any (other ops read the 16-bit offsets)
            launch_csr(A, Packed<Op>{op}, st, start, stop);
            return;
        }
    }
    if (A.nontemporal && Op::STREAM) {
        switch (A.unroll) {
            case 1: launch_csr_variant<Op, 1, true>(A, op, st, start, stop); break;
            case 2: launch_csr_variant<Op, 2, true>(A, op, st, start, stop); break;
            case 8: launch_csr_variant<Op, 8, true>(A, op, st, start, stop); break;
            default: launch_csr_variant<Op, 4, true>(A, op, st, start, stop); break;
        }
    } else {
        switch (A.unroll) {
            case 1: launch_csr_variant<Op, 1, false>(A, op, st, start, stop); break;
            case 2: launch_csr_variant<Op, 2, false>(A, op, st, start, stop); break;
            case 8: launch_csr_variant<Op, 8, false>(A, op, st, start, stop); break;
            default: launch_csr_variant<Op, 4, false>(A, op, st, start, stop); break;
        }
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
    static constexpr bool STREAM = true;
    const T* g0;
    const T* g1;
    DevProb<T> p;
    DevIter<T> v;
    const Ctrl* ctrl;
    int j;
    int check;
    T sigma, a0, a1;
    T xk, x0k, ck, lk, uk;
    double sigd;
    double q[1];
    double* partials;
    __device__ __forceinline__ bool init(const BlockDesc& d) {
        const Ctrl& c = ctrl[d.lp];
        if (!c.active) return false;
        const int64_t k = c.k_base + j;
        sigd = c.sigma;
        sigma = T(c.sigma);
        a0 = T(1.0 / double(k + 2));
        a1 = T(double(k + 1) / double(k + 2));
        return true;
    }
    __device__ __forceinline__ void pre(int col) {
        xk = v.x[col];
        x0k = v.x0[col];
        ck = p.c[col];
        lk = p.l[col];
        uk = p.u[col];
    }
    __device__ __forceinline__ void epi(int col, T aty, T) {
        const T w = xk + sigma * (aty - ck);
        const T xb = clampv(w, lk, uk);
        const T xh = T(2) * xb - xk;
        v.xh[col] = xh;
        v.x[col] = a0 * x0k + a1 * xh;
        if (check) {
            if constexpr (std::is_same<T, float>::value) {
                // The check's bar point, z and step come from w formed in FP64: in FP32 the step
                // sigma (A^T y - c) is rounded against x (to 2^-24 |x|), and z = (xbar - w) / sigma
                // would carry that rounding divided by sigma, a floor on the dual residual and gap
                // that grows as sigma shrinks.
                const double wd = double(xk) + sigd * (double(aty) - double(ck));
                const double xbd = clampv(wd, double(lk), double(uk));
                v.xb[col] = T(xbd);
                v.zb[col] = T((xbd - wd) / sigd);
                v.dx[col] = T(double(xk) - xbd);
            } else {
                v.xb[col] = xb;
                v.zb[col] = (xb - w) / sigma;
                v.dx[col] = xk - xb;
            }
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
    static constexpr bool STREAM = true;
    const T* g0;
    const T* g1;
    DevProb<T> p;
    DevIter<T> v;
    const Ctrl* ctrl;
    int j;
    int check;
    T s, a0, a1;
    T yk, y0k, lok, hik;
    double sd;
    double q[1];
    double* partials;
    __device__ __forceinline__ bool init(const BlockDesc& d) {
        const Ctrl& c = ctrl[d.lp];
        if (!c.active) return false;
        const int64_t k = c.k_base + j;
        sd = c.s;
        s = T(c.s);
        a0 = T(1.0 / double(k + 2));
        a1 = T(double(k + 1) / double(k + 2));
        return true;
    }
    __device__ __forceinline__ void pre(int row) {
        yk = v.y[row];
        y0k = v.y0[row];
        lok = p.lo[row];
        hik = p.hi[row];
    }
    __device__ __forceinline__ void epi(int row, T ax, T) {
        const T vv = yk - s * ax;
        const T up = vv + s * lok;
        const T dn = vv + s * hik;
        const T yb = up > T(0) ? up : (dn < T(0) ? dn : T(0));
        const T yh = T(2) * yb - yk;
        v.y[row] = a0 * y0k + a1 * yh;
        if (check) {
            if constexpr (std::is_same<T, float>::value) {   // as in the primal step: ybar and
                const double vd = double(yk) - sd * double(ax);   // y - ybar from FP64 arithmetic
                const double upd = vd + sd * double(lok);
                const double dnd = vd + sd * double(hik);
                const double ybd = upd > 0.0 ? upd : (dnd < 0.0 ? dnd : 0.0);
                v.yb[row] = T(ybd);
                v.dy[row] = T(double(yk) - ybd);
            } else {
                v.yb[row] = yb;
                v.dy[row] = yk - yb;
            }
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
//   q6 = sum |lo_i| ybar_i+ + |hi_i| ybar_i-                  (magnitude of q3's terms)
//   q7 = sum |ybar_i|                                         (size of ybar)
//   q8 = sum dist((A d)_i, rows' recession cone)^2 with d = xbar - x = -dx (the step's primal
//        move, a candidate ray of an LP without finite optimum): (A d)_i must be 0 for two
//        finite sides, >= 0 with only lo_i finite, <= 0 with only hi_i finite
template <typename M, typename P, typename V>
struct CheckRowsOp {
    using Tm = M;
    using Acc = M;
    static constexpr int NV = 2, NQ = kRowQ;
    static constexpr bool STREAM = false;
    const V* g0;
    const V* g1;
    DevProb<P> p;
    DevIter<V> v;
    const Ctrl* ctrl;
    double beta_b;
    double q[NQ];
    double* partials;
    __device__ __forceinline__ void pre(int) {}
    __device__ __forceinline__ bool init(const BlockDesc& d) {
        beta_b = ctrl[d.lp].beta_b;
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[k] = 0.0;
        return true;
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
        if (yb > 0.0) q[6] += fabs(lo) * yb;
        else if (yb < 0.0) q[6] -= fabs(hi) * yb;
        q[7] += fabs(yb);
        const double ad = -double(adx);
        const bool fl = isfinite(lo), fh = isfinite(hi);
        const double vr = (fl && fh) ? fabs(ad) : fl ? (ad < 0.0 ? -ad : 0.0) : fh ? (ad > 0.0 ? ad : 0.0) : 0.0;
        q[8] += vr * vr;
    }
};

// Column side, over the rows of A^T with (A^T ybar)_j:
//   q0 = sum (beta_c/dc_j * (c_j - (A^T ybar)_j - zbar_j))^2   (unscaled dual residual)
//   q1 = sum c_j xbar_j                                        (scaled primal objective)
//   q2 = sum l_j zbar_j+ - u_j zbar_j-                          (scaled dual objective, columns)
//   q3 = sum dx_j^2,  q4 = sum (xbar_j - x0_j)^2,  q5 = non-finite count
// and, with dz = -(A^T ybar)_j (the column part of a primal infeasibility certificate built
// from ybar, which is sign-feasible by construction):
//   q6 = sum l_j dz_j+ - u_j dz_j- over finite bounds,  q7 = the same with |l_j|, |u_j|,
//   q8 = sum of dz_j+ with l_j = -inf and dz_j- with u_j = +inf (sign violations)
// and, with d = -dx = xbar - x (the step's primal move, a candidate ray):
//   q9 = sum c_j d_j,  q10 = sum dist(d_j, columns' recession cone)^2 (d_j must be 0 for two
//   finite bounds, >= 0 with only l_j finite, <= 0 with only u_j finite),  q11 = sum c_j^2
template <typename M, typename P, typename V>
struct CheckColsOp {
    using Tm = M;
    using Acc = M;
    static constexpr int NV = 1, NQ = kColQ;
    static constexpr bool STREAM = false;
    const V* g0;
    const V* g1;
    DevProb<P> p;
    DevIter<V> v;
    const Ctrl* ctrl;
    double beta_c;
    double q[NQ];
    double* partials;
    __device__ __forceinline__ void pre(int) {}
    __device__ __forceinline__ bool init(const BlockDesc& d) {
        beta_c = ctrl[d.lp].beta_c;
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[k] = 0.0;
        return true;
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
        const double dz = -double(aty);
        const double l = double(p.l[col]), u = double(p.u[col]);
        if (dz > 0.0) {
            if (isfinite(l)) {
                q[6] += l * dz;
                q[7] += fabs(l) * dz;
            } else {
                q[8] += dz;
            }
        } else if (dz < 0.0) {
            if (isfinite(u)) {
                q[6] += u * dz;
                q[7] -= fabs(u) * dz;
            } else {
                q[8] -= dz;
            }
        }
        const double d = -dx;
        q[9] += c * d;
        const bool fl = isfinite(l), fu = isfinite(u);
        const double vc = (fl && fu) ? fabs(d) : fl ? (d < 0.0 ? -d : 0.0) : fu ? (d > 0.0 ? d : 0.0) : 0.0;
        q[10] += vc * vc;
        q[11] += c * c;
    }
};

// ---------------------------------------------------------------- per-row bookkeeping (no product)

// restart of LP d.lp: anchor = iterate = bar point (rows: y; columns: x)
template <typename T, bool ROWS>
struct RestartOp {
    using Tm = T;
    using Acc = T;
    static constexpr int NV = 0, NQ = 0;
    static constexpr bool STREAM = false;
    const T* g0;
    const T* g1;
    DevIter<T> v;
    const Ctrl* ctrl;
    double q[1];
    double* partials;
    __device__ __forceinline__ void pre(int) {}
    __device__ __forceinline__ bool init(const BlockDesc& d) { return ctrl[d.lp].restart != 0; }
    __device__ __forceinline__ void epi(int i, T, T) {
        if constexpr (ROWS) {
            const T b = v.yb[i];
            v.y0[i] = b;
            v.y[i] = b;
        } else {
            const T a = v.xb[i];
            v.x0[i] = a;
            v.x[i] = a;
        }
    }
};

// original-space bar point: x = beta_b dc xbar, z = beta_c zbar / dc, y = beta_c dr ybar
template <typename T, bool ROWS>
struct UnscaleOp {
    using Tm = T;
    using Acc = T;
    static constexpr int NV = 0, NQ = 0;
    static constexpr bool STREAM = false;
    const T* g0;
    const T* g1;
    DevIter<T> v;
    const Ctrl* ctrl;
    const double *dr, *dc;
    double *x, *y, *z;
    double bb, bc;
    double q[1];
    double* partials;
    __device__ __forceinline__ void pre(int) {}
    __device__ __forceinline__ bool init(const BlockDesc& d) {
        bb = ctrl[d.lp].beta_b;
        bc = ctrl[d.lp].beta_c;
        return true;
    }
    __device__ __forceinline__ void epi(int i, T, T) {
        if constexpr (ROWS) {
            y[i] = bc * dr[i] * double(v.yb[i]);
        } else {
            x[i] = bb * dc[i] * double(v.xb[i]);
            z[i] = bc * double(v.zb[i]) / dc[i];
        }
    }
};

// ---------------------------------------------------------------- plain product

template <typename T>
struct SpmvOp {
    using Tm = T;
    using Acc = T;
    static constexpr int NV = 1, NQ = 0;
    static constexpr bool STREAM = false;
    const T* g0;
    const T* g1;
    T* out;
    double q[1];
    double* partials;
    __device__ __forceinline__ void pre(int) {}
    __device__ __forceinline__ bool init(const BlockDesc&) { return true; }
    __device__ __forceinline__ void epi(int row, T s, T) { out[row] = s; }
};

template <typename T>
__global__ void cast_kernel(const double* s, T* d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = T(s[i]);
}


template <typename T>
void launch_primal_step(const DevCsr<T>& At, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                        int j, bool check, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
    PrimalOp<T> op{};
    op.g0 = v.y;
    op.p = p;
    op.v = v;
    op.ctrl = ctrl;
    op.j = j;
    op.check = check ? 1 : 0;
    launch_csr(At, op, st, start, stop);
}

template <typename T>
void launch_dual_step(const DevCsr<T>& A, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                      int j, bool check, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
    DualOp<T> op{};
    op.g0 = v.xh;
    op.p = p;
    op.v = v;
    op.ctrl = ctrl;
    op.j = j;
    op.check = check ? 1 : 0;
    launch_csr(A, op, st, start, stop);
}

template <typename Tm, typename Tp, typename Tv>
void launch_check_rows(const DevCsr<Tm>& A, const DevProb<Tp>& p, const DevIter<Tv>& v, const Ctrl* ctrl,
                       double* partials, hipStream_t st) {
    CheckRowsOp<Tm, Tp, Tv> op{};
    op.g0 = v.xb;
    op.g1 = v.dx;
    op.p = p;
    op.v = v;
    op.ctrl = ctrl;
    op.partials = partials;
    launch_csr(A, op, st);
}

template <typename Tm, typename Tp, typename Tv>
void launch_check_cols(const DevCsr<Tm>& At, const DevProb<Tp>& p, const DevIter<Tv>& v, const Ctrl* ctrl,
                       double* partials, hipStream_t st) {
    CheckColsOp<Tm, Tp, Tv> op{};
    op.g0 = v.yb;
    op.p = p;
    op.v = v;
    op.ctrl = ctrl;
    op.partials = partials;
    launch_csr(At, op, st);
}

template <typename T>
void launch_restart(const DevCsr<T>& A, const DevCsr<T>& At, const DevIter<T>& v, const Ctrl* ctrl,
                    hipStream_t st) {
    RestartOp<T, true> r{};
    r.v = v;
    r.ctrl = ctrl;
    launch_csr(A, r, st);
    RestartOp<T, false> c{};
    c.v = v;
    c.ctrl = ctrl;
    launch_csr(At, c, st);
}

template <typename T>
void launch_spmv(const DevCsr<T>& A, const T* x, T* y, hipStream_t st) {
    SpmvOp<T> op{};
    op.g0 = x;
    op.out = y;
    launch_csr(A, op, st);
}

template <typename T>
void launch_unscale(const DevCsr<T>& A, const DevCsr<T>& At, const DevIter<T>& v, const double* dr,
                    const double* dc, const Ctrl* ctrl, double* x, double* y, double* z, hipStream_t st) {
    UnscaleOp<T, true> r{};
    r.v = v;
    r.ctrl = ctrl;
    r.dr = dr;
    r.dc = dc;
    r.y = y;
    launch_csr(A, r, st);
    UnscaleOp<T, false> c{};
    c.v = v;
    c.ctrl = ctrl;
    c.dr = dr;
    c.dc = dc;
    c.x = x;
    c.z = z;
    launch_csr(At, c, st);
}

template <typename T>
void launch_cast(const double* src, T* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(cast_kernel<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, src,
                       dst, n);
}

}  // namespace hpr

#endif  // HPR_CSR_H
