// Internal device data layout and kernel launchers of the gfx950 LP solver.
//
// One engine serves a single LP and a batch alike: the LPs of a batch are pooled into one
// block-diagonal problem (rows and columns of LP l occupy contiguous ranges), each kernel
// launch covers every LP, and per-LP scalars live in device arrays indexed by the LP id
// that each thread block carries in its descriptor.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpr {

constexpr int kBlock = 256;      // threads per block: 4 wavefronts of 64 lanes
constexpr int kNumBins = 7;      // lanes per row: 1, 2, 4, 8, 16, 32, 64
constexpr int kVec = 4;          // every stored row is padded to a multiple of 4 entries
constexpr int kRowQ = 9;         // FP64 quantities of the row check
constexpr int kColQ = 12;        // FP64 quantities of the column check
constexpr int kColOff = 9;       // per-LP sums: [0, kRowQ) rows, [kColOff, kColOff + kColQ) columns
constexpr int kSumStride = 24;
constexpr double kInfeasTol = 1e-6;   // relative margin of the infeasibility certificates
constexpr double kRayTol32 = 1e-3;    // ... of the dual infeasibility test with FP32 storage
constexpr int kChunk = 8192;     // entries per block of the segmented vector kernels
constexpr int kMaxBatch = 1024;  // LPs per engine (one control thread each)

// One thread block of a matrix product: rows list[first .. first + count) of bin `bin`
// (2^bin lanes per row), all belonging to LP `lp`; count is at most kBlock / 2^bin rows, or up to
// kMaxRounds times that for a block with a full window and bin >= 3 (its rows taken in rounds).
// LDS windows of the gathered vector (products with one gathered vector):
//   wlen > 0: "full", every column the block's rows use lies in [wlo, wlo + wlen);
//   wlen < 0: "split", the window [wlo, wlo - wlen) holds most of them, the rest are read from
//             global memory;
//   ns > 0:   "sliced", the block walks ns consecutive windows of slice_w columns from wlo, one
//             at a time in LDS; row r of the block has its entries below the k-th window's first
//             column counted in slice_cum[cum_first + r * (ns + 1) + k] (k = 0 .. ns; the rows'
//             entries are in column order), entries outside all windows are read from global
//             memory.
struct BlockDesc {
    int32_t bin;
    int32_t lp;
    int32_t first;
    int32_t count;
    int32_t wlo;
    int32_t wlen;
    int32_t ns;
    int32_t cum_first;
};
constexpr int kMaxSlices = 8;       // windows per sliced block
constexpr int kMaxRounds = 4;       // rounds of rows per block with a full window
constexpr int kWinBytes = 16384;   // LDS per block for a staged window
constexpr int kXcds = 8;           // accelerator complex dies of the MI355X, each with its own L2

// One entry of a schedule's row list, fetched by one 16-byte load: the row, its number of
// quads (4 stored entries; the top bit marks a "wide" row), the smallest column of the row
// and the position of its first entry divided by 4.
struct RowRef {
    int32_t row;
    int32_t quads;      // bit 31: wide row (column span >= 65536, read from the 32-bit indices)
    int32_t base;       // smallest column of the row
    int32_t start4;     // first stored entry / 4
};
constexpr int32_t kWide = int32_t(0x80000000u);

// A sparse matrix on the device: CSR whose rows start at multiples of 4 entries. Padding
// entries carry value 0 and a column index the row already uses. Column indices are global
// (pooled). A row whose columns span less than 65536 is read through 16-bit offsets from its
// smallest column (a quad = 16 bytes of FP32 values + 8 bytes of offsets); wider rows through
// the 32-bit indices.
template <typename Tm>
struct DevCsr {
    const int32_t* col;        // [padded nnz] 32-bit column indices
    const uint16_t* col16;     // [padded nnz] column - row base (narrow rows)
    const uint32_t* qpack;     // [padded nnz / 4] per quad of a narrow row: bit 31 set = packed
                               // (bits 0-12 first offset, 13-18 / 19-24 / 25-30 the gaps to the
                               // second, third and fourth entry); clear = read col16. Null: the
                               // matrix reads col16 only (too few quads pack)
    const Tm* val;             // [padded nnz]
    const RowRef* rows;        // row list in schedule order
    const BlockDesc* sched;    // [nblocks]
    const int32_t* slice_cum;  // per sliced block and row: entries below each window (BlockDesc)
    int32_t slice_w;           // columns per window of a sliced block
    int32_t ncols;             // length of the gathered vector
    int32_t has_sliced;        // 1: some block of the schedule is sliced
    int32_t has_rounds;        // 1: some block of the schedule takes its rows in rounds
    int32_t nblocks;
    int32_t unroll;            // U: 1, 2, 4 or 8 quads per lane and pass
    int32_t nontemporal;       // 1: stream the matrix with non-temporal loads
};

// Per-LP scalars read by the iteration kernels.
struct Ctrl {
    double sigma;       // primal step
    double s;           // dual step 1 / (lambda sigma)
    double lambda;
    double beta_b, beta_c;
    int64_t k_base;     // Halpern counter at the first iteration of the current block
    int32_t active;     // 0: finished, the LP's blocks return at once
    int32_t restart;    // 1: copy the bar point into anchor and iterate (set at a check)
};

// Per-LP control state of the check logic (device-resident, read back at the end).
struct LpState {
    double r0, r_prev;           // merit at the last restart and at the previous check
    double norm_b, norm_c, obj_offset;
    double rel_p, rel_d, rel_gap, rel_kkt, pobj, dobj, merit;
    double p32[6];               // FP32-storage check values kept while FP64 confirms them
    double mark_kkt;             // FP32 storage: rel_kkt at the last halving of the best one
    int64_t mark_it;             // and the iteration count there
    int64_t it, k, restarts;
    int32_t term;                // 0 running, else HPR_SOLVED ...
    int32_t candidate;           // FP32 check passed, awaiting FP64 confirmation
    int32_t warm;                // the solve started from the caller's point (sigma weight)
};

// Problem vectors of the scaled LP (type Tp) and the diagonal scaling (FP64).
template <typename Tp>
struct DevProb {
    const Tp *c, *l, *u;         // [n] scaled cost and column bounds
    const Tp *lo, *hi;           // [m] scaled row bounds
    const double *dr, *dc;       // [m], [n]
};

// Iterates in the scaled space (type Tv).
template <typename Tv>
struct DevIter {
    Tv *x, *x0, *xh, *xb, *zb, *dx;   // [n] iterate, anchor, reflection, bar point, zbar, x - xbar
    Tv *y, *y0, *yb, *dy;             // [m] iterate, anchor, bar point, y - ybar
};

// Launchers (kernels.hip). All run on `st` and may be captured into a graph; the fused steps
// take optional start/stop events stamped at the kernel's own start and end (timing runs only,
// not under capture).
template <typename T>
void launch_primal_step(const DevCsr<T>& At, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                        int j, bool check, hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
template <typename T>
void launch_dual_step(const DevCsr<T>& A, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                      int j, bool check, hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Check kernels: per-block FP64 partial sums into partials [quantity][nblocks].
template <typename Tm, typename Tp, typename Tv>
void launch_check_rows(const DevCsr<Tm>& A, const DevProb<Tp>& p, const DevIter<Tv>& v, const Ctrl* ctrl,
                       double* partials, hipStream_t st);
template <typename Tm, typename Tp, typename Tv>
void launch_check_cols(const DevCsr<Tm>& At, const DevProb<Tp>& p, const DevIter<Tv>& v, const Ctrl* ctrl,
                       double* partials, hipStream_t st);
// out[l * kSumStride + off + q] = sum of partials[q][seg[l] .. seg[l+1]) in a fixed order.
void launch_finish_sums(const double* partials, int nq, int nblocks, const int32_t* seg, int nlp,
                        double* out, int off, hipStream_t st);
// Copies the bar point into anchor and iterate for the LPs whose Ctrl::restart is set.
template <typename T>
void launch_restart(const DevCsr<T>& A, const DevCsr<T>& At, const DevIter<T>& v, const Ctrl* ctrl,
                    hipStream_t st);
// The per-LP decisions of a check (one thread per LP); phase 1 after the storage-precision
// check, phase 2 after an FP64 confirmation of candidates, phase 3 stores FP64 values
// for reporting, phase 4 ends every running LP at the time limit.
struct ControlArgs {
    Ctrl* ctrl;
    LpState* st;
    const double* sums;      // storage-precision check sums [nlp][kSumStride]
    const double* sums64;    // FP64 check sums (phases 2, 3)
    int32_t* stat;           // [0] running LPs, [1] candidates
    int nlp;
    int nb;                  // iterations in the block just run (phase 1)
    int fp32;
    int phase;
    int64_t max_iter;
    double tol;
    int restart_rule;
    int sigma_update;
    double sigma_smoothing;       // weight of sigma* in the log-space update (cold start)
    double sigma_smoothing_warm;  // the same from the caller's start point
    int64_t stall_iters;          // FP32 storage: minimum iterations of the stall test (0: off)
};
void launch_control(const ControlArgs& a, hipStream_t st);
// y = A x (plain product, used by the power method).
template <typename T>
void launch_spmv(const DevCsr<T>& A, const T* x, T* y, hipStream_t st);
// Segmented vector kernels over pooled ranges seg[0..nlp] (entries of LP l in [seg[l], seg[l+1])):
// partials[l * max_chunks + c] = sum of squares of chunk c of LP l; start vector from SplitMix64
// with LP-local indices; scale by factor[l].
void launch_seg_sumsq(const double* v, const int64_t* seg, int nlp, int max_chunks, double* partials,
                      hipStream_t st);
void launch_seg_start_vector(double* v, const int64_t* seg, int nlp, int max_chunks, uint64_t seed,
                             hipStream_t st);
void launch_seg_scale(double* v, const int64_t* seg, int nlp, int max_chunks, const double* factor,
                      hipStream_t st);
// hist[l] = sqrt(sums[l * kSumStride]), fac[l] = 1 / hist[l] (1 when it is 0), for l < nlp
void launch_power_norms(const double* sums, int nlp, double* hist, double* fac, hipStream_t st);
// original-space point: x = beta_b dc xb, y = beta_c dr yb, z = beta_c zb / dc (FP64 out)
template <typename T>
void launch_unscale(const DevCsr<T>& A, const DevCsr<T>& At, const DevIter<T>& v, const double* dr,
                    const double* dc, const Ctrl* ctrl, double* x, double* y, double* z, hipStream_t st);
// Round and the Fixing-Strategy of Algorithm 1 for G units and T hours (one thread per unit):
// cols, fixval, rounded [G][T][3] (col < 0: value fixval), fixed [G][T].
void launch_fix_strategy(const double* x, const int32_t* cols, const double* fixval, int G, int T, double tau,
                         int8_t* fixed, int8_t* rounded, hipStream_t st);
// ---- device setup of one LP (setup.hip)

// A device buffer that grows on demand and frees itself; release() hands the memory over.
struct DevScratch {
    void* p = nullptr;
    size_t cap = 0;
    DevScratch() = default;
    DevScratch(const DevScratch&) = delete;
    DevScratch& operator=(const DevScratch&) = delete;
    ~DevScratch();
    hipError_t reserve(size_t bytes);
    void* release() {
        void* q = p;
        p = nullptr;
        cap = 0;
        return q;
    }
};

// One padded layout built on the device: row starts [rows + 1], 32-bit columns, 16-bit offsets,
// FP64 (and FP32) values [padded], per row the smallest and largest column and the wide flag,
// and the runs of equal column / tile (tptr [rows + 1], tid, tcnt [nruns]).
struct DevLayout {
    DevScratch start, col, col16, val64, val32, base, top, wide, tptr, tid, tcnt;
    int64_t padded = 0, nruns = 0;
};

struct DevSetupIn {
    const int64_t* rp;       // caller's CSR on the device (rows in column order)
    const int32_t* ci;
    const double* v;
    int32_t m, n;
    int64_t nnz;
    double* dr;              // [m], [n] device: diagonal scaling
    double* dc;
    double* dr_host;         // [m], [n] host: the same factors (formed here)
    double* dc_host;
    int32_t ruiz_iters;      // Ruiz passes (0: none)
    int32_t pc;              // Pock-Chambolle pass
    int32_t fp32;            // also write FP32 values
    int32_t tile;            // columns per tile of the window choice
};

struct DevSetupOut {
    DevLayout a, at;
    DevScratch row_of, idx, perm, keys, tptr, f, lens;   // work buffers
};

// Scaling factors and both padded layouts of one LP on `st` (returns the first HIP error).
hipError_t device_setup(const DevSetupIn& in, DevSetupOut& out, hipStream_t st);

// FP64 -> T copy
template <typename T>
void launch_cast(const double* src, T* dst, int64_t n, hipStream_t st);

// qpack of a layout (DevCsr::qpack) from its 16-bit offsets, row starts and wide-row flags;
// count[0] and count[1] (device, zeroed by the caller) receive the narrow and packed quads.
void launch_pack_quads(const uint16_t* col16, const int64_t* start, const uint8_t* wide, int32_t rows,
                       int64_t nquads, uint32_t* qpack, unsigned long long* count, hipStream_t st);

}  // namespace hpr
