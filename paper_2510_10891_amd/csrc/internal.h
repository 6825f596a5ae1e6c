// Internal device data layout and kernel launchers of the gfx950 LP solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpr {

constexpr int kBlock = 256;      // threads per block: 4 wavefronts of 64 lanes
constexpr int kNumBins = 7;      // lanes per row: 1, 2, 4, 8, 16, 32, 64
constexpr int kVec = 4;          // every stored row is padded to a multiple of 4 entries
constexpr int kMaxQ = 8;         // FP64 quantities reduced by one check kernel
constexpr int kRowQ = 6;         // quantities of the row check
constexpr int kColQ = 6;         // quantities of the column check

// Rows of one matrix grouped by how many lanes work on a row. With U quads (4 entries)
// per lane and pass, bin b holds rows of at most U * 2^b quads (the last bin also takes
// every longer row, whose lanes then loop); a block of bin b covers kBlock / 2^b rows.
struct Bins {
    int32_t row_off[kNumBins];       // offset of bin b in the row list
    int32_t nrows[kNumBins];
    int32_t block_off[kNumBins + 1]; // first block of bin b; [kNumBins] = total blocks
};

// A sparse matrix on the device: CSR whose rows start at multiples of 4 entries, so a
// lane reads 4 values and 4 column indices with 16-byte loads. Padding entries carry
// value 0 and a column index the row already uses.
template <typename Tm>
struct DevCsr {
    const int64_t* start;   // [rows + 1]
    const int32_t* col;     // [padded nnz]
    const Tm* val;          // [padded nnz]
    const int32_t* rows;    // row list ordered by bin
    Bins bins;
    int32_t nrows;
    int32_t unroll;         // U: 1, 2, 4 or 8 quads per lane and pass
};

// Scalars the iteration reads on the device (written by the host between blocks).
struct Ctrl {
    double sigma;       // primal step
    double s;           // dual step 1 / (lambda sigma)
    double lambda;
    int64_t k_base;     // Halpern counter at the first iteration of the current block
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

// Launchers (kernels.hip). All run on `st`.
template <typename T>
void launch_primal_step(const DevCsr<T>& At, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                        int j, bool check, hipStream_t st);
template <typename T>
void launch_dual_step(const DevCsr<T>& A, const DevProb<T>& p, const DevIter<T>& v, const Ctrl* ctrl,
                      int j, bool check, hipStream_t st);
// Check kernels: per-block FP64 partial sums into partials [quantity][nblocks].
template <typename Tm, typename Tp, typename Tv>
void launch_check_rows(const DevCsr<Tm>& A, const DevProb<Tp>& p, const DevIter<Tv>& v, double beta_b,
                       double* partials, hipStream_t st);
template <typename Tm, typename Tp, typename Tv>
void launch_check_cols(const DevCsr<Tm>& At, const DevProb<Tp>& p, const DevIter<Tv>& v, double beta_c,
                       double* partials, hipStream_t st);
// Sums partials [nq][nblocks] in a fixed order into out[nq] (one block per quantity).
void launch_finish_sums(const double* partials, int nq, int nblocks, double* out, hipStream_t st);
// y = A x (plain product, used by the power method).
template <typename T>
void launch_spmv(const DevCsr<T>& A, const T* x, T* y, hipStream_t st);
// partials[b] = sum of v_i^2 over block b's slice (FP64); nblocks = sumsq_blocks(n).
template <typename T>
void launch_sumsq(const T* v, int64_t n, double* partials, hipStream_t st);
int sumsq_blocks(int64_t n);
template <typename T>
void launch_scale(T* v, int64_t n, double factor, hipStream_t st);
template <typename T>
void launch_start_vector(T* v, int64_t n, uint64_t seed, hipStream_t st);
// x0 = x = xb ; y0 = y = yb
template <typename T>
void launch_restart(const DevIter<T>& v, int n, int m, hipStream_t st);
// original-space point: x = beta_b dc xb, y = beta_c dr yb, z = beta_c zb / dc (FP64 out)
template <typename T>
void launch_unscale(const DevIter<T>& v, const double* dr, const double* dc, int n, int m, double beta_b,
                    double beta_c, double* x, double* y, double* z, hipStream_t st);
// FP64 -> T copy
template <typename T>
void launch_cast(const double* src, T* dst, int64_t n, hipStream_t st);

}  // namespace hpr
