// Host runtime of the gfx950 LP solver: the C interface declared in hprlp.h.
//
// An Engine holds one LP or a batch pooled into one block-diagonal problem. Creation
// validates each LP, scales it (Section III-A: optional Ruiz passes, Pock-Chambolle with
// alpha = 1, bound/cost normalisation), builds the padded CSR layouts of A~ and A~^T and
// their block schedules (lane-group bins, LDS windows of the gathered vectors, XCD dealing;
// host work on several threads), tunes the schedule by timing, and estimates every LP's
// lambda = lambda_max(A~A~^T) with the power method on the device. A solve runs blocks of
// iterations of eq.(hpr); the last iteration of a block writes the bar point, two check
// kernels reduce the KKT residuals (Theorem 1's residual map, normalised) and the merit in
// FP64, and a control kernel takes every LP's decisions (termination, restart, sigma) on
// the device. Blocks are replayed as captured HIP graphs; the host polls once per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include <sys/mman.h>

#include "../../include/hprlp.h"
#include "internal.h"

using namespace hpr;

// ---------------------------------------------------------------- errors

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct HipError {
    int code;
};

#define HIP_OK(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            fail(e_ == hipErrorOutOfMemory ? HPR_ERR_NOMEM : HPR_ERR_HIP, "%s failed: %s", #expr, \
                 hipGetErrorString(e_));                                                         \
            throw HipError{e_ == hipErrorOutOfMemory ? HPR_ERR_NOMEM : HPR_ERR_HIP};              \
        }                                                                                        \
    } while (0)

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- device buffers

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 16;
        HIP_OK(hipMalloc(&p, b));
        bytes = b;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

static void sync_stream(hipStream_t st) { HIP_OK(hipStreamSynchronize(st)); }

// Allocator whose resize leaves new elements uninitialised: the large host layouts are written
// in full by several threads, so zero-filling them first on one thread would only cost time.
// Blocks of 2 MiB and more are 2 MiB-aligned and marked for transparent huge pages, so their
// first touch costs one page fault per 2 MiB instead of one per 4 KiB.
template <typename T>
struct NoInit : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInit<U>;
    };
    NoInit() = default;
    template <typename U>
    NoInit(const NoInit<U>&) noexcept {}
    T* allocate(size_t count) {
        const size_t bytes = count * sizeof(T);
        constexpr size_t kHuge = size_t(2) << 20;
        if (bytes < kHuge) return std::allocator<T>::allocate(count);
        void* p = std::aligned_alloc(kHuge, (bytes + kHuge - 1) / kHuge * kHuge);
        if (!p) throw std::bad_alloc();
        (void)madvise(p, bytes, MADV_HUGEPAGE);
        return static_cast<T*>(p);
    }
    void deallocate(T* p, size_t count) {
        if (count * sizeof(T) < (size_t(2) << 20)) std::allocator<T>::deallocate(p, count);
        else std::free(p);
    }
    template <typename U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <typename U, typename... A>
    void construct(U* p, A&&... a) {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <typename T>
using HostVec = std::vector<T, NoInit<T>>;

template <typename T, typename Al>
static void upload(DBuf& d, const std::vector<T, Al>& h, hipStream_t st) {
    d.alloc(h.size() * sizeof(T));
    if (!h.empty()) HIP_OK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// ---------------------------------------------------------------- host-side layouts

// Padded layout of one matrix (structure on the host, ready for upload).
struct Layout {
    HostVec<int64_t> start;
    HostVec<int32_t> col;
    HostVec<double> val;
};

// 16-bit offsets of every entry from its row's smallest column (rows spanning 65536 columns
// or more are "wide": their offsets are 0 and unused, the 32-bit indices are read instead);
// base / top = smallest / largest column of each row. Rows in ranges on several threads.
static void short_indices(const Layout& L, HostVec<uint16_t>& col16, std::vector<int32_t>& base,
                          std::vector<int32_t>& top, std::vector<uint8_t>& wide, int threads);

// ---------------------------------------------------------------- validation
// ---------------------------------------------------------------- validation

static int validate(const hpr_lp* lp, bool* sorted_rows = nullptr) {
    if (!lp) return fail(HPR_ERR_INVALID, "lp is NULL");
    if (lp->n < 1) return fail(HPR_ERR_INVALID, "n must be >= 1 (got %d)", lp->n);
    if (lp->m < 0 || lp->nnz < 0) return fail(HPR_ERR_INVALID, "negative m or nnz");
    if (!lp->col_lo || !lp->col_hi || !lp->c) return fail(HPR_ERR_INVALID, "col_lo, col_hi and c are required");
    if (lp->m > 0 && (!lp->row_ptr || !lp->row_lo || !lp->row_hi))
        return fail(HPR_ERR_INVALID, "row_ptr, row_lo and row_hi are required when m > 0");
    if (lp->m == 0 && lp->nnz != 0) return fail(HPR_ERR_INVALID, "nnz must be 0 when m = 0");
    if (lp->nnz > 0 && (!lp->col_idx || !lp->val)) return fail(HPR_ERR_INVALID, "col_idx and val are required");
    if (!std::isfinite(lp->obj_offset)) return fail(HPR_ERR_INVALID, "obj_offset is not finite");
    if (lp->m > 0) {
        if (lp->row_ptr[0] != 0 || lp->row_ptr[lp->m] != lp->nnz)
            return fail(HPR_ERR_INVALID, "row_ptr must start at 0 and end at nnz");
        for (int32_t i = 0; i < lp->m; ++i)
            if (lp->row_ptr[i + 1] < lp->row_ptr[i]) return fail(HPR_ERR_INVALID, "row_ptr decreases at row %d", i);
    }
    std::vector<int32_t> mark((size_t)lp->n, -1);
    bool sorted = true;
    for (int32_t i = 0; i < lp->m; ++i)
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
            const int32_t j = lp->col_idx[k];
            if (j < 0 || j >= lp->n) return fail(HPR_ERR_INVALID, "column index %d out of range in row %d", j, i);
            if (mark[j] == i) return fail(HPR_ERR_INVALID, "column %d repeated in row %d", j, i);
            mark[j] = i;
            if (!std::isfinite(lp->val[k])) return fail(HPR_ERR_INVALID, "non-finite value in row %d", i);
            if (k > lp->row_ptr[i] && lp->col_idx[k - 1] > j) sorted = false;
        }
    if (sorted_rows) *sorted_rows = sorted;
    auto bad_pair = [](double lo, double hi) {
        return std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY;
    };
    for (int32_t i = 0; i < lp->m; ++i)
        if (bad_pair(lp->row_lo[i], lp->row_hi[i])) return fail(HPR_ERR_INVALID, "bad row bounds at row %d", i);
    for (int32_t j = 0; j < lp->n; ++j) {
        if (bad_pair(lp->col_lo[j], lp->col_hi[j])) return fail(HPR_ERR_INVALID, "bad column bounds at %d", j);
        if (!std::isfinite(lp->c[j])) return fail(HPR_ERR_INVALID, "non-finite cost at %d", j);
    }
    return HPR_OK;
}

static int validate_opts(const hpr_opts* o) {
    if (!o) return fail(HPR_ERR_INVALID, "opts is NULL");
    if (o->max_iter < 1) return fail(HPR_ERR_INVALID, "max_iter must be >= 1");
    if (o->check_every < 1) return fail(HPR_ERR_INVALID, "check_every must be >= 1");
    if (!(o->sigma0 > 0) || !std::isfinite(o->sigma0)) return fail(HPR_ERR_INVALID, "sigma0 must be > 0");
    if (!(o->tol >= 0)) return fail(HPR_ERR_INVALID, "tol must be >= 0");
    if (o->precision != HPR_FP64 && o->precision != HPR_FP32) return fail(HPR_ERR_INVALID, "unknown precision");
    if (o->power_max_iter < 1) return fail(HPR_ERR_INVALID, "power_max_iter must be >= 1");
    if (std::isnan(o->lambda)) return fail(HPR_ERR_INVALID, "lambda is NaN");
    if ((o->scaling & HPR_SCALE_RUIZ) && o->ruiz_iters < 0) return fail(HPR_ERR_INVALID, "ruiz_iters < 0");
    if (!(o->warm_fallback_ratio > 0)) return fail(HPR_ERR_INVALID, "warm_fallback_ratio must be > 0");
    if (o->warm_fallback < 0 || o->warm_fallback > 2) return fail(HPR_ERR_INVALID, "warm_fallback must be 0, 1 or 2");
    if (!(o->sigma_smoothing > 0 && o->sigma_smoothing <= 1) ||
        !(o->sigma_smoothing_warm > 0 && o->sigma_smoothing_warm <= 1))
        return fail(HPR_ERR_INVALID, "sigma_smoothing and sigma_smoothing_warm must be in (0, 1]");
    if (o->unroll != 0 && o->unroll != 1 && o->unroll != 2 && o->unroll != 4 && o->unroll != 8)
        return fail(HPR_ERR_INVALID, "unroll must be 0, 1, 2, 4 or 8");
    if (o->lds_windows < -1 || o->lds_windows > 7)
        return fail(HPR_ERR_INVALID, "lds_windows must be in [-1, 7]");
    if (o->stall_iters < 0) return fail(HPR_ERR_INVALID, "stall_iters must be >= 0");
    return HPR_OK;
}

static double finite_side(double lo, double hi) {
    const bool fl = std::isfinite(lo), fh = std::isfinite(hi);
    if (fl && fh) return std::fabs(lo) > std::fabs(hi) ? lo : hi;
    if (fl) return lo;
    if (fh) return hi;
    return 0.0;
}

// ---------------------------------------------------------------- per-LP host data and scaling

struct LpHost {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    int64_t row_off = 0, col_off = 0;            // position in the pooled numbering
    double beta_b = 1, beta_c = 1, lambda = 1, norm_b = 0, norm_c = 0, obj_offset = 0;
    std::vector<double> dr, dc;                 // diagonal scaling
    std::vector<double> lo_s, hi_s, l_s, u_s, c_s;   // scaled rows, bounds and cost
    std::vector<double> x_start, y_start;       // start point in the original space (empty = zero)
};

// Runs f(0) .. f(n - 1) on up to `threads` threads; the first exception is rethrown here.
template <typename F>
static void parallel_for(int n, int threads, F f) {
    if (n <= 0) return;
    threads = std::max(1, std::min(threads, n));
    if (threads == 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::exception_ptr> errs((size_t)threads);
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            try {
                for (int i = next++; i < n; i = next++) f(i);
            } catch (...) {
                errs[t] = std::current_exception();
            }
        });
    for (std::thread& th : pool) th.join();
    for (std::exception_ptr& e : errs)
        if (e) std::rethrow_exception(e);
}

static int host_threads() {
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, hw ? hw : 1u));
}

static void short_indices(const Layout& L, HostVec<uint16_t>& col16, std::vector<int32_t>& base,
                          std::vector<int32_t>& top, std::vector<uint8_t>& wide, int threads) {
    const int64_t R = (int64_t)L.start.size() - 1;
    col16.resize(L.col.size());
    base.assign(R, 0);
    top.assign(R, 0);
    wide.assign(R, 0);
    constexpr int kChunks = 64;
    parallel_for(kChunks, threads, [&](int p) {
        for (int64_t i = R * p / kChunks; i < R * (p + 1) / kChunks; ++i) {
            const int64_t b = L.start[i], e = L.start[i + 1];
            if (b == e) continue;
            int32_t lo = L.col[b], hi = L.col[b];
            for (int64_t k = b; k < e; ++k) {
                lo = std::min(lo, L.col[k]);
                hi = std::max(hi, L.col[k]);
            }
            base[i] = lo;
            top[i] = hi;
            const bool w = (int64_t)hi - lo >= 65536;
            wide[i] = w ? 1 : 0;
            for (int64_t k = b; k < e; ++k) col16[k] = w ? (uint16_t)0 : (uint16_t)(L.col[k] - lo);
        }
    });
}

// The host preparation walks the caller's CSR in kParts row ranges of about equal entry
// counts (a fixed partition, so sums combine in the same order whatever the thread count).
constexpr int kParts = 16;

static std::vector<int32_t> row_parts(const hpr_lp* lp) {
    std::vector<int32_t> cut(kParts + 1, lp->m);
    cut[0] = 0;
    const int64_t nnz = lp->m > 0 ? lp->row_ptr[lp->m] : 0;
    int32_t i = 0;
    for (int p = 1; p < kParts; ++p) {
        const int64_t goal = nnz * p / kParts;
        while (i < lp->m && lp->row_ptr[i] < goal) ++i;
        cut[p] = std::max(cut[p - 1], i);
    }
    return cut;
}

// The entries of A in column order: for column j, positions tptr[j] .. tptr[j+1] of trow (the
// entry's row) and tent (its position in the caller's arrays), rows increasing within a column
// (a stable counting sort, partition by partition).
struct ColOrder {
    std::vector<int64_t> tptr;
    HostVec<int32_t> trow;
    HostVec<int64_t> tent;
};

static void column_order(const hpr_lp* lp, const std::vector<int32_t>& cut, int threads, ColOrder& co) {
    const int32_t m = lp->m, n = lp->n;
    const int64_t* rp = lp->row_ptr;
    std::vector<std::vector<int64_t>> cnt(kParts);
    parallel_for(kParts, threads, [&](int p) {
        cnt[p].assign((size_t)n, 0);
        for (int64_t k = (m ? rp[cut[p]] : 0); k < (m ? rp[cut[p + 1]] : 0); ++k) cnt[p][lp->col_idx[k]]++;
    });
    co.tptr.assign((size_t)n + 1, 0);
    int64_t off = 0;
    for (int32_t j = 0; j < n; ++j) {
        co.tptr[j] = off;
        for (int p = 0; p < kParts; ++p) {
            const int64_t c = cnt[p][j];
            cnt[p][j] = off;            // first slot of partition p in column j
            off += c;
        }
    }
    co.tptr[n] = off;
    co.trow.resize(off);
    co.tent.resize(off);
    parallel_for(kParts, threads, [&](int p) {
        std::vector<int64_t>& slot = cnt[p];
        for (int32_t i = cut[p]; i < cut[p + 1]; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int64_t q = slot[lp->col_idx[k]]++;
                co.trow[q] = i;
                co.tent[q] = k;
            }
    });
}

// Section III-A: optional Ruiz passes (rows/columns divided by the square root of their
// largest magnitude), then Pock-Chambolle with alpha = 1 (divided by the square root of the
// absolute row/column sums; empty ones keep 1). A pass reduces every row over its entries in
// the caller's order and every column over its entries in row order, both from the factors
// at the pass's start, with the terms |a_ij dr_i dc_j| formed as (a dr) dc: the device setup
// does the same, so both give the same factors bit for bit.
static void scale_factors(const hpr_lp* lp, const hpr_opts& o, LpHost& h, const ColOrder& co, int threads) {
    const int32_t m = lp->m, n = lp->n;
    h.dr.assign((size_t)m, 1.0);
    h.dc.assign((size_t)n, 1.0);
    std::vector<double> drn((size_t)m);
    const int64_t* rp = lp->row_ptr;
    constexpr int kChunks = 64;
    auto pass = [&](bool sum) {
        parallel_for(kChunks, threads, [&](int p) {
            for (int64_t i = (int64_t)m * p / kChunks; i < (int64_t)m * (p + 1) / kChunks; ++i) {
                double r = 0.0;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                    const double a = std::fabs(lp->val[k] * h.dr[i] * h.dc[lp->col_idx[k]]);
                    r = sum ? r + a : std::max(r, a);
                }
                drn[i] = h.dr[i] * (r > 0 ? 1.0 / std::sqrt(r) : 1.0);
            }
        });
        parallel_for(kChunks, threads, [&](int p) {
            for (int64_t j = (int64_t)n * p / kChunks; j < (int64_t)n * (p + 1) / kChunks; ++j) {
                double c = 0.0;
                for (int64_t q = co.tptr[j]; q < co.tptr[j + 1]; ++q) {
                    const double a = std::fabs(lp->val[co.tent[q]] * h.dr[co.trow[q]] * h.dc[j]);
                    c = sum ? c + a : std::max(c, a);
                }
                h.dc[j] *= c > 0 ? 1.0 / std::sqrt(c) : 1.0;
            }
        });
        h.dr.swap(drn);
    };
    if (o.scaling & HPR_SCALE_RUIZ)
        for (int32_t it = 0; it < o.ruiz_iters; ++it) pass(false);
    if (o.scaling & HPR_SCALE_PC) pass(true);
}

// From the diagonal scaling: the scaled bounds and cost, then division of the bounds by
// beta_b = 1 + ||b~|| (b~ the finite sides of the scaled rows) and of the cost by
// beta_c = 1 + ||c~||, and the norms of the original rhs and cost.
static void scale_vectors(const hpr_lp* lp, const hpr_opts& o, LpHost& h) {
    const int32_t m = lp->m, n = lp->n;
    h.lo_s.resize(m);
    h.hi_s.resize(m);
    for (int32_t i = 0; i < m; ++i) {
        h.lo_s[i] = lp->row_lo[i] * h.dr[i];
        h.hi_s[i] = lp->row_hi[i] * h.dr[i];
    }
    h.l_s.resize(n);
    h.u_s.resize(n);
    h.c_s.resize(n);
    for (int32_t j = 0; j < n; ++j) {
        h.l_s[j] = lp->col_lo[j] / h.dc[j];
        h.u_s[j] = lp->col_hi[j] / h.dc[j];
        h.c_s[j] = lp->c[j] * h.dc[j];
    }
    h.beta_b = h.beta_c = 1.0;
    if (o.scaling & HPR_SCALE_BC) {
        double b2 = 0.0, c2 = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            const double b = finite_side(h.lo_s[i], h.hi_s[i]);
            b2 += b * b;
        }
        for (int32_t j = 0; j < n; ++j) c2 += h.c_s[j] * h.c_s[j];
        h.beta_b = 1.0 + std::sqrt(b2);
        h.beta_c = 1.0 + std::sqrt(c2);
        for (int32_t i = 0; i < m; ++i) {
            h.lo_s[i] /= h.beta_b;
            h.hi_s[i] /= h.beta_b;
        }
        for (int32_t j = 0; j < n; ++j) {
            h.l_s[j] /= h.beta_b;
            h.u_s[j] /= h.beta_b;
            h.c_s[j] /= h.beta_c;
        }
    }
    double b2 = 0.0, c2 = 0.0;   // norms of the original rhs and cost (relative residuals)
    for (int32_t i = 0; i < m; ++i) {
        const double b = finite_side(lp->row_lo[i], lp->row_hi[i]);
        b2 += b * b;
    }
    for (int32_t j = 0; j < n; ++j) c2 += lp->c[j] * lp->c[j];
    h.norm_b = std::sqrt(b2);
    h.norm_c = std::sqrt(c2);
    h.obj_offset = lp->obj_offset;
}

// Padded layouts of A~ = Dr A Dc (rows of the caller's CSR, each put in column order) and of
// A~^T (rows = columns of A, from the column order), written straight from the caller's arrays:
// every row's storage is padded to a multiple of 4 entries with value 0 at the row's largest
// column; entries a_ij dr_i dc_j.
static void make_layouts(const hpr_lp* lp, const LpHost& h, const ColOrder& co, const std::vector<int32_t>& cut,
                         int threads, Layout& la, Layout& lt) {
    const int32_t m = lp->m, n = lp->n;
    const int64_t* rp = lp->row_ptr;
    auto pad = [](int64_t len) { return (len + kVec - 1) / kVec * kVec; };
    la.start.resize((size_t)m + 1);
    int64_t off = 0;
    for (int32_t i = 0; i < m; ++i) {
        la.start[i] = off;
        off += pad(rp[i + 1] - rp[i]);
    }
    la.start[m] = off;
    la.col.resize(off);
    la.val.resize(off);
    parallel_for(kParts, threads, [&](int p) {
        std::vector<std::pair<int32_t, double>> tmp;
        for (int32_t i = cut[p]; i < cut[p + 1]; ++i) {
            const int64_t b = rp[i], e = rp[i + 1];
            const double di = h.dr[i];
            int64_t d = la.start[i];
            bool sorted = true;
            for (int64_t k = b + 1; k < e; ++k) sorted = sorted && lp->col_idx[k - 1] < lp->col_idx[k];
            if (sorted) {
                for (int64_t k = b; k < e; ++k, ++d) {
                    const int32_t j = lp->col_idx[k];
                    la.col[d] = j;
                    la.val[d] = lp->val[k] * di * h.dc[j];
                }
            } else {   // entries in column order (the sliced windows rely on it)
                tmp.clear();
                for (int64_t k = b; k < e; ++k) tmp.emplace_back(lp->col_idx[k], lp->val[k]);
                std::sort(tmp.begin(), tmp.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
                for (const auto& t : tmp) {
                    la.col[d] = t.first;
                    la.val[d] = t.second * di * h.dc[t.first];
                    ++d;
                }
            }
            for (; d < la.start[i + 1]; ++d) {   // padding: value 0 at the row's largest column
                la.col[d] = la.col[d - 1];
                la.val[d] = 0.0;
            }
        }
    });
    lt.start.resize((size_t)n + 1);
    int64_t toff = 0;
    for (int32_t j = 0; j < n; ++j) {
        lt.start[j] = toff;
        toff += pad(co.tptr[j + 1] - co.tptr[j]);
    }
    lt.start[n] = toff;
    lt.col.resize(toff);
    lt.val.resize(toff);
    constexpr int kChunks = 64;
    parallel_for(kChunks, threads, [&](int p) {
        for (int64_t j = (int64_t)n * p / kChunks; j < (int64_t)n * (p + 1) / kChunks; ++j) {
            int64_t d = lt.start[j];
            for (int64_t q = co.tptr[j]; q < co.tptr[j + 1]; ++q, ++d) {
                const int32_t i = co.trow[q];
                lt.col[d] = i;
                lt.val[d] = lp->val[co.tent[q]] * h.dr[i] * h.dc[j];
            }
            for (; d < lt.start[j + 1]; ++d) {
                lt.col[d] = lt.col[d - 1];
                lt.val[d] = 0.0;
            }
        }
    });
}

// ---------------------------------------------------------------- pooled matrices and schedules

// The work list of one pooled matrix for U quads per lane and pass: per LP, per bin (bin b:
// rows of at most U * 2^b quads, 2^b lanes each; the last bin takes longer rows too), the
// rows in index order cut into blocks of kBlock / 2^b rows. seg[l] = first block of LP l.
// The hardware hands consecutive thread blocks to the XCDs in turn (block i to XCD i mod 8).
// Reorders the blocks sched[first ..] (one bin of one LP, neighbouring rows in order) so that
// each XCD receives one contiguous eighth of them: rows of one XCD then gather from one stretch
// of the vector, which its own L2 holds, and every XCD still gets an equal share of the bin.
static void deal_to_xcds(std::vector<BlockDesc>& sched, size_t first) {
    const size_t n = sched.size() - first;
    if (n < 2 * (size_t)kXcds) return;
    std::vector<BlockDesc> part(sched.begin() + (std::ptrdiff_t)first, sched.end());
    size_t out = first;
    const size_t len = (n + kXcds - 1) / kXcds;      // blocks per eighth (the last may be short)
    for (size_t k = 0; k < len; ++k)
        for (size_t p = 0; p < (size_t)kXcds; ++p) {
            const size_t i = p * len + k;
            if (k < len && i < n && i < (p + 1) * len) sched[out++] = part[i];
        }
}

// Per row, the number of stored entries in each aligned tile of `tile` columns it touches.
struct TileCounts {
    int32_t tile = 0;
    std::vector<int64_t> ptr;     // [rows + 1]
    std::vector<int32_t> id, cnt;
};

// Sliced windows for a block that no single window serves: consecutive aligned windows of
// win_max columns (two tiles each), walked one at a time. Picks the run of at most kMaxSlices
// windows that saves the most (entries inside minus a quarter of the columns copied: a copied
// entry is one lane of a coalesced 16-byte load, a gathered one a scattered 4-byte access), if
// it holds at least half of the block's entries; then stores, per row, the number of its
// entries below each window boundary (rows are in column order, padding at the row's largest
// column).
static void slice_block(BlockDesc& d, const int32_t* rows_of_block,
                        const std::vector<std::pair<int32_t, int64_t>>& tiles, const TileCounts& tc, int64_t ncols,
                        int64_t entries, int32_t win_max, std::vector<int32_t>& cum) {
    if (tiles.empty() || win_max <= 0) return;
    const int64_t W = win_max;
    // entries per window id (tile / 2), windows in increasing order
    std::vector<std::pair<int64_t, int64_t>> win;
    for (const auto& t : tiles) {
        const int64_t j = t.first / 2;
        if (!win.empty() && win.back().first == j) win.back().second += t.second;
        else win.emplace_back(j, t.second);
    }
    double best_gain = 0.0;
    int64_t best_j0 = -1, best_ns = 0, best_in = 0;
    for (size_t a = 0; a < win.size(); ++a) {
        int64_t in = 0;
        for (size_t z = a; z < win.size(); ++z) {
            const int64_t ns = win[z].first - win[a].first + 1;
            if (ns > kMaxSlices) break;
            in += win[z].second;
            const int64_t lo = win[a].first * W;
            const int64_t copied = std::min<int64_t>(ns * W, ncols - lo);
            const double gain = (double)in - 0.25 * (double)copied;
            if (gain > best_gain) best_gain = gain, best_j0 = win[a].first, best_ns = ns, best_in = in;
        }
    }
    if (best_j0 < 0 || 2 * best_in < entries) return;
    d.wlo = (int32_t)(best_j0 * W);
    d.ns = (int32_t)best_ns;
    d.cum_first = (int32_t)cum.size();
    for (int32_t r = 0; r < d.count; ++r) {
        const int32_t i = rows_of_block[r];
        int64_t below = 0;   // entries of row i in tiles before the current boundary
        int64_t t = tc.ptr[i];
        for (int64_t k = 0; k <= best_ns; ++k) {
            const int64_t bound_tile = 2 * (best_j0 + k);
            while (t < tc.ptr[i + 1] && tc.id[t] < bound_tile) below += tc.cnt[t++];
            cum.push_back((int32_t)below);
        }
    }
}

// A block gets an LDS window of the gathered vector when its rows' columns span at most
// win_max entries, no row is wide, and the window is no larger than the block's number of
// stored entries (so copying it reads less than gathering from global memory would): the
// "full" window, wlen > 0. Otherwise, the two consecutive aligned tiles (2 tiles = win_max
// columns, clipped to the vector's ncols entries) holding most of the block's entries become
// a "split" window (wlen < 0) when they hold at least half of the entries and no fewer
// entries than the window has columns. Blocks that get neither may get sliced windows
// (`sliced`). With slice_cap >= 0, the rows of such blocks in bins above slice_cap are instead
// regrouped into blocks of bin slice_cap (2^slice_cap lanes per row, so more rows share each
// window copy) before their windows are sliced; rows stay in index order. With lane_cap >= 0
// every row of a bin above lane_cap goes to bin lane_cap (at most 2^lane_cap lanes per row)
// before blocks are formed, so full and split windows are shared by more rows too.
static void make_schedule_pass(const std::vector<int64_t>& start, const std::vector<int32_t>& base,
                               const std::vector<int32_t>& top, const std::vector<uint8_t>& wide,
                               const TileCounts& tc, int64_t ncols,
                               const std::vector<int64_t>& lp_rows, int U, int32_t win_max, bool split, bool sliced,
                               int slice_cap, int lane_cap, bool rounds, std::vector<RowRef>& rows,
                               std::vector<BlockDesc>& sched, std::vector<int32_t>& seg, std::vector<int32_t>& cum) {
    std::vector<std::pair<int32_t, int64_t>> tiles;
    cum.clear();
    const int L = (int)lp_rows.size() - 1;
    rows.clear();
    sched.clear();
    seg.assign((size_t)L + 1, 0);
    std::vector<int32_t> by_bin[kNumBins];
    std::vector<int32_t> deferred;   // rows of blocks to regroup at bin slice_cap
    // the block of rows list[0 .. count): its row list entries and its LDS windows; returns false
    // (nothing emitted) when the block is to be regrouped
    auto emit = [&](int b, int l, const int32_t* list, int32_t count, bool may_defer) -> bool {
        BlockDesc d;
        d.bin = b;
        d.lp = l;
        d.first = (int32_t)rows.size();
        d.count = count;
        int64_t wlo = INT64_MAX, whi = -1, entries = 0;
        bool any_wide = false;
        for (int32_t r = 0; r < count; ++r) {
            const int32_t i = list[r];
            const int32_t quads = (int32_t)((start[i + 1] - start[i]) / kVec);
            if (quads == 0) continue;
            any_wide = any_wide || wide[i];
            wlo = std::min<int64_t>(wlo, base[i]);
            whi = std::max<int64_t>(whi, top[i]);
            entries += (int64_t)quads * kVec;
        }
        d.wlo = 0;
        d.wlen = 0;
        d.ns = 0;
        d.cum_first = 0;
        if (whi >= 0) wlo -= wlo % 4;   // 16-byte aligned start for the window copy
        if (!any_wide && whi >= 0 && whi - wlo + 1 <= win_max && whi - wlo + 1 <= entries) {
            d.wlo = (int32_t)wlo;
            d.wlen = (int32_t)(whi - wlo + 1);
        } else if (split && tc.tile > 0 && entries > 0) {
            tiles.clear();
            for (int32_t r = 0; r < count; ++r) {
                const int32_t i = list[r];
                for (int64_t t = tc.ptr[i]; t < tc.ptr[i + 1]; ++t) tiles.emplace_back(tc.id[t], tc.cnt[t]);
            }
            std::sort(tiles.begin(), tiles.end());
            size_t w = 0;   // merge equal tiles
            for (size_t t = 0; t < tiles.size(); ++t) {
                if (w > 0 && tiles[w - 1].first == tiles[t].first) tiles[w - 1].second += tiles[t].second;
                else tiles[w++] = tiles[t];
            }
            tiles.resize(w);
            int64_t best = -1, best_in = 0;
            for (size_t t = 0; t < tiles.size(); ++t) {
                int64_t in = tiles[t].second;
                if (t + 1 < tiles.size() && tiles[t + 1].first == tiles[t].first + 1) in += tiles[t + 1].second;
                if (in > best_in) best_in = in, best = tiles[t].first;
            }
            if (best >= 0) {
                const int64_t lo = best * (int64_t)tc.tile;
                const int64_t len = std::min<int64_t>(2 * (int64_t)tc.tile, ncols - lo);
                if (len > 0 && 2 * best_in >= entries && best_in >= len) {
                    d.wlo = (int32_t)lo;
                    d.wlen = -(int32_t)len;
                }
            }
            if (d.wlen == 0 && sliced) {
                if (may_defer) {
                    deferred.insert(deferred.end(), list, list + count);
                    return false;
                }
                slice_block(d, list, tiles, tc, ncols, entries, win_max, cum);
            }
        }
        for (int32_t r = 0; r < count; ++r) {
            const int32_t i = list[r];
            const int32_t quads = (int32_t)((start[i + 1] - start[i]) / kVec);
            rows.push_back(RowRef{i, quads | (wide[i] ? kWide : 0), base[i], (int32_t)(start[i] / kVec)});
        }
        sched.push_back(d);
        return true;
    };
    // Rows per block: `count` rows (one round), or, for rows of at least 8 lanes (bin >= 3),
    // further rounds of per_block rows while the block's full window (every column of its rows,
    // at most win_max) spans at least win_max / 2 columns and is more than a quarter of its stored
    // entries, so that one large window copy serves more gathers; at most kMaxRounds rounds, and
    // only when the longer block still gets its full window. Blocks of shorter rows, or with
    // smaller windows, keep one round: rounds run the rows' latency chains (row entry, quads,
    // gathers, epilogue) one after another, which only a large copy saved pays for (measured:
    // rounds on the 2 KB windows of the 2,000-bus relaxation's security rows slowed its dual
    // step, on the 16 KB windows of the 13,500-bus one they sped it up).
    auto with_rounds = [&](int b, const int32_t* list, int32_t count, size_t left, int per_block) -> int32_t {
        if (!rounds || win_max <= 0 || b < 3) return count;
        struct Ext {
            int64_t lo = INT64_MAX, hi = -1, entries = 0;
            bool wide = false;
            int64_t span() const { return hi < 0 ? 0 : hi - (lo - lo % 4) + 1; }
        };
        auto add = [&](Ext x, int32_t from, int32_t to) {
            for (int32_t r = from; r < to; ++r) {
                const int32_t i = list[r];
                const int64_t quads = (start[i + 1] - start[i]) / kVec;
                if (quads == 0) continue;
                x.wide = x.wide || wide[i];
                x.lo = std::min<int64_t>(x.lo, base[i]);
                x.hi = std::max<int64_t>(x.hi, top[i]);
                x.entries += quads * kVec;
            }
            return x;
        };
        Ext cur = add(Ext{}, 0, count);
        if (cur.wide || cur.hi < 0 || cur.span() > win_max || 2 * cur.span() < win_max) return count;
        int32_t n = count;
        for (int round = 1; round < kMaxRounds && 4 * cur.span() > cur.entries && (size_t)n < left; ++round) {
            const int32_t m = (int32_t)std::min<size_t>((size_t)n + (size_t)per_block, left);
            const Ext next = add(cur, n, m);
            if (next.wide || next.span() > win_max) break;
            cur = next;
            n = m;
        }
        return (n > count && cur.span() > cur.entries) ? count : n;
    };
    for (int l = 0; l < L; ++l) {
        seg[l] = (int32_t)sched.size();
        for (auto& v : by_bin) v.clear();
        for (int64_t i = lp_rows[l]; i < lp_rows[l + 1]; ++i) {
            const int64_t quads = (start[i + 1] - start[i]) / kVec;
            int b = 0;
            while (b < kNumBins - 1 && (int64_t)U * (int64_t(1) << b) < quads) ++b;
            if (lane_cap >= 0 && b > lane_cap) b = lane_cap;   // longer rows take more passes
            by_bin[b].push_back((int32_t)i);
        }
        for (int b = 0; b < kNumBins; ++b) {
            const int per_block = kBlock >> b;
            const size_t bin_first = sched.size();
            const bool may_defer = sliced && slice_cap >= 0 && b > slice_cap;
            deferred.clear();
            for (size_t k = 0; k < by_bin[b].size();) {
                const int32_t* list = by_bin[b].data() + k;
                const size_t left = by_bin[b].size() - k;
                const int32_t count = with_rounds(b, list, (int32_t)std::min<size_t>(per_block, left), left, per_block);
                emit(b, l, list, count, may_defer);
                k += (size_t)count;
            }
            deal_to_xcds(sched, bin_first);
            if (!deferred.empty()) {   // regrouped: 2^slice_cap lanes per row
                const std::vector<int32_t> list = deferred;
                const int per = kBlock >> slice_cap;
                const size_t first = sched.size();
                for (size_t k = 0; k < list.size(); k += per)
                    emit(slice_cap, l, list.data() + k, (int32_t)std::min<size_t>(per, list.size() - k), false);
                deal_to_xcds(sched, first);
            }
        }
    }
    seg[L] = (int32_t)sched.size();
}

// The schedule, with blocks in rounds only where they carry at least a quarter of the stored
// entries: a schedule with any such block runs the product kernels' instantiation with the round
// loop (a few more registers), which a handful of such blocks does not pay for.
static void make_schedule(const std::vector<int64_t>& start, const std::vector<int32_t>& base,
                          const std::vector<int32_t>& top, const std::vector<uint8_t>& wide,
                          const TileCounts& tc, int64_t ncols,
                          const std::vector<int64_t>& lp_rows, int U, int32_t win_max, bool split, bool sliced,
                          int slice_cap, int lane_cap, std::vector<RowRef>& rows, std::vector<BlockDesc>& sched,
                          std::vector<int32_t>& seg, std::vector<int32_t>& cum) {
    make_schedule_pass(start, base, top, wide, tc, ncols, lp_rows, U, win_max, split, sliced, slice_cap, lane_cap,
                       true, rows, sched, seg, cum);
    int64_t in_rounds = 0, all = 0;
    for (const BlockDesc& d : sched) {
        int64_t q = 0;
        for (int32_t r = 0; r < d.count; ++r) q += rows[(size_t)d.first + r].quads & ~kWide;
        all += q;
        if (d.count > (kBlock >> d.bin)) in_rounds += q;
    }
    if (in_rounds > 0 && 4 * in_rounds < all)
        make_schedule_pass(start, base, top, wide, tc, ncols, lp_rows, U, win_max, split, sliced, slice_cap,
                           lane_cap, false, rows, sched, seg, cum);
}

// lds_windows modes 4 and 5: sliced blocks regrouped with 16 and 8 lanes per row (bins 4, 3);
// modes 6 and 7: every row capped at 16 and 8 lanes
static int slice_cap_of(int mode) { return mode == 4 ? 4 : (mode == 5 ? 3 : -1); }
static int lane_cap_of(int mode) { return mode == 6 ? 4 : (mode == 7 ? 3 : -1); }

struct DevMatrix {
    DBuf start, col, col16, qpack, rows, sched, seg, val64, val32, slice_cum;
    int64_t narrow_quads = 0, packed_quads = 0;  // quads of 16-bit-offset rows, and those packed
    bool use_pack = false;                       // the products read the packed words
    DBuf sched_act, seg_act;                 // compacted schedule: the blocks of running LPs only
    std::vector<int64_t> start_h, lp_rows;   // host copies for rescheduling
    std::vector<int32_t> base_h, top_h;
    std::vector<uint8_t> wide_h;
    int32_t win_max = 0;                     // LDS window limit in vector entries
    int32_t win_mode = 2;                    // 0: no windows, 1: full, 2: full and split, 3: and sliced,
                                             // 4, 5: sliced blocks regrouped (16, 8 lanes per row),
                                             // 6, 7: every row at most 16, 8 lanes
    int32_t has_sliced = 0;                  // the current schedule has sliced blocks
    int32_t has_rounds = 0;                  // ... blocks that take their rows in rounds
    TileCounts tiles;
    int64_t ncols = 0;                       // length of the gathered vector
    std::vector<BlockDesc> sched_h;
    std::vector<int32_t> seg_h;
    int32_t nrows = 0, nblocks = 0, nblocks_act = 0, unroll = 4, nontemporal = 0;
    bool use_act = false;
    int64_t padded = 0;
    HostVec<uint16_t> c16;                   // 16-bit offsets between host preparation and upload
    // host part of the upload (no HIP calls; A and A^T are prepared on two threads)
    void prepare(const Layout& L, const std::vector<int64_t>& lp_rows_in, int64_t ncols_in, bool fp32,
                 int lds_windows, int threads) {
        nrows = (int32_t)L.start.size() - 1;
        ncols = ncols_in;
        win_mode = lds_windows < 0 ? 2 : lds_windows;
        padded = (int64_t)L.col.size();
        start_h.assign(L.start.begin(), L.start.end());
        lp_rows = lp_rows_in;
        short_indices(L, c16, base_h, top_h, wide_h, threads);
        win_max = kWinBytes / (fp32 ? (int)sizeof(float) : (int)sizeof(double));
        count_tiles(L, win_max / 2, threads);
    }
    void upload_from(const Layout& L, bool fp32, hipStream_t st) {
        if (padded / kVec >= INT32_MAX) {
            fail(HPR_ERR_INVALID, "matrix too large: more than 2^33 stored entries");
            throw HipError{HPR_ERR_INVALID};
        }
        upload(start, L.start, st);
        upload(col, L.col, st);
        upload(col16, c16, st);
        pack(st);
        HostVec<uint16_t>().swap(c16);
        upload(val64, L.val, st);
        if (fp32) {
            val32.alloc(L.val.size() * sizeof(float));
            launch_cast<float>(val64.as<double>(), val32.as<float>(), (int64_t)L.val.size(), st);
        }
        set_unroll(4, st);
    }
    // Takes over a layout built on the device (device_setup): the device buffers become this
    // matrix's, and the per-row metadata the schedules need is copied to the host.
    void adopt(DevLayout& L, const std::vector<int64_t>& lp_rows_in, int32_t rows, int64_t ncols_in, bool fp32,
               int lds_windows, hipStream_t st) {
        nrows = rows;
        ncols = ncols_in;
        win_mode = lds_windows < 0 ? 2 : lds_windows;
        padded = L.padded;
        lp_rows = lp_rows_in;
        win_max = kWinBytes / (fp32 ? (int)sizeof(float) : (int)sizeof(double));
        if (padded / kVec >= INT32_MAX) {
            fail(HPR_ERR_INVALID, "matrix too large: more than 2^33 stored entries");
            throw HipError{HPR_ERR_INVALID};
        }
        start_h.resize((size_t)rows + 1);
        base_h.resize(rows);
        top_h.resize(rows);
        wide_h.resize(rows);
        tiles.tile = win_max / 2;
        tiles.ptr.resize((size_t)rows + 1);
        tiles.id.resize(L.nruns);
        tiles.cnt.resize(L.nruns);
        auto get = [&](void* dst, const DevScratch& src, size_t bytes) {
            if (bytes) HIP_OK(hipMemcpyAsync(dst, src.p, bytes, hipMemcpyDeviceToHost, st));
        };
        get(start_h.data(), L.start, sizeof(int64_t) * ((size_t)rows + 1));
        get(base_h.data(), L.base, sizeof(int32_t) * rows);
        get(top_h.data(), L.top, sizeof(int32_t) * rows);
        get(wide_h.data(), L.wide, rows);
        get(tiles.ptr.data(), L.tptr, sizeof(int64_t) * ((size_t)rows + 1));
        get(tiles.id.data(), L.tid, sizeof(int32_t) * L.nruns);
        get(tiles.cnt.data(), L.tcnt, sizeof(int32_t) * L.nruns);
        HIP_OK(hipStreamSynchronize(st));
        auto take = [](DBuf& d, DevScratch& src) {
            d.release();
            d.bytes = src.cap;
            d.p = src.release();
        };
        take(start, L.start);
        take(col, L.col);
        take(col16, L.col16);
        take(val64, L.val64);
        if (fp32) take(val32, L.val32);
        pack(st);
        set_unroll(4, st);
    }
    // qpack from col16 (start, col16 and wide_h in place); waits for the stream
    void pack(hipStream_t st) {
        const int64_t nq = padded / kVec;
        qpack.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nq, 1));
        DBuf wd, cnt;
        upload(wd, wide_h, st);
        cnt.alloc(2 * sizeof(unsigned long long));
        HIP_OK(hipMemsetAsync(cnt.p, 0, 2 * sizeof(unsigned long long), st));
        launch_pack_quads(col16.as<uint16_t>(), start.as<int64_t>(), wd.as<uint8_t>(), nrows, nq,
                          qpack.as<uint32_t>(), static_cast<unsigned long long*>(cnt.p), st);
        HIP_OK(hipGetLastError());
        unsigned long long h[2] = {0, 0};
        HIP_OK(hipMemcpyAsync(h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, st));
        sync_stream(st);
        narrow_quads = (int64_t)h[0];
        packed_quads = (int64_t)h[1];
        // an unpacked quad costs its packed word and its 16-bit offsets (12 bytes instead of 8)
        // and a dependent load: measured, 82% packed quads made the 13,500-bus dual step slower
        // (5-bit gaps) and 98% made the 2,000-bus one faster, so the words are read only from 90% on
        use_pack = narrow_quads > 0 && packed_quads >= 0.9 * (double)narrow_quads;
        if (!use_pack) qpack.release();
    }
    void count_tiles(const Layout& L, int32_t tile, int threads) {
        // rows are in column order: a row's tiles are runs of equal col / tile; counted first,
        // then written, rows in ranges on several threads
        tiles.tile = tile;
        tiles.ptr.assign((size_t)nrows + 1, 0);
        constexpr int kChunks = 64;
        parallel_for(kChunks, threads, [&](int p) {
            for (int64_t i = (int64_t)nrows * p / kChunks; i < (int64_t)nrows * (p + 1) / kChunks; ++i) {
                int64_t runs = 0;
                for (int64_t k = L.start[i]; k < L.start[i + 1]; ++k)
                    runs += (k == L.start[i] || L.col[k] / tile != L.col[k - 1] / tile) ? 1 : 0;
                tiles.ptr[i + 1] = runs;
            }
        });
        for (int32_t i = 0; i < nrows; ++i) tiles.ptr[i + 1] += tiles.ptr[i];
        tiles.id.resize(tiles.ptr[nrows]);
        tiles.cnt.resize(tiles.ptr[nrows]);
        parallel_for(kChunks, threads, [&](int p) {
            for (int64_t i = (int64_t)nrows * p / kChunks; i < (int64_t)nrows * (p + 1) / kChunks; ++i) {
                int64_t q = tiles.ptr[i] - 1;
                for (int64_t k = L.start[i]; k < L.start[i + 1]; ++k) {
                    const int32_t t = L.col[k] / tile;
                    if (k == L.start[i] || t != L.col[k - 1] / tile) {
                        ++q;
                        tiles.id[q] = t;
                        tiles.cnt[q] = 0;
                    }
                    ++tiles.cnt[q];
                }
            }
        });
    }
    // host schedules already built for a U (kept while the tuner switches between them)
    struct Built {
        int U, mode;
        std::vector<RowRef> rows;
        std::vector<BlockDesc> sched;
        std::vector<int32_t> seg;
        std::vector<int32_t> cum;
    };
    std::vector<Built> built;
    // builds the host schedules of the given (U, window mode) pairs that are not built yet,
    // on several threads (host only)
    void prebuild(const std::vector<std::pair<int, int>>& cands, int threads) {
        std::vector<size_t> todo;
        for (const auto& c : cands) {
            bool have = false;
            for (const Built& x : built) have = have || (x.U == c.first && x.mode == c.second);
            for (size_t t : todo) have = have || (built[t].U == c.first && built[t].mode == c.second);
            if (!have) {
                built.push_back(Built{c.first, c.second, {}, {}, {}, {}});
                todo.push_back(built.size() - 1);
            }
        }
        parallel_for((int)todo.size(), threads, [&](int i) {
            Built& b = built[todo[i]];
            make_schedule(start_h, base_h, top_h, wide_h, tiles, ncols, lp_rows, b.U, b.mode >= 1 ? win_max : 0,
                          b.mode >= 2, b.mode >= 3, slice_cap_of(b.mode), lane_cap_of(b.mode), b.rows, b.sched,
                          b.seg, b.cum);
        });
    }
    void set_unroll(int U, hipStream_t st) {
        const Built* b = nullptr;
        for (const Built& x : built)
            if (x.U == U && x.mode == win_mode) b = &x;
        if (!b) {
            built.push_back(Built{U, win_mode, {}, {}, {}, {}});
            make_schedule(start_h, base_h, top_h, wide_h, tiles, ncols, lp_rows, U, win_mode >= 1 ? win_max : 0,
                          win_mode >= 2, win_mode >= 3, slice_cap_of(win_mode), lane_cap_of(win_mode),
                          built.back().rows, built.back().sched, built.back().seg, built.back().cum);
            b = &built.back();
        }
        unroll = U;
        nblocks = (int32_t)b->sched.size();
        upload(rows, b->rows, st);
        upload(sched, b->sched, st);
        upload(seg, b->seg, st);
        if (!b->cum.empty()) upload(slice_cum, b->cum, st);
        HIP_OK(hipStreamSynchronize(st));
        sched_h = b->sched;
        seg_h = b->seg;
        has_sliced = has_rounds = 0;
        for (const BlockDesc& d : sched_h) {
            has_sliced |= d.ns > 0 ? 1 : 0;
            has_rounds |= d.count > (kBlock >> d.bin) ? 1 : 0;
        }
        use_act = false;
    }
    void window_counts(int32_t& full, int32_t& split, int32_t& sliced, int32_t& all, int32_t& rounds) const {
        full = split = sliced = rounds = 0;
        for (const BlockDesc& d : sched_h) {
            if (d.count > (kBlock >> d.bin)) ++rounds;
            if (d.wlen > 0) ++full;
            if (d.wlen < 0) ++split;
            if (d.ns > 0) ++sliced;
        }
        all = (int32_t)sched_h.size();
    }
    // after tuning: no further schedules are built
    void drop_built() {
        std::vector<Built>().swap(built);
        tiles = TileCounts{};
    }
    // Launch only the blocks of the LPs with running[l] != 0 (each LP's blocks stay in their
    // order, so per-block partial sums and their per-LP totals are unchanged).
    void compact(const std::vector<int32_t>& running, hipStream_t st) {
        const int L = (int)seg_h.size() - 1;
        std::vector<BlockDesc> sc;
        std::vector<int32_t> sg((size_t)L + 1, 0);
        for (int l = 0; l < L; ++l) {
            sg[l] = (int32_t)sc.size();
            if (running[l]) sc.insert(sc.end(), sched_h.begin() + seg_h[l], sched_h.begin() + seg_h[l + 1]);
        }
        sg[L] = (int32_t)sc.size();
        nblocks_act = (int32_t)sc.size();
        upload(sched_act, sc, st);
        upload(seg_act, sg, st);
        HIP_OK(hipStreamSynchronize(st));   // sc and sg are local
        use_act = true;
    }
    void full() { use_act = false; }
    const int32_t* seg_ptr() const { return use_act ? seg_act.as<int32_t>() : seg.as<int32_t>(); }
    template <typename T>
    DevCsr<T> view() const {
        DevCsr<T> d;
        d.col = col.as<int32_t>();
        d.col16 = col16.as<uint16_t>();
        d.qpack = use_pack ? qpack.as<uint32_t>() : nullptr;
        d.val = std::is_same<T, float>::value ? (const T*)val32.p : (const T*)val64.p;
        d.rows = rows.as<RowRef>();
        d.sched = use_act ? sched_act.as<BlockDesc>() : sched.as<BlockDesc>();
        d.nblocks = use_act ? nblocks_act : nblocks;
        d.unroll = unroll;
        d.nontemporal = nontemporal;
        d.slice_cum = slice_cum.as<int32_t>();
        d.slice_w = win_max;
        d.ncols = (int32_t)ncols;
        d.has_sliced = has_sliced;
        d.has_rounds = has_rounds;
        return d;
    }
};

// ---------------------------------------------------------------- the engine (one LP or a batch)

struct Engine {
    int L = 0;
    int64_t M = 0, N = 0;                       // pooled rows and columns
    hpr_opts opts{};
    bool fp32 = false;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0;
    std::vector<LpHost> lps;

    DevMatrix A, At;
    DBuf c64, l64, u64, lo64, hi64, c32, l32, u32, lo32, hi32, dr_d, dc_d;
    DBuf x, x0, xh, xb, zb, dx, y, y0, yb, dy;
    DBuf part_r, part_c, sums, sums64, ctrl, state, stat;
    DBuf ux, uy, uz;
    int32_t* stat_h = nullptr;                  // pinned
    std::vector<Ctrl> ctrl_h;
    std::vector<LpState> state_h;

    hipGraphExec_t g_first = nullptr, g_block = nullptr;
    bool graphs_built = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // primal start/stop, dual start/stop
    hpr_kernel_stats kstats{};
    bool solved_once = false;
    double setup_s = 0, solve_s = 0;
    double t_prep = 0, t_upload = 0, t_tune = 0, t_power = 0;   // phases of hpr_create
    std::vector<double> done_at;             // per LP: seconds into the solve when it stopped
    std::vector<int32_t> warm_used, use_start_mask;   // per LP: solve started from the caller's point

    ~Engine() {
        if (st) (void)hipStreamSynchronize(st);
        drop_graphs();
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (stat_h) (void)hipHostFree(stat_h);
        if (own_stream && st) (void)hipStreamDestroy(st);
    }
    void drop_graphs() {
        if (g_first) (void)hipGraphExecDestroy(g_first);
        if (g_block) (void)hipGraphExecDestroy(g_block);
        g_first = g_block = nullptr;
        graphs_built = false;
    }
    void sync() { HIP_OK(hipStreamSynchronize(st)); }

    template <typename T>
    DevProb<T> prob() const {
        DevProb<T> p;
        const bool f = std::is_same<T, float>::value;
        p.c = (const T*)(f ? c32.p : c64.p);
        p.l = (const T*)(f ? l32.p : l64.p);
        p.u = (const T*)(f ? u32.p : u64.p);
        p.lo = (const T*)(f ? lo32.p : lo64.p);
        p.hi = (const T*)(f ? hi32.p : hi64.p);
        p.dr = dr_d.as<double>();
        p.dc = dc_d.as<double>();
        return p;
    }
    template <typename T>
    DevIter<T> iter() const {
        DevIter<T> v;
        v.x = x.as<T>(); v.x0 = x0.as<T>(); v.xh = xh.as<T>(); v.xb = xb.as<T>(); v.zb = zb.as<T>();
        v.dx = dx.as<T>();
        v.y = y.as<T>(); v.y0 = y0.as<T>(); v.yb = yb.as<T>(); v.dy = dy.as<T>();
        return v;
    }
};

extern "C" void hpr_default_opts(hpr_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-4;
    o->max_iter = 1000000;
    o->time_limit_s = 0;
    o->precision = HPR_FP64;
    o->scaling = HPR_SCALE_PC | HPR_SCALE_BC;
    o->ruiz_iters = 10;
    o->check_every = 64;
    o->sigma0 = 1.0;
    o->lambda = 0.0;
    o->seed = 0;
    o->restart = 1;
    o->sigma_update = 1;
    o->power_max_iter = 200;
    o->power_tol = 1e-6;
    o->profile = 0;
    o->unroll = 0;
    o->lds_windows = -1;
    o->use_graph = 1;
    o->warm_fallback = 2;
    o->warm_fallback_ratio = 1000.0;
    o->sigma_smoothing = 1.0;
    o->sigma_smoothing_warm = 0.5;
    o->stall_iters = 0;
    o->stream = nullptr;
}

extern "C" const char* hpr_last_error(void) { return g_err.c_str(); }

// upload the pooled scaled vectors (and their FP32 copies)
static void upload_vectors(Engine* e) {
    std::vector<double> c(e->N), l(e->N), u(e->N), dc(e->N), lo(e->M), hi(e->M), dr(e->M);
    for (const LpHost& h : e->lps) {
        std::copy(h.c_s.begin(), h.c_s.end(), c.begin() + h.col_off);
        std::copy(h.l_s.begin(), h.l_s.end(), l.begin() + h.col_off);
        std::copy(h.u_s.begin(), h.u_s.end(), u.begin() + h.col_off);
        std::copy(h.dc.begin(), h.dc.end(), dc.begin() + h.col_off);
        std::copy(h.lo_s.begin(), h.lo_s.end(), lo.begin() + h.row_off);
        std::copy(h.hi_s.begin(), h.hi_s.end(), hi.begin() + h.row_off);
        std::copy(h.dr.begin(), h.dr.end(), dr.begin() + h.row_off);
    }
    hipStream_t st = e->st;
    upload(e->c64, c, st);
    upload(e->l64, l, st);
    upload(e->u64, u, st);
    upload(e->lo64, lo, st);
    upload(e->hi64, hi, st);
    upload(e->dr_d, dr, st);
    upload(e->dc_d, dc, st);
    if (e->fp32) {
        const int64_t n = e->N, m = std::max<int64_t>(e->M, 1);
        e->c32.alloc(sizeof(float) * n);
        e->l32.alloc(sizeof(float) * n);
        e->u32.alloc(sizeof(float) * n);
        e->lo32.alloc(sizeof(float) * m);
        e->hi32.alloc(sizeof(float) * m);
        launch_cast<float>(e->c64.as<double>(), e->c32.as<float>(), e->N, st);
        launch_cast<float>(e->l64.as<double>(), e->l32.as<float>(), e->N, st);
        launch_cast<float>(e->u64.as<double>(), e->u32.as<float>(), e->N, st);
        launch_cast<float>(e->lo64.as<double>(), e->lo32.as<float>(), e->M, st);
        launch_cast<float>(e->hi64.as<double>(), e->hi32.as<float>(), e->M, st);
    }
    e->sync();   // the host vectors above are locals
}

static void alloc_iterates(Engine* e) {
    const size_t es = e->fp32 ? sizeof(float) : sizeof(double);
    const size_t n = (size_t)e->N, m = (size_t)std::max<int64_t>(e->M, 1);
    for (DBuf* b : {&e->x, &e->x0, &e->xh, &e->xb, &e->zb, &e->dx}) b->alloc(es * n);
    for (DBuf* b : {&e->y, &e->y0, &e->yb, &e->dy}) b->alloc(es * m);
    e->sums.alloc(sizeof(double) * kSumStride * e->L);
    e->sums64.alloc(sizeof(double) * kSumStride * e->L);
    e->ctrl.alloc(sizeof(Ctrl) * e->L);
    e->state.alloc(sizeof(LpState) * e->L);
    e->stat.alloc(sizeof(int32_t) * 2);
    e->ux.alloc(sizeof(double) * n);
    e->uy.alloc(sizeof(double) * m);
    e->uz.alloc(sizeof(double) * n);
    HIP_OK(hipHostMalloc((void**)&e->stat_h, sizeof(int32_t) * 2, hipHostMallocDefault));
    e->ctrl_h.assign(e->L, Ctrl{});
    e->state_h.assign(e->L, LpState{});
}

static void alloc_partials(Engine* e) {
    e->part_r.alloc(sizeof(double) * kRowQ * std::max(e->A.nblocks, 1));
    e->part_c.alloc(sizeof(double) * kColQ * std::max(e->At.nblocks, 1));
}

static void put_ctrl(Engine* e) {
    HIP_OK(hipMemcpyAsync(e->ctrl.p, e->ctrl_h.data(), sizeof(Ctrl) * e->L, hipMemcpyHostToDevice, e->st));
    e->sync();
}

// Choices of the schedule tuner, kept for the life of the process and keyed by a coarse signature
// of the matrix (which step streams it, value width, window size, whether it reads packed words,
// its stored entries and rows on a 1/8-octave grid, and the share of its entries in rows of each
// length class to 1%): the LPs of successive-fixing rounds and of a batch's members repeat such
// signatures, and re-timing them would cost a tenth of a second per handle.
struct TuneKey {
    int32_t which, vbytes, win, pack, entries_q, rows_q;
    std::array<int16_t, 12> share;
    bool operator<(const TuneKey& o) const {
        return std::tie(which, vbytes, win, pack, entries_q, rows_q, share) <
               std::tie(o.which, o.vbytes, o.win, o.pack, o.entries_q, o.rows_q, o.share);
    }
};
struct TuneChoice {
    int32_t U, mode, nt;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune_cache;

static TuneKey tune_key(const DevMatrix& M, int which, int vbytes) {
    TuneKey k{};
    k.which = which;
    k.vbytes = vbytes;
    k.win = M.win_max;
    k.pack = M.use_pack ? 1 : 0;
    k.entries_q = (int32_t)std::lround(8.0 * std::log2(1.0 + (double)M.padded));
    k.rows_q = (int32_t)std::lround(8.0 * std::log2(1.0 + (double)M.nrows));
    std::array<int64_t, 12> ent{};
    for (int32_t i = 0; i < M.nrows; ++i) {
        const int64_t quads = (M.start_h[i + 1] - M.start_h[i]) / kVec;
        int b = 0;
        while (b < 10 && (int64_t(1) << b) < quads) ++b;
        ent[M.wide_h[i] ? 11 : b] += quads;
    }
    const double tot = std::max<double>(1.0, (double)(M.padded / kVec));
    for (int b = 0; b < 12; ++b) k.share[b] = (int16_t)std::lround(100.0 * (double)ent[b] / tot);
    return k;
}

// Schedule tuner: for each pooled matrix, time the fused step kernel that streams it (dual
// step for A~, primal step for A~^T) with U = 1, 2, 4 quads per lane and pass, then the best U
// with ordinary and with non-temporal loads of the matrix, and keep the fastest (or take the
// choice made for a matrix of the same signature earlier in the process). A forced
// opts.unroll skips all timing (ordinary loads), so two engines with the same forced options
// run the same schedule (same summation order, bitwise equal results).
template <typename T>
static void autotune(Engine* e) {
    hipStream_t st = e->st;
    for (DBuf* b : {&e->x, &e->x0, &e->xh, &e->xb, &e->zb, &e->dx, &e->y, &e->y0, &e->yb, &e->dy})
        HIP_OK(hipMemsetAsync(b->p, 0, b->bytes, st));
    for (int l = 0; l < e->L; ++l) {
        Ctrl& c = e->ctrl_h[l];
        c = Ctrl{};
        c.sigma = 1.0;
        c.s = 1.0;
        c.lambda = 1.0;
        c.beta_b = e->lps[l].beta_b;
        c.beta_c = e->lps[l].beta_c;
        c.active = 1;
    }
    put_ctrl(e);
    const int fU = e->opts.unroll;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const DevProb<T> p = e->prob<T>();
    const DevIter<T> v = e->iter<T>();
    for (int which = 0; which < 2; ++which) {
        DevMatrix& Mx = which == 0 ? e->A : e->At;
        Mx.nontemporal = 0;
        if (fU || Mx.nrows == 0) {
            Mx.set_unroll(fU ? fU : 4, st);
            Mx.drop_built();
            continue;
        }
        const bool tune_split = e->opts.lds_windows < 0;
        const TuneKey key = tune_key(Mx, which, (int)sizeof(T));
        if (tune_split) {
            TuneChoice hit{0, 0, 0};
            {
                std::lock_guard<std::mutex> lock(g_tune_mu);
                const auto it = g_tune_cache.find(key);
                if (it != g_tune_cache.end()) hit = it->second;
            }
            if (hit.U) {
                Mx.win_mode = hit.mode;
                Mx.set_unroll(hit.U, st);
                Mx.nontemporal = hit.nt;
                Mx.drop_built();
                continue;
            }
        }
        auto time_it = [&]() {
            const DevCsr<T> view = Mx.view<T>();
            auto launch = [&]() {
                if (which == 0) launch_dual_step<T>(view, p, v, e->ctrl.as<Ctrl>(), 0, false, st);
                else launch_primal_step<T>(view, p, v, e->ctrl.as<Ctrl>(), 0, false, st);
            };
            launch();
            HIP_OK(hipEventRecord(e0, st));
            for (int r = 0; r < 5; ++r) launch();
            HIP_OK(hipEventRecord(e1, st));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        // candidates (U, and split windows on/off when the option leaves that open) timed in
        // interleaved rounds, each keeping its fastest round, so that a clock ramp during the
        // first rounds does not favour the later candidates
        struct Cand {
            int U, mode;
            float ms;
        };
        std::vector<Cand> cand;
        for (int U : {1, 2, 4}) {
            if (tune_split) {
                for (int mode : {1, 2, 3, 4, 5, 6, 7}) cand.push_back(Cand{U, mode, 1e30f});
            } else {
                cand.push_back(Cand{U, Mx.win_mode, 1e30f});
            }
        }
        {
            std::vector<std::pair<int, int>> pairs;
            for (const Cand& c : cand) pairs.emplace_back(c.U, c.mode);
            Mx.prebuild(pairs, host_threads());
            // a mode that adds no block of its kind gives the same schedule as the mode below it
            std::vector<Cand> kept;
            for (const Cand& c : cand) {
                bool same = false;
                if (tune_split && c.mode >= 2 && c.mode <= 5)
                    for (const DevMatrix::Built& b : Mx.built)
                        if (b.U == c.U && b.mode == c.mode) {
                            // modes 3-5 differ from mode 2 only where blocks are sliced
                            bool adds = false;
                            for (const BlockDesc& d : b.sched) adds = adds || (c.mode == 2 ? d.wlen < 0 : d.ns > 0);
                            same = !adds;
                        }
                if (!same && c.mode >= 4) {   // a regrouping or cap that changes nothing repeats a lower mode
                    const DevMatrix::Built *me = nullptr, *lower = nullptr;
                    for (const DevMatrix::Built& b : Mx.built) {
                        if (b.U == c.U && b.mode == c.mode) me = &b;
                        if (b.U == c.U && b.mode == c.mode - 1) lower = &b;
                    }
                    if (me && lower && me->sched.size() == lower->sched.size() &&
                        std::memcmp(me->sched.data(), lower->sched.data(), sizeof(BlockDesc) * me->sched.size()) == 0)
                        same = true;
                }
                if (!same) kept.push_back(c);
            }
            cand.swap(kept);
        }
        for (int round = 0; round < 2; ++round)
            for (Cand& c : cand) {
                Mx.win_mode = c.mode;
                Mx.set_unroll(c.U, st);
                c.ms = std::min(c.ms, time_it());
            }
        const Cand* best = &cand[0];
        for (const Cand& c : cand)
            if (c.ms < best->ms) best = &c;
        Mx.win_mode = best->mode;
        Mx.set_unroll(best->U, st);
        float ms_plain = 1e30f, ms_nt = 1e30f;
        for (int round = 0; round < 2; ++round) {
            Mx.nontemporal = 0;
            ms_plain = std::min(ms_plain, time_it());
            Mx.nontemporal = 1;
            ms_nt = std::min(ms_nt, time_it());
        }
        Mx.nontemporal = ms_nt < ms_plain ? 1 : 0;
        if (tune_split) {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tune_cache[key] = TuneChoice{best->U, best->mode, Mx.nontemporal};
        }
        Mx.drop_built();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_OK(hipGetLastError());
}

// lambda_l = lambda_max(A~_l A~_l^T) for every LP by the power method in FP64 on the pooled
// matrix: v <- A~(A~^T v), normalised per LP; estimate ||A~ A~^T v|| for unit v; an LP stops
// at relative change <= power_tol or after power_max_iter products; lambda = 1.01 * estimate,
// capped at 1 when the Pock-Chambolle scaling is on (it bounds ||A~|| by 1), and 1 when the
// estimate is 0. Start vectors: SplitMix64 with LP-local indices. The norms and the
// normalisation stay on the device; every estimate is kept in a history that the host reads
// every kPowerChunk products and replays the stopping rule on, in order (products after an
// LP's stop change nothing it reports).
static void power_method(Engine* e) {
    constexpr int kPowerChunk = 8;
    const int L = e->L;
    hipStream_t st = e->st;
    std::vector<int64_t> seg(L + 1);
    int max_chunks = 1;
    for (int l = 0; l < L; ++l) {
        seg[l] = e->lps[l].row_off;
        max_chunks = std::max<int>(max_chunks, (int)((e->lps[l].m + kChunk - 1) / kChunk));
    }
    seg[L] = e->M;
    std::vector<int32_t> bseg(L + 1);
    for (int l = 0; l <= L; ++l) bseg[l] = l * max_chunks;
    std::vector<char> done(L, 0);
    std::vector<double> est(L, 0.0), prev(L, 0.0);
    for (int l = 0; l < L; ++l)
        if (e->lps[l].m == 0 || e->lps[l].nnz == 0) done[l] = 1;
    const bool any = std::find(done.begin(), done.end(), 0) != done.end();
    if (any) {
        const int maxit = e->opts.power_max_iter;
        DBuf v, t, w, part, segd, bsegd, fac, hist;
        v.alloc(sizeof(double) * std::max<int64_t>(e->M, 1));
        w.alloc(sizeof(double) * std::max<int64_t>(e->M, 1));
        t.alloc(sizeof(double) * std::max<int64_t>(e->N, 1));
        part.alloc(sizeof(double) * L * max_chunks);
        upload(segd, seg, st);
        upload(bsegd, bseg, st);
        fac.alloc(sizeof(double) * L);
        hist.alloc(sizeof(double) * L * (size_t)(kPowerChunk + 1));
        std::vector<double> hist_h((size_t)L * kPowerChunk);
        const DevCsr<double> A = e->A.view<double>(), At = e->At.view<double>();
        // norms of p per LP into hist row `slot`, and p scaled to unit norm
        auto normalise = [&](double* p, int slot) {
            launch_seg_sumsq(p, segd.as<int64_t>(), L, max_chunks, part.as<double>(), st);
            launch_finish_sums(part.as<double>(), 1, L * max_chunks, bsegd.as<int32_t>(), L, e->sums.as<double>(), 0,
                               st);
            launch_power_norms(e->sums.as<double>(), L, hist.as<double>() + (size_t)slot * L, fac.as<double>(), st);
            launch_seg_scale(p, segd.as<int64_t>(), L, max_chunks, fac.as<double>(), st);
        };
        launch_seg_start_vector(v.as<double>(), segd.as<int64_t>(), L, max_chunks, e->opts.seed, st);
        normalise(v.as<double>(), kPowerChunk);
        for (int it0 = 1; it0 <= maxit; it0 += kPowerChunk) {
            const int n = std::min(kPowerChunk, maxit - it0 + 1);
            for (int k = 0; k < n; ++k) {
                launch_spmv<double>(At, v.as<double>(), t.as<double>(), st);
                launch_spmv<double>(A, t.as<double>(), w.as<double>(), st);
                normalise(w.as<double>(), k);
                std::swap(v.p, w.p);
            }
            HIP_OK(hipGetLastError());
            HIP_OK(hipMemcpyAsync(hist_h.data(), hist.p, sizeof(double) * L * n, hipMemcpyDeviceToHost, st));
            e->sync();
            bool all = true;
            for (int l = 0; l < L; ++l) {
                for (int k = 0; k < n && !done[l]; ++k) {
                    const int it = it0 + k;
                    const double s = hist_h[(size_t)k * L + l];
                    est[l] = s;
                    if (s == 0.0) done[l] = 1;
                    else if (it > 1 && std::fabs(s - prev[l]) <= e->opts.power_tol * s) done[l] = 1;
                    else prev[l] = s;
                }
                all = all && done[l];
            }
            if (all) break;
        }
    }
    for (int l = 0; l < L; ++l) {
        LpHost& h = e->lps[l];
        if (h.m == 0 || h.nnz == 0 || est[l] == 0.0) {
            h.lambda = 1.0;
            continue;
        }
        double lam = 1.01 * est[l];
        if ((e->opts.scaling & HPR_SCALE_PC) && lam > 1.0) lam = 1.0;
        h.lambda = lam;
    }
}

// Host preparation of one LP: scaling and the padded layouts of A~ and A~^T (independent per
// LP, so a batch prepares several LPs at once with one thread each; a single LP uses several).
struct PrepLp {
    LpHost h;
    Layout la, lt;
};

static void prep_lp(const hpr_lp* lp, const hpr_opts& o, PrepLp& p, int threads) {
    const std::vector<int32_t> cut = row_parts(lp);
    ColOrder co;
    column_order(lp, cut, threads, co);
    scale_factors(lp, o, p.h, co, threads);
    scale_vectors(lp, o, p.h);
    make_layouts(lp, p.h, co, cut, threads, p.la, p.lt);
}

// An LP whose arrays are device memory (hpr_lp.on_device), read into host copies on `st`.
struct StagedLp {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v, lo, hi, l, u, c;
    hpr_lp lp{};
};

static int stage_device_lp(const hpr_lp* in, hipStream_t st, StagedLp& s) {
    if (in->n < 1 || in->m < 0 || in->nnz < 0) return fail(HPR_ERR_INVALID, "bad m, n or nnz");
    if (in->m == 0 && in->nnz != 0) return fail(HPR_ERR_INVALID, "nnz must be 0 when m = 0");
    if (!in->col_lo || !in->col_hi || !in->c) return fail(HPR_ERR_INVALID, "col_lo, col_hi and c are required");
    if (in->m > 0 && (!in->row_ptr || !in->row_lo || !in->row_hi))
        return fail(HPR_ERR_INVALID, "row_ptr, row_lo and row_hi are required when m > 0");
    if (in->nnz > 0 && (!in->col_idx || !in->val)) return fail(HPR_ERR_INVALID, "col_idx and val are required");
    const size_t m = (size_t)in->m, n = (size_t)in->n, nnz = (size_t)in->nnz;
    try {
        s.rp.resize(m + 1);
        s.ci.resize(nnz);
        s.v.resize(nnz);
        s.lo.resize(m);
        s.hi.resize(m);
        s.l.resize(n);
        s.u.resize(n);
        s.c.resize(n);
        auto get = [&](void* dst, const void* src, size_t bytes) {
            if (bytes) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        };
        if (m > 0) {
            get(s.rp.data(), in->row_ptr, sizeof(int64_t) * (m + 1));
            get(s.lo.data(), in->row_lo, sizeof(double) * m);
            get(s.hi.data(), in->row_hi, sizeof(double) * m);
        } else {
            s.rp.assign(1, 0);
        }
        get(s.ci.data(), in->col_idx, sizeof(int32_t) * nnz);
        get(s.v.data(), in->val, sizeof(double) * nnz);
        get(s.l.data(), in->col_lo, sizeof(double) * n);
        get(s.u.data(), in->col_hi, sizeof(double) * n);
        get(s.c.data(), in->c, sizeof(double) * n);
        HIP_OK(hipStreamSynchronize(st));
    } catch (const HipError& err) {
        return err.code;
    } catch (const std::bad_alloc&) {
        return fail(HPR_ERR_NOMEM, "host allocation failed");
    }
    s.lp = hpr_lp{in->m, in->n, in->nnz, s.rp.data(), s.ci.data(), s.v.data(), s.lo.data(), s.hi.data(),
                  s.l.data(), s.u.data(), s.c.data(), in->obj_offset, 0};
    return HPR_OK;
}

static int engine_create_host(const hpr_lp* lps, int count, const hpr_opts* opts_in, Engine** out);

static int engine_create(const hpr_lp* lps, int count, const hpr_opts* opts_in, Engine** out) {
    g_err.clear();
    if (!out) return fail(HPR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > kMaxBatch) return fail(HPR_ERR_INVALID, "count must be in [1, %d]", kMaxBatch);
    if (!lps) return fail(HPR_ERR_INVALID, "lp is NULL");
    bool any_dev = false;
    for (int l = 0; l < count; ++l) any_dev = any_dev || lps[l].on_device != 0;
    if (!any_dev) return engine_create_host(lps, count, opts_in, out);
    std::vector<StagedLp> staged((size_t)count);
    std::vector<hpr_lp> host((size_t)count);
    hipStream_t st = opts_in ? (hipStream_t)opts_in->stream : nullptr;
    for (int l = 0; l < count; ++l) {
        if (lps[l].on_device != 0 && lps[l].on_device != 1) return fail(HPR_ERR_INVALID, "on_device must be 0 or 1");
        if (!lps[l].on_device) {
            host[l] = lps[l];
            continue;
        }
        const int rc = stage_device_lp(&lps[l], st, staged[l]);
        if (rc) return rc;
        host[l] = staged[l].lp;
    }
    return engine_create_host(host.data(), count, opts_in, out);
}

static int engine_create_host(const hpr_lp* lps, int count, const hpr_opts* opts_in, Engine** out) {
    g_err.clear();
    if (!out) return fail(HPR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > kMaxBatch) return fail(HPR_ERR_INVALID, "count must be in [1, %d]", kMaxBatch);
    if (!lps) return fail(HPR_ERR_INVALID, "lp is NULL");
    hpr_opts o;
    if (opts_in) o = *opts_in;
    else hpr_default_opts(&o);
    int rc = validate_opts(&o);
    if (rc) return rc;
    bool sorted = true;
    for (int l = 0; l < count; ++l) {
        rc = validate(&lps[l], &sorted);
        if (rc) {
            if (count > 1) {
                std::string msg = g_err;
                return fail(rc, "LP %d: %s", l, msg.c_str());
            }
            return rc;
        }
    }
    const double t0 = now_s();
    std::unique_ptr<Engine> e;
    try {
        e.reset(new Engine());
        e->L = count;
        e->opts = o;
        e->fp32 = o.precision == HPR_FP32;
        e->lps.resize(count);
        HIP_OK(hipGetDevice(&e->device));
        if (o.stream) {
            e->st = (hipStream_t)o.stream;
        } else {
            HIP_OK(hipStreamCreateWithFlags(&e->st, hipStreamNonBlocking));
            e->own_stream = true;
        }
        Layout PA, PAt;
        PA.start.assign(1, 0);
        PAt.start.assign(1, 0);
        std::vector<int64_t> rows_a(1, 0), rows_at(1, 0);
        const int threads = host_threads();
        const int chunk = count == 1 ? 1 : threads;
        // One LP whose rows are in column order is set up on the device: the caller's CSR is
        // uploaded once and scaled, transposed and laid out there (device_setup); batches and
        // rows out of order take the host path, which computes the same values.
        const bool on_gpu = count == 1 && sorted && lps[0].m > 0 && lps[0].nnz > 0 && lps[0].nnz < INT32_MAX;
        if (on_gpu) {
            const hpr_lp* lp = &lps[0];
            LpHost& h = e->lps[0];
            h.m = lp->m;
            h.n = lp->n;
            h.nnz = lp->nnz;
            DBuf drp, dci, dv, ddr, ddc;
            drp.alloc(sizeof(int64_t) * ((size_t)lp->m + 1));
            dci.alloc(sizeof(int32_t) * (size_t)lp->nnz);
            dv.alloc(sizeof(double) * (size_t)lp->nnz);
            ddr.alloc(sizeof(double) * (size_t)lp->m);
            ddc.alloc(sizeof(double) * (size_t)lp->n);
            HIP_OK(hipMemcpyAsync(drp.p, lp->row_ptr, drp.bytes, hipMemcpyHostToDevice, e->st));
            HIP_OK(hipMemcpyAsync(dci.p, lp->col_idx, dci.bytes, hipMemcpyHostToDevice, e->st));
            HIP_OK(hipMemcpyAsync(dv.p, lp->val, dv.bytes, hipMemcpyHostToDevice, e->st));
            DevSetupIn in;
            in.rp = drp.as<int64_t>();
            in.ci = dci.as<int32_t>();
            in.v = dv.as<double>();
            in.m = lp->m;
            in.n = lp->n;
            in.nnz = lp->nnz;
            in.dr = ddr.as<double>();
            in.dc = ddc.as<double>();
            h.dr.resize(lp->m);
            h.dc.resize(lp->n);
            in.dr_host = h.dr.data();
            in.dc_host = h.dc.data();
            in.ruiz_iters = (o.scaling & HPR_SCALE_RUIZ) ? o.ruiz_iters : 0;
            in.pc = (o.scaling & HPR_SCALE_PC) ? 1 : 0;
            in.fp32 = e->fp32 ? 1 : 0;
            in.tile = kWinBytes / (e->fp32 ? (int)sizeof(float) : (int)sizeof(double)) / 2;
            {
                DevSetupOut out;
                HIP_OK(device_setup(in, out, e->st));
                scale_vectors(lp, o, h);
                e->M = lp->m;
                e->N = lp->n;
                rows_a.push_back(e->M);
                rows_at.push_back(e->N);
                e->A.adopt(out.a, rows_a, lp->m, e->N, e->fp32, o.lds_windows, e->st);
                e->At.adopt(out.at, rows_at, lp->n, e->M, e->fp32, o.lds_windows, e->st);
            }
        }
        for (int c0 = 0; c0 < (on_gpu ? 0 : count); c0 += chunk) {
            const int c1 = std::min(count, c0 + chunk);
            std::vector<PrepLp> prep((size_t)(c1 - c0));
            if (count == 1) prep_lp(&lps[0], o, prep[0], threads);
            else parallel_for(c1 - c0, threads, [&](int i) { prep_lp(&lps[c0 + i], o, prep[i], 1); });
            for (int l = c0; l < c1; ++l) {
                const hpr_lp* lp = &lps[l];
                PrepLp& p = prep[l - c0];
                LpHost& h = e->lps[l];
                h = std::move(p.h);
                h.m = lp->m;
                h.n = lp->n;
                h.nnz = lp->nnz;
                h.row_off = e->M;
                h.col_off = e->N;
                if (count == 1) {         // one LP: the layouts are the pools
                    PA = std::move(p.la);
                    PAt = std::move(p.lt);
                } else {                  // append with global column indices
                    const Layout& la = p.la;
                    const Layout& lt = p.lt;
                    const int64_t base_a = PA.start.back(), base_t = PAt.start.back();
                    PA.start.reserve(PA.start.size() + lp->m);
                    PAt.start.reserve(PAt.start.size() + lp->n);
                    for (size_t i = 1; i < la.start.size(); ++i) PA.start.push_back(base_a + la.start[i]);
                    for (size_t i = 1; i < lt.start.size(); ++i) PAt.start.push_back(base_t + lt.start[i]);
                    const size_t ca = PA.col.size(), ct = PAt.col.size();
                    PA.col.resize(ca + la.col.size());
                    PAt.col.resize(ct + lt.col.size());
                    for (size_t k = 0; k < la.col.size(); ++k) PA.col[ca + k] = la.col[k] + (int32_t)h.col_off;
                    for (size_t k = 0; k < lt.col.size(); ++k) PAt.col[ct + k] = lt.col[k] + (int32_t)h.row_off;
                    PA.val.insert(PA.val.end(), la.val.begin(), la.val.end());
                    PAt.val.insert(PAt.val.end(), lt.val.begin(), lt.val.end());
                    p.la = Layout();
                    p.lt = Layout();
                }
                e->M += lp->m;
                e->N += lp->n;
                rows_a.push_back(e->M);
                rows_at.push_back(e->N);
                if (e->M > INT32_MAX || e->N > INT32_MAX) {
                    fail(HPR_ERR_INVALID, "pooled rows or columns exceed 2^31");
                    throw HipError{HPR_ERR_INVALID};
                }
            }
        }
        if (!on_gpu)
            parallel_for(2, threads, [&](int i) {
                const int th = std::max(1, threads / 2);
                if (i == 0) e->A.prepare(PA, rows_a, e->N, e->fp32, o.lds_windows, th);
                else e->At.prepare(PAt, rows_at, e->M, e->fp32, o.lds_windows, th);
            });
        const double t1 = now_s();
        if (!on_gpu) {
            e->A.upload_from(PA, e->fp32, e->st);
            e->At.upload_from(PAt, e->fp32, e->st);
        }
        e->sync();
        upload_vectors(e.get());
        alloc_iterates(e.get());
        const double t2 = now_s();
        if (e->fp32) autotune<float>(e.get());
        else autotune<double>(e.get());
        alloc_partials(e.get());
        const double t3 = now_s();
        if (o.lambda > 0) {
            for (LpHost& h : e->lps) h.lambda = o.lambda;
        } else {
            power_method(e.get());
        }
        e->sync();
        const double t4 = now_s();
        e->t_prep = t1 - t0;
        e->t_upload = t2 - t1;
        e->t_tune = t3 - t2;
        e->t_power = t4 - t3;
    } catch (const HipError& err) {
        return err.code;
    } catch (const std::bad_alloc&) {
        return fail(HPR_ERR_NOMEM, "host allocation failed");
    }
    e->setup_s = now_s() - t0;
    *out = e.release();
    return HPR_OK;
}

static int engine_set_bounds(Engine* e, int i, const double* col_lo, const double* col_hi) {
    if (i < 0 || i >= e->L) return fail(HPR_ERR_INVALID, "LP index %d out of range", i);
    LpHost& h = e->lps[i];
    const int32_t n = h.n;
    std::vector<double> lo(h.l_s), hi(h.u_s);
    for (int32_t j = 0; j < n; ++j) {
        const double a = col_lo ? col_lo[j] : h.l_s[j] * h.beta_b * h.dc[j];
        const double b = col_hi ? col_hi[j] : h.u_s[j] * h.beta_b * h.dc[j];
        if (std::isnan(a) || std::isnan(b) || a > b || a == INFINITY || b == -INFINITY)
            return fail(HPR_ERR_INVALID, "bad column bounds at %d", j);
        if (col_lo) lo[j] = a / (h.beta_b * h.dc[j]);
        if (col_hi) hi[j] = b / (h.beta_b * h.dc[j]);
    }
    try {
        h.l_s = lo;
        h.u_s = hi;
        double* l64 = e->l64.as<double>() + h.col_off;
        double* u64 = e->u64.as<double>() + h.col_off;
        HIP_OK(hipMemcpyAsync(l64, h.l_s.data(), sizeof(double) * n, hipMemcpyHostToDevice, e->st));
        HIP_OK(hipMemcpyAsync(u64, h.u_s.data(), sizeof(double) * n, hipMemcpyHostToDevice, e->st));
        if (e->fp32) {
            launch_cast<float>(l64, e->l32.as<float>() + h.col_off, n, e->st);
            launch_cast<float>(u64, e->u32.as<float>() + h.col_off, n, e->st);
        }
        e->sync();
    } catch (const HipError& err) {
        return err.code;
    }
    return HPR_OK;
}

static int engine_set_start(Engine* e, int i, const double* x0, const double* y0) {
    if (i < 0 || i >= e->L) return fail(HPR_ERR_INVALID, "LP index %d out of range", i);
    LpHost& h = e->lps[i];
    if (x0) {
        for (int32_t j = 0; j < h.n; ++j)
            if (!std::isfinite(x0[j])) return fail(HPR_ERR_INVALID, "non-finite x0 at %d", j);
        h.x_start.assign(x0, x0 + h.n);
    } else {
        h.x_start.clear();
    }
    if (y0) {
        for (int32_t r = 0; r < h.m; ++r)
            if (!std::isfinite(y0[r])) return fail(HPR_ERR_INVALID, "non-finite y0 at %d", r);
        h.y_start.assign(y0, y0 + h.m);
    } else {
        h.y_start.clear();
    }
    return HPR_OK;
}

// ---------------------------------------------------------------- solve

namespace {

// start point: projection of the scaled warm start (or of zero) onto the bounds and onto the
// sign pattern of the rows (y_i > 0 needs a finite lower side, y_i < 0 a finite upper side)
template <typename T>
void upload_start(Engine* e, bool use_start) {
    std::vector<T> xs(e->N), ys(std::max<int64_t>(e->M, 1));
    for (int l = 0; l < e->L; ++l) {
        const LpHost& h = e->lps[l];
        const bool warm = use_start && (e->use_start_mask.empty() || e->use_start_mask[l]);
        for (int32_t j = 0; j < h.n; ++j) {
            double v = (!warm || h.x_start.empty()) ? 0.0 : h.x_start[j] / (h.beta_b * h.dc[j]);
            v = v < h.l_s[j] ? h.l_s[j] : (v > h.u_s[j] ? h.u_s[j] : v);
            xs[h.col_off + j] = T(v);
        }
        for (int32_t r = 0; r < h.m; ++r) {
            double v = (!warm || h.y_start.empty()) ? 0.0 : h.y_start[r] / (h.beta_c * h.dr[r]);
            if (!std::isfinite(h.lo_s[r]) && v > 0) v = 0.0;
            if (!std::isfinite(h.hi_s[r]) && v < 0) v = 0.0;
            ys[h.row_off + r] = T(v);
        }
    }
    const size_t es = sizeof(T);
    HIP_OK(hipMemcpyAsync(e->x0.p, xs.data(), es * e->N, hipMemcpyHostToDevice, e->st));
    HIP_OK(hipMemcpyAsync(e->x.p, xs.data(), es * e->N, hipMemcpyHostToDevice, e->st));
    if (e->M > 0) {
        HIP_OK(hipMemcpyAsync(e->y0.p, ys.data(), es * e->M, hipMemcpyHostToDevice, e->st));
        HIP_OK(hipMemcpyAsync(e->y.p, ys.data(), es * e->M, hipMemcpyHostToDevice, e->st));
    }
    e->sync();
}

ControlArgs control_args(Engine* e, int phase, int nb) {
    ControlArgs a;
    a.ctrl = e->ctrl.as<Ctrl>();
    a.st = e->state.as<LpState>();
    a.sums = e->sums.as<double>();
    a.sums64 = e->sums64.as<double>();
    a.stat = e->stat.as<int32_t>();
    a.nlp = e->L;
    a.nb = nb;
    a.fp32 = e->fp32 ? 1 : 0;
    a.phase = phase;
    a.max_iter = e->opts.max_iter;
    a.tol = e->opts.tol;
    a.restart_rule = e->opts.restart;
    a.sigma_update = e->opts.sigma_update;
    a.sigma_smoothing = e->opts.sigma_smoothing;
    a.sigma_smoothing_warm = e->opts.sigma_smoothing_warm;
    a.stall_iters = e->opts.stall_iters;
    return a;
}

// Check kernels in precision (Tm, Tp, Tv) and the per-LP finish into `out`.
template <typename Tm, typename Tp, typename Tv>
void enqueue_check(Engine* e, double* out) {
    const DevCsr<Tm> A = e->A.view<Tm>(), At = e->At.view<Tm>();
    const DevProb<Tp> p = e->prob<Tp>();
    const DevIter<Tv> v = e->iter<Tv>();
    launch_check_rows<Tm, Tp, Tv>(A, p, v, e->ctrl.as<Ctrl>(), e->part_r.as<double>(), e->st);
    launch_check_cols<Tm, Tp, Tv>(At, p, v, e->ctrl.as<Ctrl>(), e->part_c.as<double>(), e->st);
    launch_finish_sums(e->part_r.as<double>(), kRowQ, A.nblocks, e->A.seg_ptr(), e->L, out, 0, e->st);
    launch_finish_sums(e->part_c.as<double>(), kColQ, At.nblocks, e->At.seg_ptr(), e->L, out, kColOff, e->st);
}

// One block of nb iterations, the storage-precision check, the control (phase 1) and the
// restarts. With `sample`, the first iteration's two kernels are timed by events stamped at
// their own start and end.
template <typename T>
void enqueue_block(Engine* e, int nb, bool sample) {
    const DevCsr<T> A = e->A.view<T>(), At = e->At.view<T>();
    const DevProb<T> p = e->prob<T>();
    const DevIter<T> v = e->iter<T>();
    for (int j = 0; j < nb; ++j) {
        const bool chk = (j == nb - 1);
        const bool timed = sample && j == 0;
        launch_primal_step<T>(At, p, v, e->ctrl.as<Ctrl>(), j, chk, e->st, timed ? e->ev[0] : nullptr,
                              timed ? e->ev[1] : nullptr);
        launch_dual_step<T>(A, p, v, e->ctrl.as<Ctrl>(), j, chk, e->st, timed ? e->ev[2] : nullptr,
                            timed ? e->ev[3] : nullptr);
    }
    enqueue_check<T, T, T>(e, e->sums.as<double>());
    launch_control(control_args(e, 1, nb), e->st);
    launch_restart<T>(A, At, v, e->ctrl.as<Ctrl>(), e->st);
}

template <typename T>
hipGraphExec_t capture_block(Engine* e, int nb) {
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(e->st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    bool ok = true;
    try {
        enqueue_block<T>(e, nb, false);
    } catch (const HipError&) {
        ok = false;
    }
    if (hipStreamEndCapture(e->st, &g) != hipSuccess || !ok || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return exec;
}

int32_t read_stat(Engine* e, int which) {
    HIP_OK(hipMemcpyAsync(e->stat_h, e->stat.p, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, e->st));
    e->sync();
    return e->stat_h[which];
}

// The solve: blocks of iterations (the first of one iteration, then check_every, the last
// cut at max_iter), each ending with a check of every running LP; the device takes every
// decision (control_kernel), the host only polls how many LPs are still running, confirms
// FP32-storage candidates in FP64 and applies the time limit.
// per-LP controls and state; `use_start`: the solve starts from the uploaded caller's points
// (the LPs that have one and are not masked out), which selects the warm sigma weight
void init_control(Engine* e, bool use_start) {
    const hpr_opts& o = e->opts;
    for (int l = 0; l < e->L; ++l) {
        const LpHost& h = e->lps[l];
        Ctrl& c = e->ctrl_h[l];
        c = Ctrl{};
        c.sigma = o.sigma0;
        c.lambda = h.lambda;
        c.s = 1.0 / (h.lambda * o.sigma0);
        c.beta_b = h.beta_b;
        c.beta_c = h.beta_c;
        c.k_base = 0;
        c.active = 1;
        c.restart = 0;
        LpState& S = e->state_h[l];
        S = LpState{};
        S.norm_b = h.norm_b;
        S.norm_c = h.norm_c;
        S.obj_offset = h.obj_offset;
        S.mark_kkt = INFINITY;
        S.mark_it = 0;
        const bool has_start = !h.x_start.empty() || !h.y_start.empty();
        S.warm = (use_start && has_start && (e->use_start_mask.empty() || e->use_start_mask[l])) ? 1 : 0;
    }
    HIP_OK(hipMemcpyAsync(e->state.p, e->state_h.data(), sizeof(LpState) * e->L, hipMemcpyHostToDevice, e->st));
    put_ctrl(e);
}

// rel_kkt of every LP at the first check (one iteration) from the uploaded start points
template <typename T>
std::vector<double> probe_first_check(Engine* e, bool use_start) {
    upload_start<T>(e, use_start);
    init_control(e, use_start);
    if (e->g_first) HIP_OK(hipGraphLaunch(e->g_first, e->st));
    else enqueue_block<T>(e, 1, false);
    HIP_OK(hipMemcpyAsync(e->state_h.data(), e->state.p, sizeof(LpState) * e->L, hipMemcpyDeviceToHost, e->st));
    e->sync();
    std::vector<double> r(e->L);
    for (int l = 0; l < e->L; ++l) r[l] = e->state_h[l].rel_kkt;
    return r;
}

// (Re)capture the graphs of a first block (one iteration) and of a full block for the
// schedules the matrices use now.
template <typename T>
void build_graphs(Engine* e) {
    e->drop_graphs();
    e->g_first = capture_block<T>(e, 1);
    e->g_block = capture_block<T>(e, e->opts.check_every);
    e->graphs_built = true;
}

// Batches: when the running LPs have halved since the last change, later blocks launch only
// their thread blocks (the finished LPs' blocks would return at once, but a launch over all of
// them costs dispatch time for every iteration the slowest LP still needs).
template <typename T>
void compact_schedules(Engine* e) {
    HIP_OK(hipMemcpyAsync(e->ctrl_h.data(), e->ctrl.p, sizeof(Ctrl) * e->L, hipMemcpyDeviceToHost, e->st));
    e->sync();
    std::vector<int32_t> running(e->L);
    for (int l = 0; l < e->L; ++l) running[l] = e->ctrl_h[l].active;
    e->A.compact(running, e->st);
    e->At.compact(running, e->st);
    if (e->opts.use_graph) build_graphs<T>(e);
}

// Counters of the block loop of a solve.
struct LoopState {
    int64_t it = 0, blocks = 0;
    int32_t launched = 0;       // LPs whose blocks the current schedules launch
    int32_t seen_running = 0;
};

// Back to the full schedules after a run that compacted them (the graphs captured for the
// compacted schedules are dropped; the next run captures new ones).
void full_schedules(Engine* e) {
    if (e->A.use_act || e->At.use_act) {
        e->A.full();
        e->At.full();
        e->drop_graphs();
    }
}

// Blocks of iterations from the state in `ls` until every LP has stopped, max_iter, or
// `max_blocks` blocks in this call; returns the number of LPs still running.
template <typename T>
int32_t run_blocks(Engine* e, double t0, LoopState& ls, int64_t max_blocks) {
    const hpr_opts& o = e->opts;
    int32_t running = 0;
    for (int64_t nbl = 0; nbl < max_blocks; ++nbl) {
        const int64_t it = ls.it;
        const int nb = (int)((it == 0) ? 1 : std::min<int64_t>(o.check_every, o.max_iter - it));
        const bool sample = o.profile && nb >= 2 && (ls.blocks % 4 == 1);
        hipGraphExec_t g = (nb == 1 && it == 0) ? e->g_first : (nb == o.check_every ? e->g_block : nullptr);
        if (g && !sample) HIP_OK(hipGraphLaunch(g, e->st));
        else enqueue_block<T>(e, nb, sample);
        HIP_OK(hipGetLastError());
        ls.it += nb;
        ls.blocks += 1;
        running = read_stat(e, 0);
        if (sample) {
            float a = 0.f, b = 0.f;
            HIP_OK(hipEventElapsedTime(&a, e->ev[0], e->ev[1]));
            HIP_OK(hipEventElapsedTime(&b, e->ev[2], e->ev[3]));
            e->kstats.primal_ms += a;
            e->kstats.dual_ms += b;
            e->kstats.samples += 1;
        }
        if (e->fp32 && e->stat_h[1] > 0) {
            enqueue_check<double, double, float>(e, e->sums64.as<double>());
            launch_control(control_args(e, 2, 0), e->st);
            launch_restart<T>(e->A.view<T>(), e->At.view<T>(), e->iter<T>(), e->ctrl.as<Ctrl>(), e->st);
            running = read_stat(e, 0);
        }
        if (running > 0 && o.time_limit_s > 0 && now_s() - t0 > o.time_limit_s) {
            launch_control(control_args(e, 4, 0), e->st);
            running = read_stat(e, 0);
        }
        if (e->L > 1 && running < ls.seen_running) {   // per-LP time to its stop, at check granularity
            HIP_OK(hipMemcpyAsync(e->ctrl_h.data(), e->ctrl.p, sizeof(Ctrl) * e->L, hipMemcpyDeviceToHost, e->st));
            e->sync();
            const double t = now_s() - t0;
            for (int l = 0; l < e->L; ++l)
                if (!e->ctrl_h[l].active && e->done_at[l] < 0) e->done_at[l] = t;
            ls.seen_running = running;
        }
        if (running == 0 || ls.it >= o.max_iter) break;
        if (e->L > 1 && 2 * running <= ls.launched) {
            compact_schedules<T>(e);
            ls.launched = running;
        }
    }
    return running;
}

// From the start points selected by use_start_mask (or zero): iterates, controls and loop
// counters of a fresh solve.
template <typename T>
LoopState start_run(Engine* e) {
    full_schedules(e);
    if (e->opts.use_graph && !e->graphs_built) build_graphs<T>(e);
    upload_start<T>(e, true);
    init_control(e, true);
    e->done_at.assign(e->L, -1.0);
    LoopState ls;
    ls.launched = e->L;
    ls.seen_running = e->L;
    return ls;
}

template <typename T>
void solve_loop(Engine* e, double t0) {
    const hpr_opts& o = e->opts;
    if (o.use_graph && !e->graphs_built) build_graphs<T>(e);
    if (o.warm_fallback < 0 || o.warm_fallback > 2) {
        fail(HPR_ERR_INVALID, "warm_fallback must be 0, 1 or 2");
        throw HipError{HPR_ERR_INVALID};
    }
    if (o.profile && !e->ev[0])
        for (hipEvent_t& ev : e->ev) HIP_OK(hipEventCreate(&ev));
    e->warm_used.assign(e->L, 0);
    bool any_start = false;
    for (const LpHost& h : e->lps) any_start = any_start || !h.x_start.empty() || !h.y_start.empty();
    for (int l = 0; l < e->L; ++l) e->warm_used[l] = !e->lps[l].x_start.empty() || !e->lps[l].y_start.empty();
    e->use_start_mask.clear();
    bool resumed = false;
    LoopState ls;
    if (any_start && o.warm_fallback == 1) {
        // Guard: an LP starts from zero when its first check (one iteration) from the caller's
        // point is not finite or above warm_fallback_ratio times the first check from zero.
        const std::vector<double> cold = probe_first_check<T>(e, false);
        const std::vector<double> warm = probe_first_check<T>(e, true);
        for (int l = 0; l < e->L; ++l)
            if (e->warm_used[l] && !(std::isfinite(warm[l]) && warm[l] <= o.warm_fallback_ratio * cold[l]))
                e->warm_used[l] = 0;
    } else if (any_start && o.warm_fallback == 2) {
        // Race to the second check (1 + check_every iterations): both starts run that far and
        // an LP keeps the caller's point when it stopped there as solved, or when its rel_kkt is
        // finite and no higher than the zero start's (which did not stop as solved). When every
        // LP with a point keeps it, the warm run simply continues; otherwise all LPs start again
        // from the chosen points.
        std::vector<int32_t> has = e->warm_used;
        e->use_start_mask.assign(e->L, 0);
        LoopState lc = start_run<T>(e);
        run_blocks<T>(e, t0, lc, 2);
        HIP_OK(hipMemcpyAsync(e->state_h.data(), e->state.p, sizeof(LpState) * e->L, hipMemcpyDeviceToHost, e->st));
        e->sync();
        const std::vector<LpState> cold = e->state_h;
        e->use_start_mask = has;
        LoopState lw = start_run<T>(e);
        run_blocks<T>(e, t0, lw, 2);
        HIP_OK(hipMemcpyAsync(e->state_h.data(), e->state.p, sizeof(LpState) * e->L, hipMemcpyDeviceToHost, e->st));
        e->sync();
        bool all_warm = true;
        for (int l = 0; l < e->L; ++l) {
            if (!has[l]) continue;
            const LpState& w = e->state_h[l];
            const LpState& c = cold[l];
            const bool keep = w.term == HPR_SOLVED ||
                              (c.term != HPR_SOLVED && std::isfinite(w.rel_kkt) && w.rel_kkt <= c.rel_kkt);
            e->warm_used[l] = keep ? 1 : 0;
            all_warm = all_warm && keep;
        }
        if (all_warm) {
            resumed = true;
            ls = lw;
        }
    }
    e->kstats = hpr_kernel_stats{};
    if (!resumed) {
        e->use_start_mask = e->warm_used;
        ls = start_run<T>(e);
    }
    run_blocks<T>(e, t0, ls, INT64_MAX);
    full_schedules(e);                     // the report and the solution cover every LP
    if (e->fp32) {
        // report the residuals of the returned points in FP64
        enqueue_check<double, double, float>(e, e->sums64.as<double>());
        launch_control(control_args(e, 3, 0), e->st);
    }
    HIP_OK(hipMemcpyAsync(e->state_h.data(), e->state.p, sizeof(LpState) * e->L, hipMemcpyDeviceToHost, e->st));
    HIP_OK(hipMemcpyAsync(e->ctrl_h.data(), e->ctrl.p, sizeof(Ctrl) * e->L, hipMemcpyDeviceToHost, e->st));
    e->sync();
}

}  // namespace

static int engine_solve(Engine* e, hpr_info* infos) {
    const double t0 = now_s();
    try {
        int dev = 0;
        HIP_OK(hipGetDevice(&dev));
        if (dev != e->device) HIP_OK(hipSetDevice(e->device));
        if (e->fp32) solve_loop<float>(e, t0);
        else solve_loop<double>(e, t0);
        if (dev != e->device) HIP_OK(hipSetDevice(dev));
    } catch (const HipError& err) {
        return err.code;
    } catch (const std::bad_alloc&) {
        return fail(HPR_ERR_NOMEM, "host allocation failed");
    }
    e->solve_s = now_s() - t0;
    e->solved_once = true;
    for (int l = 0; l < e->L; ++l) {
        const LpState& S = e->state_h[l];
        hpr_info& info = infos[l];
        std::memset(&info, 0, sizeof(info));
        info.term = S.term ? S.term : HPR_ITER_LIMIT;
        info.iters = S.it;
        info.restarts = S.restarts;
        info.pobj = S.pobj;
        info.dobj = S.dobj;
        info.rel_p = S.rel_p;
        info.rel_d = S.rel_d;
        info.rel_gap = S.rel_gap;
        info.rel_kkt = S.rel_kkt;
        info.lambda = e->lps[l].lambda;
        info.sigma = e->ctrl_h[l].sigma;
        info.setup_s = e->setup_s;
        info.solve_s = (e->L > 1 && e->done_at[l] >= 0) ? e->done_at[l] : e->solve_s;
        info.warm_start = e->warm_used.empty() ? 0 : e->warm_used[l];
    }
    return HPR_OK;
}

static int engine_get_solution(Engine* e, int i, double* x, double* y, double* z) {
    if (i < 0 || i >= e->L) return fail(HPR_ERR_INVALID, "LP index %d out of range", i);
    if (!e->solved_once) return fail(HPR_ERR_STATE, "no solve has run on this handle");
    const LpHost& h = e->lps[i];
    try {
        if (e->fp32)
            launch_unscale<float>(e->A.view<float>(), e->At.view<float>(), e->iter<float>(), e->dr_d.as<double>(),
                                  e->dc_d.as<double>(), e->ctrl.as<Ctrl>(), e->ux.as<double>(), e->uy.as<double>(),
                                  e->uz.as<double>(), e->st);
        else
            launch_unscale<double>(e->A.view<double>(), e->At.view<double>(), e->iter<double>(),
                                   e->dr_d.as<double>(), e->dc_d.as<double>(), e->ctrl.as<Ctrl>(),
                                   e->ux.as<double>(), e->uy.as<double>(), e->uz.as<double>(), e->st);
        if (x) HIP_OK(hipMemcpyAsync(x, e->ux.as<double>() + h.col_off, sizeof(double) * h.n, hipMemcpyDeviceToHost,
                                     e->st));
        if (y && h.m)
            HIP_OK(hipMemcpyAsync(y, e->uy.as<double>() + h.row_off, sizeof(double) * h.m, hipMemcpyDeviceToHost,
                                  e->st));
        if (z) HIP_OK(hipMemcpyAsync(z, e->uz.as<double>() + h.col_off, sizeof(double) * h.n, hipMemcpyDeviceToHost,
                                     e->st));
        e->sync();
    } catch (const HipError& err) {
        return err.code;
    }
    return HPR_OK;
}

// Round and Algorithm 1 on the device over x (host, original space) or, when x is NULL, over
// the bar point of the last solve of LP i, unscaled on the device.
static int engine_fix_binaries(Engine* e, int i, const double* x, int32_t G, int32_t T, const int32_t* cols,
                               const double* fixval, double tau, int8_t* fixed, int8_t* rounded) {
    if (i < 0 || i >= e->L) return fail(HPR_ERR_INVALID, "LP index %d out of range", i);
    if (G < 1 || T < 1 || (int64_t)G * T > (int64_t)1 << 28) return fail(HPR_ERR_INVALID, "bad G or T");
    if (!cols || !fixed || !rounded) return fail(HPR_ERR_INVALID, "cols, fixed and rounded are required");
    if (!(tau >= 0.0 && tau < 0.5)) return fail(HPR_ERR_INVALID, "tau must be in [0, 0.5)");
    const LpHost& h = e->lps[i];
    const int64_t ne = (int64_t)G * T * 3;
    for (int64_t k = 0; k < ne; ++k) {
        if (cols[k] >= h.n) return fail(HPR_ERR_INVALID, "column %d out of range at entry %lld", cols[k], (long long)k);
        if (cols[k] < 0 && (!fixval || !std::isfinite(fixval[k])))
            return fail(HPR_ERR_INVALID, "entry %lld names no column and has no finite fixed value", (long long)k);
    }
    if (!x && !e->solved_once) return fail(HPR_ERR_STATE, "no solve has run on this handle");
    if (x)
        for (int32_t j = 0; j < h.n; ++j)
            if (!std::isfinite(x[j])) return fail(HPR_ERR_INVALID, "non-finite x at %d", j);
    try {
        DBuf dcols, dfix, dx, dout;
        // host copies live until the stream is synchronised below
        const std::vector<int32_t> hcols(cols, cols + ne);
        const std::vector<double> hfix = fixval ? std::vector<double>(fixval, fixval + ne) : std::vector<double>();
        const std::vector<double> hx = x ? std::vector<double>(x, x + h.n) : std::vector<double>();
        upload(dcols, hcols, e->st);
        if (fixval) upload(dfix, hfix, e->st);
        const double* xs = nullptr;
        if (x) {
            upload(dx, hx, e->st);
            xs = dx.as<double>();
        } else {
            if (e->fp32)
                launch_unscale<float>(e->A.view<float>(), e->At.view<float>(), e->iter<float>(), e->dr_d.as<double>(),
                                      e->dc_d.as<double>(), e->ctrl.as<Ctrl>(), e->ux.as<double>(),
                                      e->uy.as<double>(), e->uz.as<double>(), e->st);
            else
                launch_unscale<double>(e->A.view<double>(), e->At.view<double>(), e->iter<double>(),
                                       e->dr_d.as<double>(), e->dc_d.as<double>(), e->ctrl.as<Ctrl>(),
                                       e->ux.as<double>(), e->uy.as<double>(), e->uz.as<double>(), e->st);
            xs = e->ux.as<double>() + h.col_off;
        }
        dout.alloc((size_t)ne + (size_t)G * T);
        int8_t* d_round = dout.as<int8_t>();
        int8_t* d_fixed = d_round + ne;
        launch_fix_strategy(xs, dcols.as<int32_t>(), fixval ? dfix.as<double>() : nullptr, G, T, tau, d_fixed,
                            d_round, e->st);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(rounded, d_round, (size_t)ne, hipMemcpyDeviceToHost, e->st));
        HIP_OK(hipMemcpyAsync(fixed, d_fixed, (size_t)G * T, hipMemcpyDeviceToHost, e->st));
        e->sync();
    } catch (const HipError& err) {
        return err.code;
    } catch (const std::bad_alloc&) {
        return fail(HPR_ERR_NOMEM, "host allocation failed");
    }
    return HPR_OK;
}

static void engine_kernel_stats(Engine* e, hpr_kernel_stats* out) {
    *out = e->kstats;
    out->unroll_a = e->A.unroll;
    out->unroll_at = e->At.unroll;
    out->nontemporal_a = e->A.nontemporal;
    out->nontemporal_at = e->At.nontemporal;
    out->setup_prep_s = e->t_prep;
    out->setup_upload_s = e->t_upload;
    out->setup_tune_s = e->t_tune;
    out->setup_power_s = e->t_power;
    e->A.window_counts(out->full_blocks_a, out->split_blocks_a, out->sliced_blocks_a, out->blocks_a,
                       out->round_blocks_a);
    e->At.window_counts(out->full_blocks_at, out->split_blocks_at, out->sliced_blocks_at, out->blocks_at,
                        out->round_blocks_at);
    out->win_mode_a = e->A.win_mode;
    out->win_mode_at = e->At.win_mode;
    out->narrow_quads_a = e->A.narrow_quads;
    out->packed_quads_a = e->A.packed_quads;
    out->narrow_quads_at = e->At.narrow_quads;
    out->packed_quads_at = e->At.packed_quads;
    out->packed_a = e->A.use_pack ? 1 : 0;
    out->packed_at = e->At.use_pack ? 1 : 0;
    if (out->samples > 0) {
        out->primal_ms /= (double)out->samples;
        out->dual_ms /= (double)out->samples;
    }
}

// ---------------------------------------------------------------- C interface

struct hpr_handle {
    Engine* e;
};
struct hpr_batch {
    Engine* e;
};

extern "C" int hpr_create(const hpr_lp* lp, const hpr_opts* opts, hpr_handle** out) {
    if (!out) return fail(HPR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Engine* e = nullptr;
    const int rc = engine_create(lp, 1, opts, &e);
    if (rc) return rc;
    *out = new hpr_handle{e};
    return HPR_OK;
}

extern "C" int hpr_destroy(hpr_handle* h) {
    if (h) {
        delete h->e;
        delete h;
    }
    return HPR_OK;
}

extern "C" int hpr_set_bounds(hpr_handle* h, const double* col_lo, const double* col_hi) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    return engine_set_bounds(h->e, 0, col_lo, col_hi);
}

extern "C" int hpr_set_start(hpr_handle* h, const double* x0, const double* y0) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    return engine_set_start(h->e, 0, x0, y0);
}

extern "C" int hpr_solve(hpr_handle* h, hpr_info* info) {
    g_err.clear();
    if (!h || !info) return fail(HPR_ERR_INVALID, "handle or info is NULL");
    return engine_solve(h->e, info);
}

extern "C" int hpr_get_solution(hpr_handle* h, double* x, double* y, double* z) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    return engine_get_solution(h->e, 0, x, y, z);
}

extern "C" int hpr_fix_binaries(hpr_handle* h, const double* x, int32_t G, int32_t T, const int32_t* cols,
                                const double* fixval, double tau, int8_t* fixed, int8_t* rounded) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    return engine_fix_binaries(h->e, 0, x, G, T, cols, fixval, tau, fixed, rounded);
}

extern "C" int hpr_get_kernel_stats(hpr_handle* h, hpr_kernel_stats* out) {
    g_err.clear();
    if (!h || !out) return fail(HPR_ERR_INVALID, "handle or out is NULL");
    engine_kernel_stats(h->e, out);
    return HPR_OK;
}

extern "C" int hpr_batch_create(const hpr_lp* lps, int32_t count, const hpr_opts* opts, hpr_batch** out) {
    if (!out) return fail(HPR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Engine* e = nullptr;
    const int rc = engine_create(lps, count, opts, &e);
    if (rc) return rc;
    *out = new hpr_batch{e};
    return HPR_OK;
}

extern "C" int hpr_batch_destroy(hpr_batch* b) {
    if (b) {
        delete b->e;
        delete b;
    }
    return HPR_OK;
}

extern "C" int hpr_batch_size(hpr_batch* b, int32_t* count) {
    g_err.clear();
    if (!b || !count) return fail(HPR_ERR_INVALID, "batch or count is NULL");
    *count = b->e->L;
    return HPR_OK;
}

extern "C" int hpr_batch_set_bounds(hpr_batch* b, int32_t i, const double* col_lo, const double* col_hi) {
    g_err.clear();
    if (!b) return fail(HPR_ERR_INVALID, "batch is NULL");
    return engine_set_bounds(b->e, i, col_lo, col_hi);
}

extern "C" int hpr_batch_set_start(hpr_batch* b, int32_t i, const double* x0, const double* y0) {
    g_err.clear();
    if (!b) return fail(HPR_ERR_INVALID, "batch is NULL");
    return engine_set_start(b->e, i, x0, y0);
}

extern "C" int hpr_batch_solve(hpr_batch* b, hpr_info* infos) {
    g_err.clear();
    if (!b || !infos) return fail(HPR_ERR_INVALID, "batch or infos is NULL");
    return engine_solve(b->e, infos);
}

extern "C" int hpr_batch_get_solution(hpr_batch* b, int32_t i, double* x, double* y, double* z) {
    g_err.clear();
    if (!b) return fail(HPR_ERR_INVALID, "batch is NULL");
    return engine_get_solution(b->e, i, x, y, z);
}

extern "C" int hpr_batch_get_kernel_stats(hpr_batch* b, hpr_kernel_stats* out) {
    g_err.clear();
    if (!b || !out) return fail(HPR_ERR_INVALID, "batch or out is NULL");
    engine_kernel_stats(b->e, out);
    return HPR_OK;
}
