// Host runtime of the gfx950 LP solver: the C interface declared in hprlp.h.
//
// hpr_create validates the LP, scales it (Section III-A: optional Ruiz passes,
// Pock-Chambolle with alpha = 1, bound/cost normalisation), builds the padded and
// binned CSR layouts of A~ and A~^T, uploads them and estimates lambda = lambda_max(A~A~^T)
// with the power method on the device. hpr_solve runs blocks of iterations of eq.(hpr)
// on the device; the last iteration of each block writes the bar point, two check
// kernels reduce the KKT residuals (Theorem 1's residual map, normalised) and the merit
// in FP64, and the host decides termination, restarts and sigma from those sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

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

template <typename T>
static void upload(DBuf& d, const std::vector<T>& h, hipStream_t st) {
    d.alloc(h.size() * sizeof(T));
    if (!h.empty()) HIP_OK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// ---------------------------------------------------------------- host-side CSR helpers

struct HostCsr {
    int32_t rows = 0, cols = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<double> val;
};

// stable counting-sort transpose: entries of a column keep increasing row order
static HostCsr transpose(const HostCsr& a) {
    HostCsr t;
    t.rows = a.cols;
    t.cols = a.rows;
    const int64_t nnz = a.ptr[a.rows];
    t.ptr.assign((size_t)a.cols + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) t.ptr[(size_t)a.idx[k] + 1]++;
    for (int32_t j = 0; j < a.cols; ++j) t.ptr[j + 1] += t.ptr[j];
    std::vector<int64_t> fill(t.ptr.begin(), t.ptr.end() - 1);
    t.idx.resize(nnz);
    t.val.resize(nnz);
    for (int32_t i = 0; i < a.rows; ++i)
        for (int64_t k = a.ptr[i]; k < a.ptr[i + 1]; ++k) {
            const int64_t d = fill[a.idx[k]]++;
            t.idx[d] = i;
            t.val[d] = a.val[k];
        }
    return t;
}

// Padded layout of one matrix (structure on the host, ready for upload).
struct Layout {
    std::vector<int64_t> start;
    std::vector<int32_t> col;
    std::vector<double> val;
};

static Layout make_layout(const HostCsr& a) {
    Layout L;
    const int32_t R = a.rows;
    L.start.resize((size_t)R + 1);
    int64_t off = 0;
    for (int32_t i = 0; i < R; ++i) {
        L.start[i] = off;
        const int64_t len = a.ptr[i + 1] - a.ptr[i];
        off += (len + kVec - 1) / kVec * kVec;
    }
    L.start[R] = off;
    L.col.resize(off);
    L.val.resize(off);
    for (int32_t i = 0; i < R; ++i) {
        int64_t d = L.start[i];
        const int64_t b = a.ptr[i], e = a.ptr[i + 1];
        for (int64_t k = b; k < e; ++k, ++d) {
            L.col[d] = a.idx[k];
            L.val[d] = a.val[k];
        }
        for (; d < L.start[i + 1]; ++d) {   // padding: value 0 at a column the row uses
            L.col[d] = a.idx[e - 1];
            L.val[d] = 0.0;
        }
    }
    return L;
}

// Lane-group bins for U quads per lane and pass: bin b takes rows of at most U * 2^b quads.
static void make_bins(const std::vector<int64_t>& start, int U, std::vector<int32_t>& rows, Bins& bins) {
    const int32_t R = (int32_t)start.size() - 1;
    std::vector<uint8_t> bin((size_t)R);
    int32_t count[kNumBins] = {0};
    for (int32_t i = 0; i < R; ++i) {
        const int64_t quads = (start[i + 1] - start[i]) / kVec;
        int b = 0;
        while (b < kNumBins - 1 && (int64_t)U * (int64_t(1) << b) < quads) ++b;
        bin[i] = (uint8_t)b;
        count[b]++;
    }
    int32_t roff = 0, boff = 0;
    for (int b = 0; b < kNumBins; ++b) {
        bins.row_off[b] = roff;
        bins.nrows[b] = count[b];
        bins.block_off[b] = boff;
        const int per_block = kBlock >> b;
        boff += (count[b] + per_block - 1) / per_block;
        roff += count[b];
    }
    bins.block_off[kNumBins] = boff;
    rows.resize((size_t)R);
    int32_t pos[kNumBins];
    for (int b = 0; b < kNumBins; ++b) pos[b] = bins.row_off[b];
    for (int32_t i = 0; i < R; ++i) rows[pos[bin[i]]++] = i;
}

// Device copy of a layout: shared structure plus FP64 and (optionally) FP32 values.
struct DevMatrix {
    DBuf start, col, rows, val64, val32;
    std::vector<int64_t> start_h;   // host copy of the offsets (rebinning)
    Bins bins{};
    int32_t nrows = 0;
    int32_t unroll = 4;
    int64_t padded = 0;
    void upload_from(const Layout& L, bool fp32, hipStream_t st) {
        nrows = (int32_t)L.start.size() - 1;
        padded = (int64_t)L.col.size();
        start_h = L.start;
        upload(start, L.start, st);
        upload(col, L.col, st);
        upload(val64, L.val, st);
        if (fp32) {
            val32.alloc(L.val.size() * sizeof(float));
            launch_cast<float>(val64.as<double>(), val32.as<float>(), (int64_t)L.val.size(), st);
        }
        rows.alloc(sizeof(int32_t) * std::max(nrows, 1));
        set_unroll(4, st);
    }
    // rebuild the bins for U quads per lane and upload the row list
    void set_unroll(int U, hipStream_t st) {
        std::vector<int32_t> r;
        make_bins(start_h, U, r, bins);
        unroll = U;
        if (!r.empty()) {
            HIP_OK(hipMemcpyAsync(rows.p, r.data(), sizeof(int32_t) * r.size(), hipMemcpyHostToDevice, st));
            HIP_OK(hipStreamSynchronize(st));
        }
    }
    template <typename T>
    DevCsr<T> view() const {
        DevCsr<T> d;
        d.start = start.as<int64_t>();
        d.col = col.as<int32_t>();
        d.val = std::is_same<T, float>::value ? (const T*)val32.p : (const T*)val64.p;
        d.rows = rows.as<int32_t>();
        d.bins = bins;
        d.nrows = nrows;
        d.unroll = unroll;
        return d;
    }
};

// ---------------------------------------------------------------- validation

static int validate(const hpr_lp* lp) {
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
    for (int32_t i = 0; i < lp->m; ++i)
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
            const int32_t j = lp->col_idx[k];
            if (j < 0 || j >= lp->n) return fail(HPR_ERR_INVALID, "column index %d out of range in row %d", j, i);
            if (mark[j] == i) return fail(HPR_ERR_INVALID, "column %d repeated in row %d", j, i);
            mark[j] = i;
            if (!std::isfinite(lp->val[k])) return fail(HPR_ERR_INVALID, "non-finite value in row %d", i);
        }
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
    if (o->unroll != 0 && o->unroll != 1 && o->unroll != 2 && o->unroll != 4 && o->unroll != 8)
        return fail(HPR_ERR_INVALID, "unroll must be 0, 1, 2, 4 or 8");
    return HPR_OK;
}

static double finite_side(double lo, double hi) {
    const bool fl = std::isfinite(lo), fh = std::isfinite(hi);
    if (fl && fh) return std::fabs(lo) > std::fabs(hi) ? lo : hi;
    if (fl) return lo;
    if (fh) return hi;
    return 0.0;
}

// ---------------------------------------------------------------- the handle

struct hpr_handle {
    int32_t m = 0, n = 0;
    hpr_opts opts{};
    bool fp32 = false;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0;

    double beta_b = 1, beta_c = 1, lambda = 1, norm_b = 0, norm_c = 0, obj_offset = 0;
    std::vector<double> dr, dc;                 // diagonal scaling
    std::vector<double> lo_s, hi_s, l_s, u_s;   // scaled bounds (host copies)
    std::vector<double> x_start, y_start;       // start point in the original space (empty = zero)

    DevMatrix A, At;
    DBuf c64, l64, u64, lo64, hi64, c32, l32, u32, lo32, hi32, dr_d, dc_d;
    DBuf x, x0, xh, xb, zb, dx, y, y0, yb, dy;
    DBuf part_r, part_c, sums, ctrl;
    DBuf ux, uy, uz;                            // unscaled FP64 output
    double* pinned = nullptr;                   // host-visible sums
    Ctrl* ctrl_h = nullptr;

    bool solved_once = false;
    double setup_s = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // profiling marks
    hpr_kernel_stats kstats{};

    ~hpr_handle() {
        if (st) (void)hipStreamSynchronize(st);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (pinned) (void)hipHostFree(pinned);
        if (ctrl_h) (void)hipHostFree(ctrl_h);
        if (own_stream && st) (void)hipStreamDestroy(st);
    }

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
    o->stream = nullptr;
}

extern "C" const char* hpr_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- setup

static void scale_host(const hpr_lp* lp, const hpr_opts& o, HostCsr& a, hpr_handle* h) {
    const int32_t m = lp->m, n = lp->n;
    h->dr.assign((size_t)m, 1.0);
    h->dc.assign((size_t)n, 1.0);
    std::vector<double> er((size_t)m), ec((size_t)n);
    auto apply = [&]() {
        for (int32_t i = 0; i < m; ++i)
            for (int64_t k = a.ptr[i]; k < a.ptr[i + 1]; ++k) a.val[k] *= er[i] * ec[a.idx[k]];
        for (int32_t i = 0; i < m; ++i) h->dr[i] *= er[i];
        for (int32_t j = 0; j < n; ++j) h->dc[j] *= ec[j];
    };
    if (o.scaling & HPR_SCALE_RUIZ) {
        for (int32_t it = 0; it < o.ruiz_iters; ++it) {
            std::fill(ec.begin(), ec.end(), 0.0);
            for (int32_t i = 0; i < m; ++i) {
                double r = 0.0;
                for (int64_t k = a.ptr[i]; k < a.ptr[i + 1]; ++k) {
                    const double v = std::fabs(a.val[k]);
                    r = std::max(r, v);
                    ec[a.idx[k]] = std::max(ec[a.idx[k]], v);
                }
                er[i] = r > 0 ? 1.0 / std::sqrt(r) : 1.0;
            }
            for (int32_t j = 0; j < n; ++j) ec[j] = ec[j] > 0 ? 1.0 / std::sqrt(ec[j]) : 1.0;
            apply();
        }
    }
    if (o.scaling & HPR_SCALE_PC) {
        std::fill(ec.begin(), ec.end(), 0.0);
        for (int32_t i = 0; i < m; ++i) {
            double r = 0.0;
            for (int64_t k = a.ptr[i]; k < a.ptr[i + 1]; ++k) {
                r += std::fabs(a.val[k]);
                ec[a.idx[k]] += std::fabs(a.val[k]);
            }
            er[i] = r > 0 ? 1.0 / std::sqrt(r) : 1.0;
        }
        for (int32_t j = 0; j < n; ++j) ec[j] = ec[j] > 0 ? 1.0 / std::sqrt(ec[j]) : 1.0;
        apply();
    }
    h->lo_s.resize(m);
    h->hi_s.resize(m);
    for (int32_t i = 0; i < m; ++i) {
        h->lo_s[i] = lp->row_lo[i] * h->dr[i];
        h->hi_s[i] = lp->row_hi[i] * h->dr[i];
    }
    h->l_s.resize(n);
    h->u_s.resize(n);
    std::vector<double> cs(n);
    for (int32_t j = 0; j < n; ++j) {
        h->l_s[j] = lp->col_lo[j] / h->dc[j];
        h->u_s[j] = lp->col_hi[j] / h->dc[j];
        cs[j] = lp->c[j] * h->dc[j];
    }
    h->beta_b = h->beta_c = 1.0;
    if (o.scaling & HPR_SCALE_BC) {
        double b2 = 0.0, c2 = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            const double b = finite_side(h->lo_s[i], h->hi_s[i]);
            b2 += b * b;
        }
        for (int32_t j = 0; j < n; ++j) c2 += cs[j] * cs[j];
        h->beta_b = 1.0 + std::sqrt(b2);
        h->beta_c = 1.0 + std::sqrt(c2);
        for (int32_t i = 0; i < m; ++i) {
            h->lo_s[i] /= h->beta_b;
            h->hi_s[i] /= h->beta_b;
        }
        for (int32_t j = 0; j < n; ++j) {
            h->l_s[j] /= h->beta_b;
            h->u_s[j] /= h->beta_b;
            cs[j] /= h->beta_c;
        }
    }
    // norms of the original rhs and cost for the relative residuals
    double b2 = 0.0, c2 = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        const double b = finite_side(lp->row_lo[i], lp->row_hi[i]);
        b2 += b * b;
    }
    for (int32_t j = 0; j < n; ++j) c2 += lp->c[j] * lp->c[j];
    h->norm_b = std::sqrt(b2);
    h->norm_c = std::sqrt(c2);

    hipStream_t st = h->st;
    upload(h->c64, cs, st);
    upload(h->l64, h->l_s, st);
    upload(h->u64, h->u_s, st);
    upload(h->lo64, h->lo_s, st);
    upload(h->hi64, h->hi_s, st);
    upload(h->dr_d, h->dr, st);
    upload(h->dc_d, h->dc, st);
    if (h->fp32) {
        h->c32.alloc(sizeof(float) * n);
        h->l32.alloc(sizeof(float) * n);
        h->u32.alloc(sizeof(float) * n);
        h->lo32.alloc(sizeof(float) * std::max(m, 1));
        h->hi32.alloc(sizeof(float) * std::max(m, 1));
        launch_cast<float>(h->c64.as<double>(), h->c32.as<float>(), n, st);
        launch_cast<float>(h->l64.as<double>(), h->l32.as<float>(), n, st);
        launch_cast<float>(h->u64.as<double>(), h->u32.as<float>(), n, st);
        launch_cast<float>(h->lo64.as<double>(), h->lo32.as<float>(), m, st);
        launch_cast<float>(h->hi64.as<double>(), h->hi32.as<float>(), m, st);
    }
    HIP_OK(hipStreamSynchronize(st));   // `cs` is a local host vector
}

static void sync(hpr_handle* h) { HIP_OK(hipStreamSynchronize(h->st)); }

// lambda_max(A~ A~^T) by the power method in FP64 on the device: v <- A~(A~^T v)/||.||,
// estimate ||A~ A~^T v|| for unit v; stop at relative change <= power_tol or after
// power_max_iter products; lambda = 1.01 * estimate, capped at 1 when the Pock-Chambolle
// scaling is on (it bounds ||A~|| by 1), and 1 when the estimate is 0.
static double power_method(hpr_handle* h) {
    const int32_t m = h->m, n = h->n;
    if (m == 0 || h->A.padded == 0) return 1.0;
    DBuf v, t, w, part;
    v.alloc(sizeof(double) * m);
    w.alloc(sizeof(double) * m);
    t.alloc(sizeof(double) * n);
    const int nb = sumsq_blocks(m);
    part.alloc(sizeof(double) * nb);
    DBuf tot;
    tot.alloc(sizeof(double));
    hipStream_t st = h->st;
    DevCsr<double> A = h->A.view<double>(), At = h->At.view<double>();
    auto norm = [&](const double* p) {
        launch_sumsq<double>(p, m, part.as<double>(), st);
        launch_finish_sums(part.as<double>(), 1, nb, tot.as<double>(), st);
        double s = 0;
        HIP_OK(hipMemcpyAsync(&s, tot.p, sizeof(double), hipMemcpyDeviceToHost, st));
        sync(h);
        return std::sqrt(s);
    };
    launch_start_vector<double>(v.as<double>(), m, h->opts.seed, st);
    const double nv = norm(v.as<double>());
    launch_scale<double>(v.as<double>(), m, 1.0 / nv, st);
    double est = 0.0, prev = 0.0;
    for (int it = 1; it <= h->opts.power_max_iter; ++it) {
        launch_spmv<double>(At, v.as<double>(), t.as<double>(), st);
        launch_spmv<double>(A, t.as<double>(), w.as<double>(), st);
        est = norm(w.as<double>());
        if (est == 0.0) break;
        launch_scale<double>(w.as<double>(), m, 1.0 / est, st);
        std::swap(v.p, w.p);
        if (it > 1 && std::fabs(est - prev) <= h->opts.power_tol * est) break;
        prev = est;
    }
    if (est == 0.0) return 1.0;
    double lam = 1.01 * est;
    if ((h->opts.scaling & HPR_SCALE_PC) && lam > 1.0) lam = 1.0;
    return lam;
}

static void alloc_iterates(hpr_handle* h) {
    const size_t es = h->fp32 ? sizeof(float) : sizeof(double);
    const size_t n = (size_t)h->n, m = (size_t)std::max(h->m, 1);
    for (DBuf* b : {&h->x, &h->x0, &h->xh, &h->xb, &h->zb, &h->dx}) b->alloc(es * n);
    for (DBuf* b : {&h->y, &h->y0, &h->yb, &h->dy}) b->alloc(es * m);
    h->sums.alloc(sizeof(double) * 2 * kMaxQ);
    h->ctrl.alloc(sizeof(Ctrl));
    h->ux.alloc(sizeof(double) * n);
    h->uy.alloc(sizeof(double) * m);
    h->uz.alloc(sizeof(double) * n);
    HIP_OK(hipHostMalloc((void**)&h->pinned, sizeof(double) * 2 * kMaxQ, hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void**)&h->ctrl_h, sizeof(Ctrl), hipHostMallocDefault));
}

// per-block partial sums of the check kernels (block counts depend on the bins)
static void alloc_partials(hpr_handle* h) {
    const int nbr = std::max(h->A.bins.block_off[kNumBins], 1);
    const int nbc = std::max(h->At.bins.block_off[kNumBins], 1);
    h->part_r.alloc(sizeof(double) * kRowQ * nbr);
    h->part_c.alloc(sizeof(double) * kColQ * nbc);
}

// Schedule tuner: for each matrix, time the fused step kernel that streams it (dual step
// for A~, primal step for A~^T) with U = 1, 2, 4, 8 quads per lane and pass (the bins
// follow U), and keep the fastest. A forced opts.unroll skips the timing.
template <typename T>
static void autotune(hpr_handle* h) {
    hipStream_t st = h->st;
    const size_t es = sizeof(T);
    for (DBuf* b : {&h->x, &h->x0, &h->xh, &h->xb, &h->zb, &h->dx, &h->y, &h->y0, &h->yb, &h->dy})
        HIP_OK(hipMemsetAsync(b->p, 0, b->bytes, st));
    (void)es;
    h->ctrl_h->sigma = 1.0;
    h->ctrl_h->s = 1.0;
    h->ctrl_h->lambda = 1.0;
    h->ctrl_h->k_base = 0;
    HIP_OK(hipMemcpyAsync(h->ctrl.p, h->ctrl_h, sizeof(Ctrl), hipMemcpyHostToDevice, st));
    const int forced = h->opts.unroll;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const DevProb<T> p = h->prob<T>();
    const DevIter<T> v = h->iter<T>();
    for (int which = 0; which < 2; ++which) {
        DevMatrix& M = which == 0 ? h->A : h->At;
        if (forced) {
            M.set_unroll(forced, st);
            continue;
        }
        if (M.nrows == 0) continue;
        int bestU = 4;
        float best = 1e30f;
        for (int U : {1, 2, 4, 8}) {
            M.set_unroll(U, st);
            const DevCsr<T> view = M.view<T>();
            auto launch = [&]() {
                if (which == 0) launch_dual_step<T>(view, p, v, h->ctrl.as<Ctrl>(), 0, false, st);
                else launch_primal_step<T>(view, p, v, h->ctrl.as<Ctrl>(), 0, false, st);
            };
            for (int r = 0; r < 2; ++r) launch();
            HIP_OK(hipEventRecord(e0, st));
            for (int r = 0; r < 8; ++r) launch();
            HIP_OK(hipEventRecord(e1, st));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bestU = U;
            }
        }
        M.set_unroll(bestU, st);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_OK(hipGetLastError());
}

extern "C" int hpr_create(const hpr_lp* lp, const hpr_opts* opts_in, hpr_handle** out) {
    g_err.clear();
    if (!out) return fail(HPR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    hpr_opts o;
    if (opts_in) o = *opts_in; else hpr_default_opts(&o);
    int rc = validate_opts(&o);
    if (rc) return rc;
    rc = validate(lp);
    if (rc) return rc;
    const double t0 = now_s();
    std::unique_ptr<hpr_handle> h;
    try {
        h.reset(new hpr_handle());
        h->m = lp->m;
        h->n = lp->n;
        h->opts = o;
        h->fp32 = o.precision == HPR_FP32;
        h->obj_offset = lp->obj_offset;
        HIP_OK(hipGetDevice(&h->device));
        if (o.stream) {
            h->st = (hipStream_t)o.stream;
        } else {
            HIP_OK(hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking));
            h->own_stream = true;
        }
        HostCsr a;
        a.rows = lp->m;
        a.cols = lp->n;
        if (lp->m > 0) a.ptr.assign(lp->row_ptr, lp->row_ptr + lp->m + 1);
        else a.ptr.assign(1, 0);
        a.idx.assign(lp->col_idx, lp->col_idx + lp->nnz);
        a.val.assign(lp->val, lp->val + lp->nnz);
        scale_host(lp, o, a, h.get());
        HostCsr at = transpose(a);
        {
            Layout la = make_layout(a);
            h->A.upload_from(la, h->fp32, h->st);
            Layout lt = make_layout(at);
            h->At.upload_from(lt, h->fp32, h->st);
            sync(h.get());   // host layouts are freed at scope end
        }
        alloc_iterates(h.get());
        if (h->fp32) autotune<float>(h.get());
        else autotune<double>(h.get());
        alloc_partials(h.get());
        h->lambda = o.lambda > 0 ? o.lambda : power_method(h.get());
        sync(h.get());
    } catch (const HipError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return fail(HPR_ERR_NOMEM, "host allocation failed");
    }
    h->setup_s = now_s() - t0;
    *out = h.release();
    return HPR_OK;
}

extern "C" int hpr_destroy(hpr_handle* h) {
    delete h;
    return HPR_OK;
}

extern "C" int hpr_set_bounds(hpr_handle* h, const double* col_lo, const double* col_hi) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    const int32_t n = h->n;
    std::vector<double> lo(h->l_s), hi(h->u_s);
    for (int32_t j = 0; j < n; ++j) {
        const double a = col_lo ? col_lo[j] : h->l_s[j] * h->beta_b * h->dc[j];
        const double b = col_hi ? col_hi[j] : h->u_s[j] * h->beta_b * h->dc[j];
        if (std::isnan(a) || std::isnan(b) || a > b || a == INFINITY || b == -INFINITY)
            return fail(HPR_ERR_INVALID, "bad column bounds at %d", j);
        if (col_lo) lo[j] = a / (h->beta_b * h->dc[j]);
        if (col_hi) hi[j] = b / (h->beta_b * h->dc[j]);
    }
    try {
        h->l_s = lo;
        h->u_s = hi;
        HIP_OK(hipMemcpyAsync(h->l64.p, lo.data(), sizeof(double) * n, hipMemcpyHostToDevice, h->st));
        HIP_OK(hipMemcpyAsync(h->u64.p, hi.data(), sizeof(double) * n, hipMemcpyHostToDevice, h->st));
        if (h->fp32) {
            launch_cast<float>(h->l64.as<double>(), h->l32.as<float>(), n, h->st);
            launch_cast<float>(h->u64.as<double>(), h->u32.as<float>(), n, h->st);
        }
        sync(h);
    } catch (const HipError& e) {
        return e.code;
    }
    return HPR_OK;
}

extern "C" int hpr_set_start(hpr_handle* h, const double* x0, const double* y0) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    if (x0) {
        for (int32_t j = 0; j < h->n; ++j)
            if (!std::isfinite(x0[j])) return fail(HPR_ERR_INVALID, "non-finite x0 at %d", j);
        h->x_start.assign(x0, x0 + h->n);
    } else {
        h->x_start.clear();
    }
    if (y0) {
        for (int32_t i = 0; i < h->m; ++i)
            if (!std::isfinite(y0[i])) return fail(HPR_ERR_INVALID, "non-finite y0 at %d", i);
        h->y_start.assign(y0, y0 + h->m);
    } else {
        h->y_start.clear();
    }
    return HPR_OK;
}

// ---------------------------------------------------------------- solve

namespace {

struct CheckVals {
    double rel_p, rel_d, rel_gap, rel_kkt, pobj, dobj, merit, move_x, move_y;
    bool bad;
};

// Launches both check kernels and the fixed-order finish; returns the host-side values.
template <typename Tm, typename Tp, typename Tv>
CheckVals run_check(hpr_handle* h, double sigma) {
    hipStream_t st = h->st;
    const DevCsr<Tm> A = h->A.view<Tm>();
    const DevCsr<Tm> At = h->At.view<Tm>();
    const DevProb<Tp> p = h->prob<Tp>();
    const DevIter<Tv> v = h->iter<Tv>();
    const int nbr = A.bins.block_off[kNumBins], nbc = At.bins.block_off[kNumBins];
    double* sums = h->sums.as<double>();
    if (nbr > 0) {
        launch_check_rows<Tm, Tp, Tv>(A, p, v, h->beta_b, h->part_r.as<double>(), st);
        launch_finish_sums(h->part_r.as<double>(), kRowQ, nbr, sums, st);
    } else {
        HIP_OK(hipMemsetAsync(sums, 0, sizeof(double) * kMaxQ, st));
    }
    launch_check_cols<Tm, Tp, Tv>(At, p, v, h->beta_c, h->part_c.as<double>(), st);
    launch_finish_sums(h->part_c.as<double>(), kColQ, nbc, sums + kMaxQ, st);
    HIP_OK(hipMemcpyAsync(h->pinned, sums, sizeof(double) * 2 * kMaxQ, hipMemcpyDeviceToHost, st));
    sync(h);
    const double* r = h->pinned;
    const double* c = h->pinned + kMaxQ;
    CheckVals cv;
    const double bb = h->beta_b * h->beta_c;
    cv.rel_p = std::sqrt(r[0]) / (1.0 + h->norm_b);
    cv.rel_d = std::sqrt(c[0]) / (1.0 + h->norm_c);
    cv.pobj = bb * c[1] + h->obj_offset;
    cv.dobj = bb * (r[3] + c[2]) + h->obj_offset;
    cv.rel_gap = std::fabs(cv.pobj - cv.dobj) / (1.0 + std::fabs(cv.pobj) + std::fabs(cv.dobj));
    cv.rel_kkt = std::max(cv.rel_p, std::max(cv.rel_d, cv.rel_gap));
    const double r2 = c[3] / sigma + h->lambda * sigma * r[1] + 2.0 * r[2];
    cv.merit = std::sqrt(r2 > 0 ? r2 : 0.0);
    cv.move_x = std::sqrt(c[4]);
    cv.move_y = std::sqrt(r[4]);
    cv.bad = (r[5] + c[5]) > 0 || !std::isfinite(cv.rel_kkt) || !std::isfinite(cv.pobj) ||
             !std::isfinite(cv.merit);
    return cv;
}

template <typename T>
void upload_start(hpr_handle* h) {
    const int32_t n = h->n, m = h->m;
    std::vector<T> xs(n), ys(std::max(m, 1));
    for (int32_t j = 0; j < n; ++j) {
        double v = h->x_start.empty() ? 0.0 : h->x_start[j] / (h->beta_b * h->dc[j]);
        v = v < h->l_s[j] ? h->l_s[j] : (v > h->u_s[j] ? h->u_s[j] : v);
        xs[j] = T(v);
    }
    for (int32_t i = 0; i < m; ++i) {
        double v = h->y_start.empty() ? 0.0 : h->y_start[i] / (h->beta_c * h->dr[i]);
        if (!std::isfinite(h->lo_s[i]) && v > 0) v = 0.0;
        if (!std::isfinite(h->hi_s[i]) && v < 0) v = 0.0;
        ys[i] = T(v);
    }
    const size_t es = sizeof(T);
    HIP_OK(hipMemcpyAsync(h->x0.p, xs.data(), es * n, hipMemcpyHostToDevice, h->st));
    HIP_OK(hipMemcpyAsync(h->x.p, xs.data(), es * n, hipMemcpyHostToDevice, h->st));
    if (m > 0) {
        HIP_OK(hipMemcpyAsync(h->y0.p, ys.data(), es * m, hipMemcpyHostToDevice, h->st));
        HIP_OK(hipMemcpyAsync(h->y.p, ys.data(), es * m, hipMemcpyHostToDevice, h->st));
    }
    sync(h);
}

void put_ctrl(hpr_handle* h, double sigma, int64_t k_base) {
    h->ctrl_h->sigma = sigma;
    h->ctrl_h->s = 1.0 / (h->lambda * sigma);
    h->ctrl_h->lambda = h->lambda;
    h->ctrl_h->k_base = k_base;
    HIP_OK(hipMemcpyAsync(h->ctrl.p, h->ctrl_h, sizeof(Ctrl), hipMemcpyHostToDevice, h->st));
}

// The solve loop. Iteration `it` (0-based) is a check when it % check_every == 0 or it is
// the last allowed one. At a check: stop if rel_kkt <= tol (in FP32 storage, confirmed by an
// FP64 re-evaluation); otherwise restart when the merit r = ||(x - xbar, y - ybar)||_M fell
// to 0.2 r0, or to 0.8 r0 while rising, or when the iterations since the last restart reach
// 0.2 of all iterations; at a restart sigma <- sqrt(sigma sigma*), sigma* = ||dx|| /
// (sqrt(lambda) ||dy||) from the anchor move (skipped below 1e-12), clamped to [1e-4, 1e4],
// and the anchor and iterate become the bar point.
template <typename T>
void solve_loop(hpr_handle* h, hpr_info* info, double t0) {
    const hpr_opts& o = h->opts;
    hipStream_t st = h->st;
    upload_start<T>(h);
    const DevCsr<T> A = h->A.view<T>(), At = h->At.view<T>();
    const DevProb<T> p = h->prob<T>();
    const DevIter<T> v = h->iter<T>();
    double sigma = o.sigma0;
    int64_t it = 0, k = 0, restarts = 0;
    double r0 = 0.0, r_prev = 0.0;
    int term = HPR_ITER_LIMIT;
    CheckVals cv{};
    put_ctrl(h, sigma, 0);
    h->kstats = hpr_kernel_stats{};
    if (o.profile && !h->ev[0])
        for (hipEvent_t& e : h->ev) HIP_OK(hipEventCreate(&e));
    while (true) {
        const int64_t nb = (it == 0) ? 1 : std::min<int64_t>(o.check_every, o.max_iter - it);
        const bool sample = o.profile && nb >= 2;
        for (int64_t j = 0; j < nb; ++j) {
            const bool chk = (j == nb - 1);
            if (sample && j == 0) HIP_OK(hipEventRecord(h->ev[0], st));
            launch_primal_step<T>(At, p, v, h->ctrl.as<Ctrl>(), (int)j, chk, st);
            if (sample && j == 0) HIP_OK(hipEventRecord(h->ev[1], st));
            launch_dual_step<T>(A, p, v, h->ctrl.as<Ctrl>(), (int)j, chk, st);
            if (sample && j == 0) HIP_OK(hipEventRecord(h->ev[2], st));
        }
        HIP_OK(hipGetLastError());
        it += nb;
        k += nb;
        cv = run_check<T, T, T>(h, sigma);
        if (sample) {
            float a = 0.f, b = 0.f;
            HIP_OK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
            HIP_OK(hipEventElapsedTime(&b, h->ev[1], h->ev[2]));
            h->kstats.primal_ms += a;
            h->kstats.dual_ms += b;
            h->kstats.samples += 1;
        }
        const bool last = it >= o.max_iter;
        const bool timed_out = o.time_limit_s > 0 && now_s() - t0 > o.time_limit_s;
        if (cv.bad) { term = HPR_NUMERIC_FAIL; break; }
        if (cv.rel_kkt <= o.tol) {
            if (!h->fp32) { term = HPR_SOLVED; break; }
            const CheckVals v64 = run_check<double, double, float>(h, sigma);
            if (v64.rel_kkt <= o.tol) { term = HPR_SOLVED; break; }
        }
        if (last) { term = HPR_ITER_LIMIT; break; }
        if (timed_out) { term = HPR_TIME_LIMIT; break; }
        const double r = cv.merit;
        if (it == 1) {
            r0 = r;
            r_prev = r;
            put_ctrl(h, sigma, k);
            continue;
        }
        bool do_restart = false;
        if (o.restart) {
            if (r <= 0.2 * r0) do_restart = true;
            else if (r <= 0.8 * r0 && r > r_prev) do_restart = true;
            else if ((double)k >= 0.2 * (double)it) do_restart = true;
        }
        if (do_restart) {
            if (o.sigma_update && cv.move_x > 1e-12 && cv.move_y > 1e-12) {
                const double star = cv.move_x / (std::sqrt(h->lambda) * cv.move_y);
                sigma = std::sqrt(sigma * star);
                sigma = sigma < 1e-4 ? 1e-4 : (sigma > 1e4 ? 1e4 : sigma);
            }
            launch_restart<T>(v, h->n, h->m, st);
            k = 0;
            restarts += 1;
            r0 = r;
        }
        r_prev = r;
        put_ctrl(h, sigma, k);
    }
    if (h->fp32 && term != HPR_NUMERIC_FAIL) {
        // report the residuals of the returned point in FP64
        const CheckVals v64 = run_check<double, double, float>(h, sigma);
        cv.rel_p = v64.rel_p; cv.rel_d = v64.rel_d; cv.rel_gap = v64.rel_gap; cv.rel_kkt = v64.rel_kkt;
        cv.pobj = v64.pobj; cv.dobj = v64.dobj;
    }
    sync(h);
    info->term = term;
    info->iters = it;
    info->restarts = restarts;
    info->pobj = cv.pobj;
    info->dobj = cv.dobj;
    info->rel_p = cv.rel_p;
    info->rel_d = cv.rel_d;
    info->rel_gap = cv.rel_gap;
    info->rel_kkt = cv.rel_kkt;
    info->lambda = h->lambda;
    info->sigma = sigma;
}

}  // namespace

extern "C" int hpr_solve(hpr_handle* h, hpr_info* info) {
    g_err.clear();
    if (!h || !info) return fail(HPR_ERR_INVALID, "handle or info is NULL");
    std::memset(info, 0, sizeof(*info));
    const double t0 = now_s();
    try {
        int dev = 0;
        HIP_OK(hipGetDevice(&dev));
        if (dev != h->device) HIP_OK(hipSetDevice(h->device));
        if (h->fp32) solve_loop<float>(h, info, t0);
        else solve_loop<double>(h, info, t0);
        if (dev != h->device) HIP_OK(hipSetDevice(dev));
    } catch (const HipError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return fail(HPR_ERR_NOMEM, "host allocation failed");
    }
    info->setup_s = h->setup_s;
    info->solve_s = now_s() - t0;
    h->solved_once = true;
    return HPR_OK;
}

extern "C" int hpr_get_kernel_stats(hpr_handle* h, hpr_kernel_stats* out) {
    g_err.clear();
    if (!h || !out) return fail(HPR_ERR_INVALID, "handle or out is NULL");
    *out = h->kstats;
    out->unroll_a = h->A.unroll;
    out->unroll_at = h->At.unroll;
    if (out->samples > 0) {
        out->primal_ms /= (double)out->samples;
        out->dual_ms /= (double)out->samples;
    }
    return HPR_OK;
}

extern "C" int hpr_get_solution(hpr_handle* h, double* x, double* y, double* z) {
    g_err.clear();
    if (!h) return fail(HPR_ERR_INVALID, "handle is NULL");
    if (!h->solved_once) return fail(HPR_ERR_STATE, "no solve has run on this handle");
    try {
        if (h->fp32)
            launch_unscale<float>(h->iter<float>(), h->dr_d.as<double>(), h->dc_d.as<double>(), h->n, h->m,
                                  h->beta_b, h->beta_c, h->ux.as<double>(), h->uy.as<double>(),
                                  h->uz.as<double>(), h->st);
        else
            launch_unscale<double>(h->iter<double>(), h->dr_d.as<double>(), h->dc_d.as<double>(), h->n, h->m,
                                   h->beta_b, h->beta_c, h->ux.as<double>(), h->uy.as<double>(),
                                   h->uz.as<double>(), h->st);
        if (x) HIP_OK(hipMemcpyAsync(x, h->ux.p, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->st));
        if (y && h->m) HIP_OK(hipMemcpyAsync(y, h->uy.p, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->st));
        if (z) HIP_OK(hipMemcpyAsync(z, h->uz.p, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->st));
        sync(h);
    } catch (const HipError& e) {
        return e.code;
    }
    return HPR_OK;
}
