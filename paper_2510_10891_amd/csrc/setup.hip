// Device-side setup of one LP (Section III-A scaling, A~^T, padded layouts): the caller's CSR is
// uploaded once and everything of size nnz is built on the GPU; only per-row metadata (padded
// row starts, smallest/largest columns, tile runs) and the diagonal scaling come back to the host,
// which builds the block schedules from them.
//
//   1. entry -> row map; A^T by a stable radix sort of the entries by column (entries of a
//      column keep increasing row order), its row pointers from the sorted keys;
//   2. scaling: optional Ruiz passes (row / column maxima of |a_ij dr_i dc_j|) and Pock-Chambolle
//      with alpha = 1 (row / column absolute sums), each row and each column reduced by one
//      thread in entry order (deterministic); the host forms the factors 1 / sqrt (empty rows
//      and columns keep 1), so they equal the host pipeline's bit for bit;
//   3. padded layouts of A~ (rows of the caller's CSR, which must be in column order) and A~^T:
//      every row padded to a multiple of 4 entries with value 0 at its largest column, values
//      a_ij dr_i dc_j in FP64 (and FP32 when asked), 32-bit columns and 16-bit offsets from the
//      row's smallest column (0 for rows spanning 65,536 columns or more);
//   4. per row: smallest and largest column, and the runs of equal column / tile (tile counts
//      of the LDS window choice).
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <cmath>
#include <vector>

#include "internal.h"

namespace hpr {

namespace {

constexpr int kT = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

__global__ void entry_rows_kernel(const int64_t* rp, int32_t m, int32_t* row_of, uint32_t* idx) {
    const int32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
        row_of[k] = i;
        idx[k] = (uint32_t)k;
    }
}

// tptr[j + 1] = number of entries of column j (from the sorted keys: first / last position)
__global__ void column_ends_kernel(const uint32_t* keys, int64_t nnz, int64_t* tptr, int32_t n) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= nnz) return;
    const uint32_t j = keys[q];
    if (q + 1 == nnz || keys[q + 1] != j) tptr[j + 1] = q + 1;   // end of column j
    (void)n;
}


// One scaling pass over rows (A in the caller's order) or columns (through the sorted entry list):
// out[i] = sum or max of |v dr dc| over the row's entries in order (the host forms the factors).
template <bool SUM, bool COLS>
__global__ void scale_pass_kernel(const int64_t* ptr, const uint32_t* perm, const int32_t* other,
                                  const double* v, const double* dr, const double* dc, double* out, int32_t count) {
    const int32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= count) return;
    double r = 0.0;
    for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int64_t k = COLS ? (int64_t)perm[q] : q;
        const int32_t o = other[k];   // the entry's column (rows pass) or row (columns pass)
        const double a = COLS ? fabs(v[k] * dr[o] * dc[i]) : fabs(v[k] * dr[i] * dc[o]);
        r = SUM ? r + a : (a > r ? a : r);
    }
    out[i] = r;
}

// padded length of row i, (len + 3) / 4 * 4, into out[i] (the scan turns it into row starts)
__global__ void padded_lengths_kernel(const int64_t* ptr, int32_t rows, int64_t* out) {
    const int32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= rows) return;
    const int64_t len = ptr[i + 1] - ptr[i];
    out[i] = (len + kVec - 1) / kVec * kVec;
}

// Row i of a layout: entries q in [ptr[i], ptr[i+1]) of the source list (perm maps list positions to
// entries for A^T, identity for A), column col_of[entry], value v[entry] dr[row] dc[col].
template <bool TRANS>
__global__ void fill_layout_kernel(const int64_t* ptr, const int64_t* start, const uint32_t* perm,
                                   const int32_t* cols_in, const int32_t* row_of, const double* v,
                                   const double* dr, const double* dc, int32_t rows, int32_t* col,
                                   uint16_t* col16, double* val64, float* val32, int32_t* base, int32_t* top,
                                   uint8_t* wide) {
    const int32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= rows) return;
    const int64_t b = ptr[i], e = ptr[i + 1], d0 = start[i], d1 = start[i + 1];
    if (b == e) {
        base[i] = 0;
        top[i] = 0;
        wide[i] = 0;
        return;
    }
    auto column = [&](int64_t q) -> int32_t {
        return TRANS ? row_of[perm[q]] : cols_in[q];
    };
    const int32_t lo = column(b), hi = column(e - 1);   // rows are in column order
    const bool w = (int64_t)hi - lo >= 65536;
    base[i] = lo;
    top[i] = hi;
    wide[i] = w ? 1 : 0;
    int64_t d = d0;
    for (int64_t q = b; q < e; ++q, ++d) {
        const int64_t k = TRANS ? (int64_t)perm[q] : q;
        const int32_t c = column(q);
        // the scaled entry a_ij dr_i dc_j, formed as (a dr) dc like the host layouts
        const double a = TRANS ? v[k] * dr[c] * dc[i] : v[k] * dr[i] * dc[c];
        col[d] = c;
        col16[d] = w ? (uint16_t)0 : (uint16_t)(c - lo);
        val64[d] = a;
        if (val32) val32[d] = (float)a;
    }
    for (; d < d1; ++d) {   // padding: value 0 at the row's largest column
        col[d] = hi;
        col16[d] = w ? (uint16_t)0 : (uint16_t)(hi - lo);
        val64[d] = 0.0;
        if (val32) val32[d] = 0.0f;
    }
}

// runs of equal col / tile per row (rows in column order): count, then write (id, count)
__global__ void tile_runs_kernel(const int64_t* start, const int32_t* col, int32_t rows, int32_t tile,
                                 const int64_t* out_ptr, int64_t* runs, int32_t* id, int32_t* cnt) {
    const int32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= rows) return;
    const int64_t b = start[i], e = start[i + 1];
    if (!out_ptr) {
        int64_t r = 0;
        for (int64_t k = b; k < e; ++k) r += (k == b || col[k] / tile != col[k - 1] / tile) ? 1 : 0;
        runs[i] = r;
        return;
    }
    int64_t q = out_ptr[i] - 1;
    for (int64_t k = b; k < e; ++k) {
        const int32_t t = col[k] / tile;
        if (k == b || t != col[k - 1] / tile) {
            ++q;
            id[q] = t;
            cnt[q] = 0;
        }
        ++cnt[q];
    }
}

#define SETUP_HIP(expr)                                  \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return e_;                 \
    } while (0)

// exclusive scan of in[0..count) into out[0..count], out[count] = total
// out[0..count] = running maximum of in[0..count]
hipError_t max_scan(const int64_t* in, int64_t* out, int32_t count, hipStream_t st, DevScratch& tmp) {
    size_t bytes = 0;
    SETUP_HIP(rocprim::inclusive_scan(nullptr, bytes, in, out, (size_t)count + 1, rocprim::maximum<int64_t>(), st));
    SETUP_HIP(tmp.reserve(bytes));
    return rocprim::inclusive_scan(tmp.p, bytes, in, out, (size_t)count + 1, rocprim::maximum<int64_t>(), st);
}

hipError_t exclusive_scan(const int64_t* in, int64_t* out, int32_t count, hipStream_t st, DevScratch& tmp) {
    size_t bytes = 0;
    SETUP_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, int64_t(0), (size_t)count + 1, rocprim::plus<int64_t>(),
                                      st));
    SETUP_HIP(tmp.reserve(bytes));
    return rocprim::exclusive_scan(tmp.p, bytes, in, out, int64_t(0), (size_t)count + 1, rocprim::plus<int64_t>(), st);
}

}  // namespace

hipError_t DevScratch::reserve(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    const hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
    if (e == hipSuccess) cap = bytes;
    return e;
}

DevScratch::~DevScratch() {
    if (p) (void)hipFree(p);
}

hipError_t device_setup(const DevSetupIn& in, DevSetupOut& out, hipStream_t st) {
    const int32_t m = in.m, n = in.n;
    const int64_t nnz = in.nnz;
    DevScratch tmp;
    // 1. entry rows, sort by column (stable: equal keys keep their entry order = row order)
    SETUP_HIP(out.row_of.reserve(sizeof(int32_t) * (nnz + 1)));
    SETUP_HIP(out.idx.reserve(sizeof(uint32_t) * (nnz + 1)));
    SETUP_HIP(out.perm.reserve(sizeof(uint32_t) * (nnz + 1)));
    SETUP_HIP(out.keys.reserve(sizeof(uint32_t) * (nnz + 1)));
    int32_t* row_of = static_cast<int32_t*>(out.row_of.p);
    uint32_t* idx = static_cast<uint32_t*>(out.idx.p);
    uint32_t* perm = static_cast<uint32_t*>(out.perm.p);
    uint32_t* keys = static_cast<uint32_t*>(out.keys.p);
    if (m > 0) hipLaunchKernelGGL(entry_rows_kernel, dim3(grid_for(m)), dim3(kT), 0, st, in.rp, m, row_of, idx);
    int bits = 1;
    while (bits < 32 && (int64_t(1) << bits) < (int64_t)n) ++bits;
    if (nnz > 0) {
        size_t bytes = 0;
        const uint32_t* kin = reinterpret_cast<const uint32_t*>(in.ci);
        SETUP_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, keys, idx, perm, (size_t)nnz, 0, bits, st));
        SETUP_HIP(tmp.reserve(bytes));
        SETUP_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, kin, keys, idx, perm, (size_t)nnz, 0, bits, st));
    }
    SETUP_HIP(out.tptr.reserve(sizeof(int64_t) * ((size_t)n + 1)));
    int64_t* tptr = static_cast<int64_t*>(out.tptr.p);
    SETUP_HIP(hipMemsetAsync(tptr, 0xFF, sizeof(int64_t) * ((size_t)n + 1), st));   // -1: no entry yet
    if (nnz > 0) hipLaunchKernelGGL(column_ends_kernel, dim3(grid_for(nnz)), dim3(kT), 0, st, keys, nnz, tptr, n);
    // columns without entries take the end of the previous column: tptr[0] = 0, then a running
    // maximum (through a copy: the scan does not work in place)
    SETUP_HIP(hipMemsetAsync(tptr, 0, sizeof(int64_t), st));
    {
        DevScratch ends;
        SETUP_HIP(ends.reserve(sizeof(int64_t) * ((size_t)n + 1)));
        SETUP_HIP(hipMemcpyAsync(ends.p, tptr, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, st));
        SETUP_HIP(max_scan(static_cast<const int64_t*>(ends.p), tptr, n, st, tmp));
        SETUP_HIP(hipStreamSynchronize(st));   // `ends` is freed at the end of this scope
    }
    // 2. scaling: the device reduces, the host forms the factors f *= (r > 0 ? 1 / sqrt(r) : 1)
    double* dr = in.dr;
    double* dc = in.dc;
    for (int32_t i = 0; i < m; ++i) in.dr_host[i] = 1.0;
    for (int32_t j = 0; j < n; ++j) in.dc_host[j] = 1.0;
    SETUP_HIP(out.f.reserve(sizeof(double) * ((size_t)m + n + 1)));
    double* rs = static_cast<double*>(out.f.p);
    double* cs = rs + m;
    auto upload_factors = [&]() -> hipError_t {
        if (m > 0) SETUP_HIP(hipMemcpyAsync(dr, in.dr_host, sizeof(double) * m, hipMemcpyHostToDevice, st));
        SETUP_HIP(hipMemcpyAsync(dc, in.dc_host, sizeof(double) * n, hipMemcpyHostToDevice, st));
        return hipStreamSynchronize(st);
    };
    SETUP_HIP(upload_factors());
    std::vector<double> rh((size_t)m), ch((size_t)n);
    auto pass = [&](bool sum) -> hipError_t {
        if (m > 0) {
            if (sum)
                hipLaunchKernelGGL((scale_pass_kernel<true, false>), dim3(grid_for(m)), dim3(kT), 0, st, in.rp,
                                   nullptr, in.ci, in.v, dr, dc, rs, m);
            else
                hipLaunchKernelGGL((scale_pass_kernel<false, false>), dim3(grid_for(m)), dim3(kT), 0, st, in.rp,
                                   nullptr, in.ci, in.v, dr, dc, rs, m);
        }
        if (sum)
            hipLaunchKernelGGL((scale_pass_kernel<true, true>), dim3(grid_for(n)), dim3(kT), 0, st, tptr, perm, row_of,
                               in.v, dr, dc, cs, n);
        else
            hipLaunchKernelGGL((scale_pass_kernel<false, true>), dim3(grid_for(n)), dim3(kT), 0, st, tptr, perm,
                               row_of, in.v, dr, dc, cs, n);
        SETUP_HIP(hipGetLastError());
        if (m > 0) SETUP_HIP(hipMemcpyAsync(rh.data(), rs, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        SETUP_HIP(hipMemcpyAsync(ch.data(), cs, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        SETUP_HIP(hipStreamSynchronize(st));
        for (int32_t i = 0; i < m; ++i) in.dr_host[i] *= rh[i] > 0 ? 1.0 / std::sqrt(rh[i]) : 1.0;
        for (int32_t j = 0; j < n; ++j) in.dc_host[j] *= ch[j] > 0 ? 1.0 / std::sqrt(ch[j]) : 1.0;
        return upload_factors();
    };
    for (int32_t it = 0; it < in.ruiz_iters; ++it) SETUP_HIP(pass(false));
    if (in.pc) SETUP_HIP(pass(true));
    // 3. layouts of A~ and A~^T
    for (int which = 0; which < 2; ++which) {
        DevLayout& L = which == 0 ? out.a : out.at;
        const int32_t rows = which == 0 ? m : n;
        const int64_t* ptr = which == 0 ? in.rp : tptr;
        SETUP_HIP(L.start.reserve(sizeof(int64_t) * ((size_t)rows + 1)));
        SETUP_HIP(out.lens.reserve(sizeof(int64_t) * ((size_t)rows + 1)));
        int64_t* start = static_cast<int64_t*>(L.start.p);
        int64_t* lens = static_cast<int64_t*>(out.lens.p);
        if (rows > 0) hipLaunchKernelGGL(padded_lengths_kernel, dim3(grid_for(rows)), dim3(kT), 0, st, ptr, rows, lens);
        SETUP_HIP(hipMemsetAsync(lens + rows, 0, sizeof(int64_t), st));
        SETUP_HIP(exclusive_scan(lens, start, rows, st, tmp));
        SETUP_HIP(hipMemcpyAsync(&L.padded, start + rows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        SETUP_HIP(hipStreamSynchronize(st));
        const int64_t P = L.padded;
        SETUP_HIP(L.col.reserve(sizeof(int32_t) * (P + 1)));
        SETUP_HIP(L.col16.reserve(sizeof(uint16_t) * (P + 1)));
        SETUP_HIP(L.val64.reserve(sizeof(double) * (P + 1)));
        if (in.fp32) SETUP_HIP(L.val32.reserve(sizeof(float) * (P + 1)));
        SETUP_HIP(L.base.reserve(sizeof(int32_t) * ((size_t)rows + 1)));
        SETUP_HIP(L.top.reserve(sizeof(int32_t) * ((size_t)rows + 1)));
        SETUP_HIP(L.wide.reserve((size_t)rows + 1));
        if (rows > 0) {
            if (which == 0)
                hipLaunchKernelGGL((fill_layout_kernel<false>), dim3(grid_for(rows)), dim3(kT), 0, st, ptr, start,
                                   nullptr, in.ci, nullptr, in.v, dr, dc, rows, (int32_t*)L.col.p,
                                   (uint16_t*)L.col16.p, (double*)L.val64.p, in.fp32 ? (float*)L.val32.p : nullptr,
                                   (int32_t*)L.base.p, (int32_t*)L.top.p, (uint8_t*)L.wide.p);
            else
                hipLaunchKernelGGL((fill_layout_kernel<true>), dim3(grid_for(rows)), dim3(kT), 0, st, ptr, start,
                                   perm, nullptr, row_of, in.v, dr, dc, rows, (int32_t*)L.col.p,
                                   (uint16_t*)L.col16.p, (double*)L.val64.p, in.fp32 ? (float*)L.val32.p : nullptr,
                                   (int32_t*)L.base.p, (int32_t*)L.top.p, (uint8_t*)L.wide.p);
        }
        // 4. tile runs
        SETUP_HIP(L.tptr.reserve(sizeof(int64_t) * ((size_t)rows + 1)));
        int64_t* runptr = static_cast<int64_t*>(L.tptr.p);
        if (rows > 0)
            hipLaunchKernelGGL(tile_runs_kernel, dim3(grid_for(rows)), dim3(kT), 0, st, start, (const int32_t*)L.col.p,
                               rows, in.tile, nullptr, lens, nullptr, nullptr);
        SETUP_HIP(hipMemsetAsync(lens + rows, 0, sizeof(int64_t), st));
        SETUP_HIP(exclusive_scan(lens, runptr, rows, st, tmp));
        SETUP_HIP(hipMemcpyAsync(&L.nruns, runptr + rows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        SETUP_HIP(hipStreamSynchronize(st));
        SETUP_HIP(L.tid.reserve(sizeof(int32_t) * (L.nruns + 1)));
        SETUP_HIP(L.tcnt.reserve(sizeof(int32_t) * (L.nruns + 1)));
        if (rows > 0)
            hipLaunchKernelGGL(tile_runs_kernel, dim3(grid_for(rows)), dim3(kT), 0, st, start, (const int32_t*)L.col.p,
                               rows, in.tile, runptr, nullptr, (int32_t*)L.tid.p, (int32_t*)L.tcnt.p);
        SETUP_HIP(hipGetLastError());
    }
    return hipStreamSynchronize(st);
}

}  // namespace hpr
