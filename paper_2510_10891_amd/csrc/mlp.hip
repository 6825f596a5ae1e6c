// Warm-start network on the GPU: a multilayer perceptron with BF16 weights and
// activations on the matrix cores (MFMA, FP32 accumulation), FP32 master weights,
// and its training step (forward, backward, Adam) written as plain kernels.
//
// Layer i: z_i = h_i W_i + b_i, h_{i+1} = max(z_i, 0) except after the last layer.
// Loss: 0.5 * mean over all output entries of (out - target)^2.
// Adam (Kingma and Ba 2015) with bias correction on the FP32 master copy; the BF16 copy
// used by the products is refreshed after every step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hprlp.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxLayers = 8;
constexpr int kTile = 16;
constexpr int kThreads = 256;

__host__ __device__ inline uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));  // inf/nan
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float from_bf16(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// C(i, j) = sum_k A(i, k) B(k, j) for an M x N output, BF16 operands addressed with
// element strides (A(i,k) = A[i*sa0 + k*sa1], B(k,j) = B[k*sb0 + j*sb1]) so transposed
// operands need no copy; one of each operand's strides is 1. A workgroup of four wavefronts
// computes a 64 x 64 block of C: per step of 32 depths it stages the A (64 x 32) and B (32 x 64)
// tiles in LDS with loads that run along the operand's contiguous dimension (coalesced), both
// stored depth-contiguous, and each wavefront runs v_mfma_f32_16x16x16_bf16 on its 32 x 32
// quarter (2 x 2 tiles, depths in ascending steps of 16: the summation order of a one-tile-per-
// wavefront loop). Out-of-range rows/columns/depths are staged as zero. With `ws` the depth range
// is split over gridDim.z slices that write FP32 partial blocks to ws[z][M][N]; finish_split_kernel
// adds them in slice order. Epilogue: + bias (FP32, may be null), optional ReLU, FP32 and/or BF16
// store.
struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int64_t sa0, sa1, sb0, sb1;
    int M, N, K;
    const float* bias;
    int relu;
    float* C32;        // [M][N] or null
    uint16_t* C16;     // [M][N] or null
    float* ws;         // split-depth partials [splits][M][N], or null (no split)
    int kslice;        // depths per slice (multiple of kBK) when ws is set
};

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdsRow = kBK + 8;     // shorts per staged row (padding against bank conflicts)

__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int i, int j, float v) {
    v += g.bias ? g.bias[j] : 0.f;
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.C32) g.C32[(int64_t)i * g.N + j] = v;
    if (g.C16) g.C16[(int64_t)i * g.N + j] = to_bf16(v);
}

__global__ __launch_bounds__(kThreads) void gemm_bf16_kernel(GemmArgs g) {
    __shared__ short As[kBM * kLdsRow];   // [row][depth]
    __shared__ short Bs[kBN * kLdsRow];   // [column][depth]
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int i0 = blockIdx.y * kBM, j0 = blockIdx.x * kBN;
    const int kb = g.ws ? blockIdx.z * g.kslice : 0;
    const int ke = g.ws ? min(g.K, kb + g.kslice) : g.K;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += kBK) {
        // stage A: 64 x 32 = 8 per thread, consecutive threads along the contiguous dimension
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int q = e * kThreads + t;
            int row, k;
            if (g.sa1 == 1) { row = q / kBK; k = q % kBK; }
            else            { k = q / kBM;  row = q % kBM; }
            const int ia = i0 + row, ka = k0 + k;
            As[row * kLdsRow + k] = (ia < g.M && ka < ke) ? (short)g.A[(int64_t)ia * g.sa0 + (int64_t)ka * g.sa1] : (short)0;
        }
        // stage B: 32 x 64
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int q = e * kThreads + t;
            int col, k;
            if (g.sb1 == 1) { k = q / kBN; col = q % kBN; }
            else            { col = q / kBK; k = q % kBK; }
            const int jb = j0 + col, kk = k0 + k;
            Bs[col * kLdsRow + k] = (jb < g.N && kk < ke) ? (short)g.B[(int64_t)kk * g.sb0 + (int64_t)jb * g.sb1] : (short)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 16) {
            bf16x4 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const short* pa = As + (wm + a * 16 + r) * kLdsRow + kk + kq;
                const short* pb = Bs + (wn + a * 16 + r) * kLdsRow + kk + kq;
                av[a] = bf16x4{pa[0], pa[1], pa[2], pa[3]};
                bv[a] = bf16x4{pb[0], pb[1], pb[2], pb[3]};
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + wn + b * 16 + r;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + wm + a * 16 + (lane >> 4) * 4 + u;
                if (i < g.M && j < g.N) {
                    if (g.ws) g.ws[((int64_t)blockIdx.z * g.M + i) * g.N + j] = acc[a][b][u];
                    else gemm_epilogue(g, i, j, acc[a][b][u]);
                }
            }
        }
}

// C = sum over the slices of ws, added in slice order, then the epilogue.
__global__ __launch_bounds__(kThreads) void finish_split_kernel(GemmArgs g, int splits) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t mn = (int64_t)g.M * g.N;
    if (idx >= mn) return;
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += g.ws[z * mn + idx];
    gemm_epilogue(g, (int)(idx / g.N), (int)(idx % g.N), v);
}

// Launch: one workgroup per 64 x 64 block of C. `ws_floats` (with g.ws) is the partial-sum
// room; the depth is split when the blocks alone would leave most of the GPU idle and the
// depth is long (the weight gradients, whose depth is the number of rows).
void gemm(GemmArgs g, hipStream_t st, int64_t ws_floats = 0) {
    if (g.M <= 0 || g.N <= 0) return;
    const int bx = (g.N + kBN - 1) / kBN, by = (g.M + kBM - 1) / kBM;
    int splits = 1;
    if (g.ws && ws_floats > 0 && g.K >= 4 * kBK * 16) {
        const int64_t blocks = (int64_t)bx * by;
        const int64_t want = (1024 + blocks - 1) / blocks;                 // ~1024 workgroups
        const int64_t room = ws_floats / ((int64_t)g.M * g.N);
        const int64_t depth = (g.K + 16 * kBK - 1) / (16 * kBK);            // >= 16 steps per slice
        splits = (int)std::max<int64_t>(1, std::min({want, room, depth, (int64_t)64}));
    }
    if (splits == 1) {
        g.ws = nullptr;
        hipLaunchKernelGGL(gemm_bf16_kernel, dim3(bx, by, 1), dim3(kThreads), 0, st, g);
        return;
    }
    g.kslice = ((g.K + splits - 1) / splits + kBK - 1) / kBK * kBK;
    splits = (g.K + g.kslice - 1) / g.kslice;
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3(bx, by, splits), dim3(kThreads), 0, st, g);
    const int64_t mn = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(finish_split_kernel, dim3((unsigned)((mn + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, g,
                       splits);
}

__global__ void f32_to_bf16_kernel(const float* s, uint16_t* d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = to_bf16(s[i]);
}

// g = (out - target) / count as BF16 (the gradient of the loss at the output) and per-block
// partial sums of (out - target)^2 (FP64) for the loss.
__global__ __launch_bounds__(kThreads) void output_grad_kernel(const float* out, const float* target, int64_t n,
                                                               float inv_count, uint16_t* g16, double* part) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float d = out[i] - target[i];
        s += (double)d * (double)d;
        g16[i] = to_bf16(d * inv_count);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dz = dh * (z > 0), BF16 in and out (z from the forward pass, FP32)
__global__ void relu_back_kernel(const float* z, uint16_t* g, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(z[i] > 0.f)) g[i] = 0;
}

// db[j] = sum_i g[i][j] (column sums in a fixed order, FP32 accumulate) in two passes: block
// (c, b) sums rows c*kBiasRows.. of columns b*kThreads.. into part[c][j] (consecutive threads on
// consecutive columns), then bias_grad_finish adds the chunks in order.
constexpr int kBiasRows = 128;

__global__ __launch_bounds__(kThreads) void bias_grad_kernel(const uint16_t* g, int rows, int cols, float* part) {
    const int j = blockIdx.y * kThreads + threadIdx.x;
    if (j >= cols) return;
    const int i0 = blockIdx.x * kBiasRows;
    const int i1 = min(rows, i0 + kBiasRows);
    float s = 0.f;
    for (int i = i0; i < i1; ++i) s += from_bf16(g[(int64_t)i * cols + j]);
    part[(int64_t)blockIdx.x * cols + j] = s;
}

__global__ __launch_bounds__(kThreads) void bias_grad_finish(const float* part, int chunks, int cols, float* db) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * cols + j];
    db[j] = s;
}

__global__ void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// Fixed device scratch of hpr_mlp_forward_device (BF16 input and hidden activations of a chunk
// of rows), one copy per GPU for the life of the process. In host code `scratch` names a
// host-side stand-in, never a device address: kernels receive the address that
// hipGetSymbolAddress returns for the current device (scratch_address), resolved once per
// device by hpr_mlp_create.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

#define MLP_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? HPR_ERR_NOMEM : HPR_ERR_HIP,       \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                \
    } while (0)

// The device address of `scratch` on device dev (resolved on the first call for that device,
// with dev current).
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HPR_ERR_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HPR_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HPR_OK;
}

}  // namespace

struct hpr_mlp {
    int L = 0;
    void* scratch_dev = nullptr;                                      // this device's `scratch`
    int sizes[kMaxLayers + 1] = {0};
    int64_t woff[kMaxLayers] = {0}, boff[kMaxLayers] = {0}, nparams = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    float *w = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;   // FP32 params / grads / moments
    uint16_t* w16 = nullptr;                                          // BF16 weights
    int64_t cap = 0;                                                  // rows the buffers hold
    uint16_t* x16 = nullptr;                                          // input, BF16
    uint16_t* h16[kMaxLayers + 1] = {nullptr};                        // activations, BF16
    float* z32[kMaxLayers] = {nullptr};                               // pre-activations, FP32
    uint16_t* g16 = nullptr;                                          // gradient scratch, BF16
    uint16_t* g16b = nullptr;
    float* xin = nullptr;                                             // staging of X and targets
    float* tgt = nullptr;
    double* part = nullptr;
    float* ws = nullptr;                                              // split-depth partials of dW
    int64_t ws_floats = 0;
    float* ws_bias = nullptr;                                         // row-chunk partials of db
    int64_t step = 0;
    ~hpr_mlp() {
        if (st) (void)hipStreamSynchronize(st);
        for (void* p : {(void*)w, (void*)grad, (void*)m, (void*)v, (void*)w16, (void*)ws}) (void)hipFree(p);
        release_rows();
        if (own_stream && st) (void)hipStreamDestroy(st);
    }
    void release_rows() {
        (void)hipFree(x16);
        for (int i = 0; i <= kMaxLayers; ++i) (void)hipFree(h16[i]), h16[i] = nullptr;
        for (int i = 0; i < kMaxLayers; ++i) (void)hipFree(z32[i]), z32[i] = nullptr;
        (void)hipFree(g16);
        (void)hipFree(g16b);
        (void)hipFree(xin);
        (void)hipFree(tgt);
        (void)hipFree(part);
        (void)hipFree(ws_bias);
        ws_bias = nullptr;
        x16 = g16 = g16b = nullptr;
        xin = tgt = nullptr;
        part = nullptr;
        cap = 0;
    }
    int width() const {
        int mx = 0;
        for (int i = 0; i <= L; ++i) mx = sizes[i] > mx ? sizes[i] : mx;
        return mx;
    }
    // room for up to 64 partial copies of the largest weight matrix, at most 64 MiB
    int ensure_ws() {
        if (ws) return HPR_OK;
        int64_t mx = 0;
        for (int i = 0; i < L; ++i) mx = std::max<int64_t>(mx, (int64_t)sizes[i] * sizes[i + 1]);
        ws_floats = std::min<int64_t>(64 * mx, (int64_t)16 << 20);
        MLP_HIP(hipMalloc(&ws, sizeof(float) * ws_floats));
        return HPR_OK;
    }
    int ensure_rows(int64_t n) {
        if (n <= cap) return HPR_OK;
        release_rows();
        const int64_t W = width();
        MLP_HIP(hipMalloc(&x16, sizeof(uint16_t) * n * sizes[0]));
        MLP_HIP(hipMalloc(&xin, sizeof(float) * n * W));
        MLP_HIP(hipMalloc(&tgt, sizeof(float) * n * sizes[L]));
        for (int i = 1; i <= L; ++i) MLP_HIP(hipMalloc(&h16[i], sizeof(uint16_t) * n * sizes[i]));
        for (int i = 0; i < L; ++i) MLP_HIP(hipMalloc(&z32[i], sizeof(float) * n * sizes[i + 1]));
        MLP_HIP(hipMalloc(&g16, sizeof(uint16_t) * n * W));
        MLP_HIP(hipMalloc(&g16b, sizeof(uint16_t) * n * W));
        MLP_HIP(hipMalloc(&part, sizeof(double) * 1024));
        MLP_HIP(hipMalloc(&ws_bias, sizeof(float) * ((n + kBiasRows - 1) / kBiasRows) * W));
        cap = n;
        return HPR_OK;
    }
};

namespace {

int refresh_bf16(hpr_mlp* q) {
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(q->nparams)), dim3(kThreads), 0, q->st, q->w, q->w16,
                       q->nparams);
    MLP_HIP(hipGetLastError());
    return HPR_OK;
}

// forward pass on rows already staged in q->xin (FP32 [n][sizes[0]]); leaves z32[L-1] = output
int forward_staged(hpr_mlp* q, int64_t n) {
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(n * q->sizes[0])), dim3(kThreads), 0, q->st, q->xin,
                       q->x16, n * q->sizes[0]);
    const uint16_t* h = q->x16;
    for (int i = 0; i < q->L; ++i) {
        GemmArgs g{};
        g.A = h;
        g.sa0 = q->sizes[i];
        g.sa1 = 1;
        g.B = q->w16 + q->woff[i];
        g.sb0 = q->sizes[i + 1];
        g.sb1 = 1;
        g.M = (int)n;
        g.N = q->sizes[i + 1];
        g.K = q->sizes[i];
        g.bias = q->w + q->boff[i];
        g.relu = i < q->L - 1;
        g.C32 = q->z32[i];
        g.C16 = i < q->L - 1 ? q->h16[i + 1] : nullptr;
        gemm(g, q->st);
        h = q->h16[i + 1];
    }
    MLP_HIP(hipGetLastError());
    return HPR_OK;
}

// loss and gradients into q->grad for rows staged in xin / tgt
int gradients_staged(hpr_mlp* q, int64_t n, float* loss) {
    int rc = q->ensure_ws();
    if (rc) return rc;
    rc = forward_staged(q, n);
    if (rc) return rc;
    const int L = q->L;
    const int64_t nout = n * q->sizes[L];
    const int nb = (int)std::min<int64_t>(1024, blocks_for(nout));
    hipLaunchKernelGGL(output_grad_kernel, dim3(nb), dim3(kThreads), 0, q->st, q->z32[L - 1], q->tgt, nout,
                       1.0f / (float)nout, q->g16, q->part);
    uint16_t* g = q->g16;       // gradient at z_i (BF16, [n][sizes[i+1]])
    uint16_t* other = q->g16b;
    for (int i = L - 1; i >= 0; --i) {
        const uint16_t* hin = i == 0 ? q->x16 : q->h16[i];
        // dW_i = h_i^T g  (K = rows)
        GemmArgs gw{};
        gw.A = hin;
        gw.sa0 = 1;
        gw.sa1 = q->sizes[i];
        gw.B = g;
        gw.sb0 = q->sizes[i + 1];
        gw.sb1 = 1;
        gw.M = q->sizes[i];
        gw.N = q->sizes[i + 1];
        gw.K = (int)n;
        gw.C32 = q->grad + q->woff[i];
        gw.ws = q->ws;
        gemm(gw, q->st, q->ws_floats);
        {   // db_i: row chunks into the workspace (free again once the dW product is done)
            const int cols = q->sizes[i + 1];
            const int chunks = (int)((n + kBiasRows - 1) / kBiasRows);
            float* part = q->ws_bias;
            hipLaunchKernelGGL(bias_grad_kernel, dim3(chunks, (cols + kThreads - 1) / kThreads), dim3(kThreads), 0,
                               q->st, g, (int)n, cols, part);
            hipLaunchKernelGGL(bias_grad_finish, dim3((cols + kThreads - 1) / kThreads), dim3(kThreads), 0, q->st,
                               part, chunks, cols, q->grad + q->boff[i]);
        }
        if (i > 0) {
            // dh_i = g W_i^T, then ReLU mask with z_{i-1}
            GemmArgs gh{};
            gh.A = g;
            gh.sa0 = q->sizes[i + 1];
            gh.sa1 = 1;
            gh.B = q->w16 + q->woff[i];
            gh.sb0 = 1;
            gh.sb1 = q->sizes[i + 1];
            gh.M = (int)n;
            gh.N = q->sizes[i];
            gh.K = q->sizes[i + 1];
            gh.C16 = other;
            gemm(gh, q->st);
            hipLaunchKernelGGL(relu_back_kernel, dim3(blocks_for(n * q->sizes[i])), dim3(kThreads), 0, q->st,
                               q->z32[i - 1], other, n * q->sizes[i]);
            std::swap(g, other);
        }
    }
    MLP_HIP(hipGetLastError());
    std::vector<double> part(nb);
    MLP_HIP(hipMemcpyAsync(part.data(), q->part, sizeof(double) * nb, hipMemcpyDeviceToHost, q->st));
    MLP_HIP(hipStreamSynchronize(q->st));
    double s = 0.0;
    for (double p : part) s += p;
    if (loss) *loss = (float)(0.5 * s / (double)nout);
    return HPR_OK;
}

int stage(hpr_mlp* q, const float* X, const float* T, int64_t n) {
    int rc = q->ensure_rows(n);
    if (rc) return rc;
    MLP_HIP(hipMemcpyAsync(q->xin, X, sizeof(float) * n * q->sizes[0], hipMemcpyHostToDevice, q->st));
    if (T) MLP_HIP(hipMemcpyAsync(q->tgt, T, sizeof(float) * n * q->sizes[q->L], hipMemcpyHostToDevice, q->st));
    return HPR_OK;
}

}  // namespace

extern "C" int hpr_mlp_create(int32_t nlayers, const int32_t* sizes, const float* params, void* stream,
                              hpr_mlp** out) {
    g_err.clear();
    if (!out) return fail(HPR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (nlayers < 1 || nlayers > kMaxLayers || !sizes) return fail(HPR_ERR_INVALID, "nlayers must be in [1, %d]", kMaxLayers);
    for (int i = 0; i <= nlayers; ++i)
        if (sizes[i] < 1 || sizes[i] > 4096) return fail(HPR_ERR_INVALID, "layer width %d out of [1, 4096]", sizes[i]);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(HPR_ERR_HIP, "hipGetDevice failed");
    void* scr = nullptr;
    const int src = scratch_address(dev, &scr);
    if (src) return src;
    hpr_mlp* q = new hpr_mlp();
    q->L = nlayers;
    q->scratch_dev = scr;
    int64_t off = 0;
    for (int i = 0; i <= nlayers; ++i) q->sizes[i] = sizes[i];
    for (int i = 0; i < nlayers; ++i) {
        q->woff[i] = off;
        off += (int64_t)sizes[i] * sizes[i + 1];
        q->boff[i] = off;
        off += sizes[i + 1];
    }
    q->nparams = off;
    auto bail = [&](int rc) {
        delete q;
        return rc;
    };
    if (stream) q->st = (hipStream_t)stream;
    else {
        if (hipStreamCreateWithFlags(&q->st, hipStreamNonBlocking) != hipSuccess) return bail(fail(HPR_ERR_HIP, "stream"));
        q->own_stream = true;
    }
    const size_t bytes = sizeof(float) * off;
    if (hipMalloc(&q->w, bytes) != hipSuccess || hipMalloc(&q->grad, bytes) != hipSuccess ||
        hipMalloc(&q->m, bytes) != hipSuccess || hipMalloc(&q->v, bytes) != hipSuccess ||
        hipMalloc(&q->w16, sizeof(uint16_t) * off) != hipSuccess)
        return bail(fail(HPR_ERR_NOMEM, "device allocation failed"));
    if (hipMemsetAsync(q->m, 0, bytes, q->st) != hipSuccess || hipMemsetAsync(q->v, 0, bytes, q->st) != hipSuccess ||
        hipMemsetAsync(q->w, 0, bytes, q->st) != hipSuccess)
        return bail(fail(HPR_ERR_HIP, "memset failed"));
    if (params && hipMemcpyAsync(q->w, params, bytes, hipMemcpyHostToDevice, q->st) != hipSuccess)
        return bail(fail(HPR_ERR_HIP, "copy failed"));
    int rc = refresh_bf16(q);
    if (rc) return bail(rc);
    if (hipStreamSynchronize(q->st) != hipSuccess) return bail(fail(HPR_ERR_HIP, "sync failed"));
    *out = q;
    return HPR_OK;
}

extern "C" int hpr_mlp_destroy(hpr_mlp* q) {
    delete q;
    return HPR_OK;
}

extern "C" int hpr_mlp_num_params(hpr_mlp* q, int64_t* n) {
    g_err.clear();
    if (!q || !n) return fail(HPR_ERR_INVALID, "NULL argument");
    *n = q->nparams;
    return HPR_OK;
}

extern "C" int hpr_mlp_set_params(hpr_mlp* q, const float* params) {
    g_err.clear();
    if (!q || !params) return fail(HPR_ERR_INVALID, "NULL argument");
    MLP_HIP(hipMemcpyAsync(q->w, params, sizeof(float) * q->nparams, hipMemcpyHostToDevice, q->st));
    MLP_HIP(hipMemsetAsync(q->m, 0, sizeof(float) * q->nparams, q->st));
    MLP_HIP(hipMemsetAsync(q->v, 0, sizeof(float) * q->nparams, q->st));
    q->step = 0;
    int rc = refresh_bf16(q);
    if (rc) return rc;
    MLP_HIP(hipStreamSynchronize(q->st));
    return HPR_OK;
}

extern "C" int hpr_mlp_get_params(hpr_mlp* q, float* params) {
    g_err.clear();
    if (!q || !params) return fail(HPR_ERR_INVALID, "NULL argument");
    MLP_HIP(hipMemcpyAsync(params, q->w, sizeof(float) * q->nparams, hipMemcpyDeviceToHost, q->st));
    MLP_HIP(hipStreamSynchronize(q->st));
    return HPR_OK;
}

extern "C" int hpr_mlp_forward(hpr_mlp* q, const float* X, int64_t n, float* Y) {
    g_err.clear();
    if (!q || !X || !Y || n < 0) return fail(HPR_ERR_INVALID, "bad argument");
    if (n == 0) return HPR_OK;
    int rc = stage(q, X, nullptr, n);
    if (rc) return rc;
    rc = forward_staged(q, n);
    if (rc) return rc;
    MLP_HIP(hipMemcpyAsync(Y, q->z32[q->L - 1], sizeof(float) * n * q->sizes[q->L], hipMemcpyDeviceToHost, q->st));
    MLP_HIP(hipStreamSynchronize(q->st));
    return HPR_OK;
}

// Rows per chunk of hpr_mlp_forward_device: the BF16 input row and two BF16 rows of the widest
// hidden layer (ping-pong) per row, in kScratchBytes, a multiple of the 16-row tile; 0 if even
// 16 rows do not fit.
static int64_t device_chunk_rows(const hpr_mlp* q, int64_t* in_bytes, int64_t* hid_bytes) {
    int hmax = 0;
    for (int i = 1; i < q->L; ++i) hmax = q->sizes[i] > hmax ? q->sizes[i] : hmax;
    const int64_t per_row = 2 * ((int64_t)q->sizes[0] + 2 * (int64_t)hmax) + 16;   // + alignment slack
    int64_t rows = (int64_t)(kScratchBytes - 3 * 256) / per_row;
    rows -= rows % kTile;
    *in_bytes = (2 * rows * q->sizes[0] + 255) / 256 * 256;
    *hid_bytes = (2 * rows * hmax + 255) / 256 * 256;
    return rows >= kTile ? rows : 0;
}

extern "C" int hpr_mlp_forward_device(hpr_mlp* q, const float* X, int64_t n, float* Y) {
    g_err.clear();
    if (!q || n < 0 || (n > 0 && (!X || !Y))) return fail(HPR_ERR_INVALID, "bad argument");
    if (n == 0) return HPR_OK;
    int64_t in_bytes = 0, hid_bytes = 0;
    const int64_t R = device_chunk_rows(q, &in_bytes, &hid_bytes);
    if (R == 0)
        return fail(HPR_ERR_INVALID, "layers too wide for the %zu-byte device scratch (16 rows of the input and two "
                    "hidden layers must fit)", kScratchBytes);
    unsigned char* base = static_cast<unsigned char*>(q->scratch_dev);
    uint16_t* x16 = reinterpret_cast<uint16_t*>(base);
    uint16_t* hbuf[2] = {reinterpret_cast<uint16_t*>(base + in_bytes),
                         reinterpret_cast<uint16_t*>(base + in_bytes + hid_bytes)};
    const int L = q->L;
    for (int64_t r0 = 0; r0 < n; r0 += R) {
        const int64_t rows = n - r0 < R ? n - r0 : R;
        hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(rows * q->sizes[0])), dim3(kThreads), 0, q->st,
                           X + r0 * q->sizes[0], x16, rows * q->sizes[0]);
        const uint16_t* h = x16;
        for (int i = 0; i < L; ++i) {
            GemmArgs g{};
            g.A = h;
            g.sa0 = q->sizes[i];
            g.sa1 = 1;
            g.B = q->w16 + q->woff[i];
            g.sb0 = q->sizes[i + 1];
            g.sb1 = 1;
            g.M = (int)rows;
            g.N = q->sizes[i + 1];
            g.K = q->sizes[i];
            g.bias = q->w + q->boff[i];
            g.relu = i < L - 1;
            g.C32 = i == L - 1 ? Y + r0 * q->sizes[L] : nullptr;
            g.C16 = i < L - 1 ? hbuf[i & 1] : nullptr;
            gemm(g, q->st);
            h = hbuf[i & 1];
        }
    }
    MLP_HIP(hipGetLastError());
    return HPR_OK;
}

extern "C" int hpr_mlp_gradients(hpr_mlp* q, const float* X, const float* T, int64_t n, float* grads, float* loss) {
    g_err.clear();
    if (!q || !X || !T || n < 1) return fail(HPR_ERR_INVALID, "bad argument");
    int rc = stage(q, X, T, n);
    if (rc) return rc;
    rc = gradients_staged(q, n, loss);
    if (rc) return rc;
    if (grads) {
        MLP_HIP(hipMemcpyAsync(grads, q->grad, sizeof(float) * q->nparams, hipMemcpyDeviceToHost, q->st));
        MLP_HIP(hipStreamSynchronize(q->st));
    }
    return HPR_OK;
}

extern "C" int hpr_mlp_train_step(hpr_mlp* q, const float* X, const float* T, int64_t n, float lr, float* loss) {
    g_err.clear();
    if (!q || !X || !T || n < 1 || !(lr > 0)) return fail(HPR_ERR_INVALID, "bad argument");
    int rc = stage(q, X, T, n);
    if (rc) return rc;
    rc = gradients_staged(q, n, loss);
    if (rc) return rc;
    q->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)q->step), c2 = 1.0f - powf(b2, (float)q->step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(q->nparams)), dim3(kThreads), 0, q->st, q->w, q->grad, q->m, q->v,
                       q->nparams, lr, b1, b2, 1e-8f, c1, c2);
    rc = refresh_bf16(q);
    if (rc) return rc;
    MLP_HIP(hipStreamSynchronize(q->st));
    return HPR_OK;
}

extern "C" const char* hpr_mlp_last_error(void) { return g_err.c_str(); }
