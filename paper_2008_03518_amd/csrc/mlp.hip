// mlp.hip -- the proposal network's training and batch inference on gfx950:
// BF16 MFMA GEMMs with fused bias / ReLU / ReLU-derivative epilogues, the
// softmax cross-entropy, bias-gradient column sums and Adam on FP32 master
// weights.  The planner's in-loop inference (one state per workgroup) is in
// planner.hip and reads the BF16 weight copies kept here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "fastmdp.h"
#include "planner.h"
#include "proposal.h"

namespace fmdp {

// ---------------------------------------------------------------------------
// GEMM: C[m][n] = sum_k A(m,k) B(k,n), BF16 operands, FP32 accumulation.
//   A(m,k) = AK ? A[m*lda + k] : A[k*lda + m]
//   B(k,n) = BK ? B[n*ldb + k] : B[k*ldb + n]
// 64 x 64 output tile per 256-thread workgroup, each wave 32 x 32 (2 x 2
// MFMA 16x16x32 tiles); K in steps of 32 staged through LDS with k
// contiguous per row, so that every operand fetch is one 16-byte LDS read.
// Requirements: K % 32 == 0 and lda, ldb % 8 == 0 (checked); a k-major
// operand (AK or BK false) is read in 8-wide chunks, so it must be readable
// up to its M (or N) rounded up to 8 (every caller's buffers are padded to
// 32).
// ---------------------------------------------------------------------------
enum { EPI_F32 = 0, EPI_RELU_BF16 = 1, EPI_DRELU_BF16 = 2 };

struct GemmEpi {
    int mode;
    float *cf;            // EPI_F32 output
    uint16_t *cb;         // BF16 outputs
    int ldc;
    const float *bias;    // per column n, may be null (EPI_F32, EPI_RELU_BF16)
    const uint16_t *ref;  // EPI_DRELU_BF16: post-ReLU activation whose sign masks C
    int ldr;
};

constexpr int kGT = 64, kGK = 32, kGPad = 8;

template <bool AK, bool BK>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
                                                        const uint16_t *__restrict__ B, int ldb, GemmEpi e) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[kGT][kGK + kGPad];
    __shared__ __attribute__((aligned(16))) uint16_t sB[kGT][kGK + kGPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < K; k0 += kGK) {
        if (AK) {
            const int r = tid >> 2, kc = (tid & 3) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (m0 + r < M) v = *reinterpret_cast<const uint4 *>(A + (size_t)(m0 + r) * lda + k0 + kc);
            *reinterpret_cast<uint4 *>(&sA[r][kc]) = v;
        } else {
            const int kr = tid >> 3, mc = (tid & 7) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (m0 + mc < M) v = *reinterpret_cast<const uint4 *>(A + (size_t)(k0 + kr) * lda + m0 + mc);
            const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int i = 0; i < 8; ++i) sA[mc + i][kr] = h[i];
        }
        if (BK) {
            const int r = tid >> 2, kc = (tid & 3) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (n0 + r < N) v = *reinterpret_cast<const uint4 *>(B + (size_t)(n0 + r) * ldb + k0 + kc);
            *reinterpret_cast<uint4 *>(&sB[r][kc]) = v;
        } else {
            const int kr = tid >> 3, nc = (tid & 7) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (n0 + nc < N) v = *reinterpret_cast<const uint4 *>(B + (size_t)(k0 + kr) * ldb + n0 + nc);
            const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int i = 0; i < 8; ++i) sB[nc + i][kr] = h[i];
        }
        __syncthreads();
        uint4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const uint4 *>(&sA[wm + i * 16 + (lane & 15)][(lane >> 4) * 8]);
            b[i] = *reinterpret_cast<const uint4 *>(&sB[wn + i * 16 + (lane & 15)][(lane >> 4) * 8]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= M || n >= N) continue;
                float v = acc[i][j][r];
                const size_t o = (size_t)m * e.ldc + n;
                if (e.mode == EPI_F32) {
                    e.cf[o] = v + (e.bias ? e.bias[n] : 0.0f);
                } else if (e.mode == EPI_RELU_BF16) {
                    e.cb[o] = f2bf(fmaxf(v + (e.bias ? e.bias[n] : 0.0f), 0.0f));
                } else {
                    e.cb[o] = f2bf(bf2f(e.ref[(size_t)m * e.ldr + n]) > 0.0f ? v : 0.0f);
                }
            }
}

// FP32 -> BF16 copy of n elements.
__global__ void to_bf16_kernel(const float *__restrict__ x, uint16_t *__restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// Softmax cross-entropy, one wave per row: loss row = logsumexp - logit[y];
// d[row][o] = (softmax_o - [o == y]) / batch for o < n_out, 0 up to ldd.
__global__ __launch_bounds__(256) void softmax_ce_kernel(int batch, int n_out, const float *__restrict__ logits,
                                                         const int *__restrict__ y, uint16_t *__restrict__ d, int ldd,
                                                         float *__restrict__ loss_row) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= batch) return;
    const float *l = logits + (size_t)row * n_out;
    float mx = -INFINITY;
    for (int o = lane; o < n_out; o += 64) mx = fmaxf(mx, l[o]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    float sum = 0.0f;
    for (int o = lane; o < n_out; o += 64) sum += expf(l[o] - mx);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    const int lab = y[row];
    const bool valid = lab >= 0 && lab < n_out;           // an invalid label: NaN loss, no gradient
    const float inv_b = 1.0f / (float)batch;
    for (int o = lane; o < ldd; o += 64) {
        float g = 0.0f;
        if (valid && o < n_out) g = (expf(l[o] - mx) / sum - (o == lab ? 1.0f : 0.0f)) * inv_b;
        d[(size_t)row * ldd + o] = f2bf(g);
    }
    if (lane == 0) loss_row[row] = valid ? mx + logf(sum) - l[lab] : NAN;
}

// out[n] = sum over rows m < rows of x[m*ld + n], n < cols (FP32 sums of BF16).
__global__ void colsum_bf16_kernel(int rows, int cols, const uint16_t *__restrict__ x, int ld, float *__restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float s = 0.0f;
    for (int m = 0; m < rows; ++m) s += bf2f(x[(size_t)m * ld + n]);
    out[n] = s;
}

// Sum of n FP32 values into out[0] (one workgroup, fixed order per thread).
__global__ __launch_bounds__(256) void sum_kernel(const float *__restrict__ x, int n, float *__restrict__ out) {
    __shared__ float part[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

// Adam with bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr * (m / c1) / (sqrt(v / c2) + eps), with c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace fmdp

using namespace fmdp;

struct fastmdp_mlp {
    int n_in = 0, n_hid = 0, n_out = 0, n_pad = 0, max_batch = 0;
    long long n_par = 0;
    long long o_W1 = 0, o_b1 = 0, o_W2 = 0, o_b2 = 0, o_W3 = 0, o_b3 = 0;
    float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;   // packed FP32
    uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;         // BF16 [out][in]; W3b has n_pad rows
    uint16_t *X16 = nullptr, *H1 = nullptr, *H2 = nullptr, *D3 = nullptr, *DZ2 = nullptr, *DZ1 = nullptr;
    float *Z3 = nullptr, *loss_row = nullptr, *loss = nullptr;
    int t = 0;                                                       // Adam steps taken
    hipStream_t own = nullptr, stream = nullptr;
};

namespace {

#define MLP_TRY(x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) {                                                                     \
            std::fprintf(stderr, "libfastmdp: %s failed: %s\n", #x, hipGetErrorString(e_));         \
            return FASTMDP_E_DEVICE;                                                                \
        }                                                                                           \
    } while (0)

template <class T>
int alloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) return 0;
    if (hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return FASTMDP_E_NOMEM;
    }
    return 0;
}

void mlp_free(fastmdp_mlp *m) {
    hipFree(m->P); hipFree(m->G); hipFree(m->Mm); hipFree(m->Vv);
    hipFree(m->W1b); hipFree(m->W2b); hipFree(m->W3b);
    hipFree(m->X16); hipFree(m->H1); hipFree(m->H2); hipFree(m->D3); hipFree(m->DZ2); hipFree(m->DZ1);
    hipFree(m->Z3); hipFree(m->loss_row); hipFree(m->loss);
    if (m->own) hipStreamDestroy(m->own);
}

hipError_t gemm(hipStream_t st, bool ak, bool bk, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B,
                int ldb, const GemmEpi &e) {
    if (K % kGK || lda % 8 || ldb % 8) return hipErrorInvalidValue;
    const dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
    if (ak && bk) hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e);
    else if (ak) hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e);
    else if (bk) hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e);
    else hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e);
    return hipGetLastError();
}

GemmEpi epi_f32(float *c, int ldc, const float *bias) { return GemmEpi{EPI_F32, c, nullptr, ldc, bias, nullptr, 0}; }
GemmEpi epi_relu(uint16_t *c, int ldc, const float *bias) {
    return GemmEpi{EPI_RELU_BF16, nullptr, c, ldc, bias, nullptr, 0};
}
GemmEpi epi_drelu(uint16_t *c, int ldc, const uint16_t *ref, int ldr) {
    return GemmEpi{EPI_DRELU_BF16, nullptr, c, ldc, nullptr, ref, ldr};
}

hipError_t to_bf16(hipStream_t st, const float *x, uint16_t *y, long long n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

// BF16 copies of the weights from the FP32 master parameters.
hipError_t refresh_bf16(fastmdp_mlp *m) {
    hipError_t e = to_bf16(m->stream, m->P + m->o_W1, m->W1b, (long long)m->n_hid * m->n_in);
    if (e == hipSuccess) e = to_bf16(m->stream, m->P + m->o_W2, m->W2b, (long long)m->n_hid * m->n_hid);
    if (e == hipSuccess) e = to_bf16(m->stream, m->P + m->o_W3, m->W3b, (long long)m->n_out * m->n_hid);
    return e;
}

// Forward pass of a batch already in X16: H1, H2 (BF16) and logits into
// `logits` ([batch][n_out] FP32).
hipError_t forward(fastmdp_mlp *m, int batch, float *logits) {
    hipStream_t st = m->stream;
    hipError_t e = gemm(st, true, true, batch, m->n_hid, m->n_in, m->X16, m->n_in, m->W1b, m->n_in,
                        epi_relu(m->H1, m->n_hid, m->P + m->o_b1));
    if (e == hipSuccess)
        e = gemm(st, true, true, batch, m->n_hid, m->n_hid, m->H1, m->n_hid, m->W2b, m->n_hid,
                 epi_relu(m->H2, m->n_hid, m->P + m->o_b2));
    if (e == hipSuccess)
        e = gemm(st, true, true, batch, m->n_out, m->n_hid, m->H2, m->n_hid, m->W3b, m->n_hid,
                 epi_f32(logits, m->n_out, m->P + m->o_b3));
    return e;
}

// Loss and gradient of a batch (x FP32 device, y device) into m->G and
// m->loss[0] (mean).
hipError_t loss_and_grad(fastmdp_mlp *m, int batch, const float *x, const int *y) {
    hipStream_t st = m->stream;
    const int nh = m->n_hid, ni = m->n_in, no = m->n_out, np = m->n_pad;
    hipError_t e = to_bf16(st, x, m->X16, (long long)batch * ni);
    if (e == hipSuccess) e = forward(m, batch, m->Z3);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(softmax_ce_kernel, dim3((batch + 3) / 4), dim3(256), 0, st, batch, no, m->Z3, y, m->D3, np,
                       m->loss_row);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, m->loss_row, batch, m->loss);
    e = hipGetLastError();
    float *G = m->G;
    // layer 3: gW3 = D3^T H2, gb3 = column sums of D3, dZ2 = (D3 W3) * [H2 > 0]
    if (e == hipSuccess) e = gemm(st, false, false, no, nh, batch, m->D3, np, m->H2, nh, epi_f32(G + m->o_W3, nh, nullptr));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(colsum_bf16_kernel, dim3((no + 255) / 256), dim3(256), 0, st, batch, no, m->D3, np, G + m->o_b3);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = gemm(st, true, false, batch, nh, np, m->D3, np, m->W3b, nh, epi_drelu(m->DZ2, nh, m->H2, nh));
    // layer 2
    if (e == hipSuccess) e = gemm(st, false, false, nh, nh, batch, m->DZ2, nh, m->H1, nh, epi_f32(G + m->o_W2, nh, nullptr));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(colsum_bf16_kernel, dim3((nh + 255) / 256), dim3(256), 0, st, batch, nh, m->DZ2, nh, G + m->o_b2);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = gemm(st, true, false, batch, nh, nh, m->DZ2, nh, m->W2b, nh, epi_drelu(m->DZ1, nh, m->H1, nh));
    // layer 1
    if (e == hipSuccess) e = gemm(st, false, false, nh, ni, batch, m->DZ1, nh, m->X16, ni, epi_f32(G + m->o_W1, ni, nullptr));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(colsum_bf16_kernel, dim3((nh + 255) / 256), dim3(256), 0, st, batch, nh, m->DZ1, nh, G + m->o_b1);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

namespace fmdp {
// Weights of a network for the planner's inference (internal accessor).
int mlp_weights(const fastmdp_mlp *m, PropNet *w) {
    if (!m || !w) return FASTMDP_E_INVAL;
    w->W1 = m->W1b; w->W2 = m->W2b; w->W3 = m->W3b;
    w->b1 = m->P + m->o_b1; w->b2 = m->P + m->o_b2; w->b3 = m->P + m->o_b3;
    w->n_in = m->n_in; w->n_hid = m->n_hid; w->n_out = m->n_out;
    return 0;
}
}  // namespace fmdp

extern "C" {

int fastmdp_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, fastmdp_mlp **out) {
    if (!out || n_in < 32 || n_in % 32 || n_hidden < 32 || n_hidden % 32 || n_out < 1 || max_batch < 1)
        return FASTMDP_E_INVAL;
    fastmdp_mlp *m = new (std::nothrow) fastmdp_mlp();
    if (!m) return FASTMDP_E_NOMEM;
    m->n_in = n_in; m->n_hid = n_hidden; m->n_out = n_out;
    m->n_pad = (n_out + 31) / 32 * 32;
    m->max_batch = (max_batch + 31) / 32 * 32;
    m->o_W1 = 0;
    m->o_b1 = m->o_W1 + (long long)n_hidden * n_in;
    m->o_W2 = m->o_b1 + n_hidden;
    m->o_b2 = m->o_W2 + (long long)n_hidden * n_hidden;
    m->o_W3 = m->o_b2 + n_hidden;
    m->o_b3 = m->o_W3 + (long long)n_out * n_hidden;
    m->n_par = m->o_b3 + n_out;
    const size_t B = (size_t)m->max_batch;
    int rc = 0;
    rc = rc ? rc : alloc(&m->P, (size_t)m->n_par);
    rc = rc ? rc : alloc(&m->G, (size_t)m->n_par);
    rc = rc ? rc : alloc(&m->Mm, (size_t)m->n_par);
    rc = rc ? rc : alloc(&m->Vv, (size_t)m->n_par);
    rc = rc ? rc : alloc(&m->W1b, (size_t)n_hidden * n_in);
    rc = rc ? rc : alloc(&m->W2b, (size_t)n_hidden * n_hidden);
    rc = rc ? rc : alloc(&m->W3b, (size_t)m->n_pad * n_hidden);
    rc = rc ? rc : alloc(&m->X16, B * n_in);
    rc = rc ? rc : alloc(&m->H1, B * n_hidden);
    rc = rc ? rc : alloc(&m->H2, B * n_hidden);
    rc = rc ? rc : alloc(&m->D3, B * m->n_pad);
    rc = rc ? rc : alloc(&m->DZ2, B * n_hidden);
    rc = rc ? rc : alloc(&m->DZ1, B * n_hidden);
    rc = rc ? rc : alloc(&m->Z3, B * n_out);
    rc = rc ? rc : alloc(&m->loss_row, B);
    rc = rc ? rc : alloc(&m->loss, (size_t)1);
    if (!rc && hipStreamCreate(&m->own) != hipSuccess) rc = FASTMDP_E_DEVICE;
    if (!rc) {
        m->stream = m->own;
        const size_t np = (size_t)m->n_par * sizeof(float);
        if (hipMemsetAsync(m->P, 0, np, m->stream) != hipSuccess ||
            hipMemsetAsync(m->Mm, 0, np, m->stream) != hipSuccess ||
            hipMemsetAsync(m->Vv, 0, np, m->stream) != hipSuccess ||
            hipMemsetAsync(m->W3b, 0, (size_t)m->n_pad * n_hidden * sizeof(uint16_t), m->stream) != hipSuccess ||
            refresh_bf16(m) != hipSuccess || hipStreamSynchronize(m->stream) != hipSuccess)
            rc = FASTMDP_E_DEVICE;
    }
    if (rc) {
        mlp_free(m);
        delete m;
        return rc;
    }
    *out = m;
    return 0;
}

void fastmdp_mlp_destroy(fastmdp_mlp *net) {
    if (!net) return;
    hipStreamSynchronize(net->stream);
    mlp_free(net);
    delete net;
}

int64_t fastmdp_mlp_num_params(const fastmdp_mlp *net) { return net ? net->n_par : FASTMDP_E_INVAL; }

int fastmdp_mlp_set_params(fastmdp_mlp *m, const float *params) {
    if (!m || !params) return FASTMDP_E_INVAL;
    const size_t np = (size_t)m->n_par * sizeof(float);
    MLP_TRY(hipMemcpyAsync(m->P, params, np, hipMemcpyHostToDevice, m->stream));
    MLP_TRY(hipMemsetAsync(m->Mm, 0, np, m->stream));
    MLP_TRY(hipMemsetAsync(m->Vv, 0, np, m->stream));
    MLP_TRY(refresh_bf16(m));
    MLP_TRY(hipStreamSynchronize(m->stream));
    m->t = 0;
    return 0;
}

int fastmdp_mlp_get_params(fastmdp_mlp *m, float *params) {
    if (!m || !params) return FASTMDP_E_INVAL;
    MLP_TRY(hipMemcpyAsync(params, m->P, (size_t)m->n_par * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    return 0;
}

int fastmdp_mlp_forward(fastmdp_mlp *m, int32_t batch, const float *x, float *logits) {
    if (!m || !x || !logits || batch < 1 || batch > m->max_batch) return FASTMDP_E_INVAL;
    MLP_TRY(to_bf16(m->stream, x, m->X16, (long long)batch * m->n_in));
    MLP_TRY(forward(m, batch, logits));
    MLP_TRY(hipStreamSynchronize(m->stream));
    return 0;
}

int fastmdp_mlp_gradient(fastmdp_mlp *m, int32_t batch, const float *x, const int32_t *y, float *grads, float *loss) {
    if (!m || !x || !y || !grads || batch < 32 || batch % 32 || batch > m->max_batch) return FASTMDP_E_INVAL;
    MLP_TRY(loss_and_grad(m, batch, x, y));
    MLP_TRY(hipMemcpyAsync(grads, m->G, (size_t)m->n_par * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    float l = 0.0f;
    MLP_TRY(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    if (loss) *loss = l / (float)batch;
    return 0;
}

int fastmdp_mlp_train_step(fastmdp_mlp *m, int32_t batch, const float *x, const int32_t *y, float lr, float *loss) {
    if (!m || !x || !y || batch < 32 || batch % 32 || batch > m->max_batch || !(lr > 0.0f)) return FASTMDP_E_INVAL;
    MLP_TRY(loss_and_grad(m, batch, x, y));
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, m->t)), c2 = (float)(1.0 - std::pow(0.999, m->t));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((m->n_par + 255) / 256)), dim3(256), 0, m->stream, m->P, m->G,
                       m->Mm, m->Vv, m->n_par, lr, b1, b2, 1e-8f, c1, c2);
    MLP_TRY(hipGetLastError());
    MLP_TRY(refresh_bf16(m));
    float l = 0.0f;
    if (loss) MLP_TRY(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    if (loss) *loss = l / (float)batch;
    return 0;
}

}  // extern "C"
