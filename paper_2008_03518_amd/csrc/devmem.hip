// devmem.hip -- device memory helpers of the C ABI (allocation, copies, row
// gather) for callers that hold the proposal's training data on the GPU
// without an allocator of their own.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "fastmdp.h"

namespace {

// dst row i = src row idx[i] (zero when idx[i] is outside [0, n_src)); rows
// of `words` 32-bit words.
__global__ void gather_rows_kernel(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src, int64_t n_src,
                                   const int64_t *__restrict__ idx, int64_t n, int words) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * words) return;
    const int64_t i = t / words;
    const int w = (int)(t - i * words);
    const int64_t r = idx[i];
    dst[t] = (r >= 0 && r < n_src) ? src[r * words + w] : 0u;
}

int dev_err(const char *what, hipError_t e) {
    std::fprintf(stderr, "libfastmdp: %s: %s\n", what, hipGetErrorString(e));
    return FASTMDP_E_DEVICE;
}

}  // namespace

extern "C" {

int fastmdp_device_alloc(int64_t bytes, void **ptr) {
    if (!ptr || bytes <= 0) return FASTMDP_E_INVAL;
    *ptr = nullptr;
    if (hipMalloc(ptr, (size_t)bytes) != hipSuccess) {
        *ptr = nullptr;
        return FASTMDP_E_NOMEM;
    }
    return 0;
}

int fastmdp_device_free(void *ptr) {
    if (!ptr) return 0;
    const hipError_t e = hipFree(ptr);
    return e == hipSuccess ? 0 : dev_err("hipFree", e);
}

int fastmdp_copy_to_device(void *dst, const void *src, int64_t bytes) {
    if (!dst || !src || bytes < 0) return FASTMDP_E_INVAL;
    if (bytes == 0) return 0;
    const hipError_t e = hipMemcpy(dst, src, (size_t)bytes, hipMemcpyHostToDevice);
    return e == hipSuccess ? 0 : dev_err("hipMemcpy", e);
}

int fastmdp_copy_to_host(void *dst, const void *src, int64_t bytes) {
    if (!dst || !src || bytes < 0) return FASTMDP_E_INVAL;
    if (bytes == 0) return 0;
    const hipError_t e = hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost);
    return e == hipSuccess ? 0 : dev_err("hipMemcpy", e);
}

int fastmdp_gather_rows(void *dst, const void *src, int64_t n_src, const int64_t *idx, int64_t n,
                        int32_t row_bytes) {
    if (!dst || !src || !idx || n < 0 || n_src < 0 || row_bytes <= 0 || row_bytes % 4) return FASTMDP_E_INVAL;
    if (n == 0) return 0;
    const int words = row_bytes / 4;
    const int64_t total = n * words;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, 0,
                       static_cast<uint32_t *>(dst), static_cast<const uint32_t *>(src), n_src, idx, n, words);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e == hipSuccess ? 0 : dev_err("gather_rows", e);
}

}  // extern "C"
