// proposal.h -- device helpers of the learned action proposal: BF16
// conversion, the MFMA operand types, and the state features (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fastmdp.h"

namespace fmdp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSectors = 16;             // bearing sectors of the traffic features
constexpr float kFeatR = 600.0f;         // metres: plans nearer than this enter the features
constexpr int kFeatUsed = 76;            // features 76..95 are zero padding

// FP32 -> BF16, round to nearest even (finite inputs; NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// 16x16 output tile, K = 32 per instruction.  Operand lanes: A row and B
// column = lane % 16, eight consecutive k per lane group lane / 16 (both
// operands use the same k order, which is all the dot product needs); result
// element (i, j) = (4 * (lane / 16) + r, lane % 16) in register r.
__device__ __forceinline__ f32x4 mfma_bf16(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Traffic feature accumulators (LDS): per (sector, half) the largest
// closeness 1 - d/600 as FP32 bits (non-negative floats order like their
// bits) and the count; the number of plans within 600 m and the nearest
// distance (FP32 bits).
struct FeatAcc {
    unsigned near[2 * kSectors];
    int cnt[2 * kSectors];
    int n_close;
    unsigned dmin;
};

__device__ __forceinline__ void feat_reset(FeatAcc &f, int tid) {
    if (tid < 2 * kSectors) {
        f.near[tid] = 0u;
        f.cnt[tid] = 0;
    }
    if (tid == 0) {
        f.n_close = 0;
        f.dmin = __float_as_uint(kFeatR);
    }
}

// One plan at offset q = p - s (FP32; w = |q|^2 as staged), seen from a state
// whose horizontal unit vector to the goal is (ux, uy); up: q_z >= 0.
__device__ __forceinline__ void feat_point(FeatAcc &f, float qx, float qy, bool up, float w, float ux, float uy) {
    const float d = sqrtf(w);
    if (!(d < kFeatR)) return;
    const float along = qx * ux + qy * uy;
    const float cross = qy * ux - qx * uy;
    const float phi = atan2f(cross, along);
    int k = (int)floorf((phi + (float)M_PI) * (float)(kSectors / (2.0 * M_PI)));
    k = k < 0 ? 0 : (k > kSectors - 1 ? kSectors - 1 : k);
    const int idx = 2 * k + (up ? 0 : 1);
    atomicMax(&f.near[idx], __float_as_uint(1.0f - d / kFeatR));
    atomicAdd(&f.cnt[idx], 1);
    atomicAdd(&f.n_close, 1);
    atomicMin(&f.dmin, __float_as_uint(d));
}

// Feature i (0 <= i < FASTMDP_N_FEAT) from the accumulators, the state s and
// the goal g (FP64), the box and ell.
__device__ __forceinline__ float feat_value(const FeatAcc &f, int i, const double s[3], const double g[3],
                                            const double lo[3], const double hi[3], double ell) {
    if (i < 2 * kSectors) return __uint_as_float(f.near[i]);
    if (i < 4 * kSectors) return (float)min(f.cnt[i - 2 * kSectors], 4) * 0.25f;
    const double bx = g[0] - s[0], by = g[1] - s[1], bz = g[2] - s[2];
    const double rh = sqrt(bx * bx + by * by);
    const double d3 = sqrt(bx * bx + by * by + bz * bz);
    switch (i) {
        case 64: return (float)(rh / 10000.0);
        case 65: return (float)(bz / 500.0);
        case 66: return (float)(d3 / ell / 1000.0);
        case 67: return (float)(log1p(d3 / ell) / 8.0);
        case 68: return (float)(s[2] / 1000.0);
        case 69: return (float)((s[2] - lo[2]) / (hi[2] - lo[2]));
        case 70: return (float)((s[0] - lo[0]) / (hi[0] - lo[0]));
        case 71: return (float)((s[1] - lo[1]) / (hi[1] - lo[1]));
        case 72: return rh > 0.0 ? (float)(bx / rh) : 1.0f;
        case 73: return rh > 0.0 ? (float)(by / rh) : 0.0f;
        case 74: return fminf((float)f.n_close / 16.0f, 1.0f);
        case 75: return __uint_as_float(f.dmin) / kFeatR;
        default: return 0.0f;
    }
}

}  // namespace fmdp
