// wave.h -- wavefront (64-lane) reductions with DPP row operations (internal).
//
// Within each row of 16 lanes, quad_perm [1,0,3,2] and [2,3,0,1] combine
// lanes i and i^1, i^2; row_half_mirror pairs the two quads of each half
// row and row_mirror the two half rows, so four DPP steps leave every row
// holding its row's reduction; the four rows are then combined from lanes
// 0, 16, 32 and 48 with readlane.  Every lane of the wave must be active.
// These replace shuffle loops that go through the LDS crossbar once per step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmdp {

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const int lo = dpp_i32<CTRL>((int)(uint32_t)v);
    const int hi = dpp_i32<CTRL>((int)(uint32_t)(v >> 32));
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    return __longlong_as_double((long long)dpp_u64<CTRL>((uint64_t)__double_as_longlong(v)));
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

constexpr int kDppQuad1032 = 0xB1, kDppQuad2301 = 0x4E, kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;

__device__ __forceinline__ float wave_max_f32(float v) {
    v = fmaxf(v, dpp_f32<kDppQuad1032>(v));
    v = fmaxf(v, dpp_f32<kDppQuad2301>(v));
    v = fmaxf(v, dpp_f32<kDppRowHalfMirror>(v));
    v = fmaxf(v, dpp_f32<kDppRowMirror>(v));
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

__device__ __forceinline__ float wave_min_f32(float v) { return -wave_max_f32(-v); }

__device__ __forceinline__ int wave_min_i32(int v) {
    v = min(v, dpp_i32<kDppQuad1032>(v));
    v = min(v, dpp_i32<kDppQuad2301>(v));
    v = min(v, dpp_i32<kDppRowHalfMirror>(v));
    v = min(v, dpp_i32<kDppRowMirror>(v));
    const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}

__device__ __forceinline__ double wave_max_f64(double v) {
    v = fmax(v, dpp_f64<kDppQuad1032>(v));
    v = fmax(v, dpp_f64<kDppQuad2301>(v));
    v = fmax(v, dpp_f64<kDppRowHalfMirror>(v));
    v = fmax(v, dpp_f64<kDppRowMirror>(v));
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const double a = __longlong_as_double((long long)readlane_u64(u, 0));
    const double b = __longlong_as_double((long long)readlane_u64(u, 16));
    const double c = __longlong_as_double((long long)readlane_u64(u, 32));
    const double d = __longlong_as_double((long long)readlane_u64(u, 48));
    return fmax(fmax(a, b), fmax(c, d));
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    uint64_t o;
    o = dpp_u64<kDppQuad1032>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppQuad2301>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppRowHalfMirror>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppRowMirror>(v);
    v = o > v ? o : v;
    uint64_t a = readlane_u64(v, 0), b = readlane_u64(v, 16), c = readlane_u64(v, 32), d = readlane_u64(v, 48);
    a = b > a ? b : a;
    c = d > c ? d : c;
    return c > a ? c : a;
}

// Minimum over the wave of each of eight values per lane, all at once:
// swaps between the two 32-lane halves and then between 16-lane rows leave
// every lane with one of the values reduced over the four lanes of its
// position (value j + 2 r in row r, j = 0 or 1); a row mirror pairs the two
// halves of a row for j = 0 (lanes 0-7 of the row) and j = 1 (lanes 8-15),
// and three DPP steps finish within each half.  Lane l returns the minimum
// of value 2 (l / 16) + (l / 8) % 2.  Every lane of the wave must be active.
__device__ __forceinline__ float wave_min8_f32(const float v[8], int lane) {
    float w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 4]), false, false);
        w[j] = fminf(__uint_as_float(p[0]), __uint_as_float(p[1]));
    }
    float x[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(w[j]), __float_as_uint(w[j + 2]), false, false);
        x[j] = fminf(__uint_as_float(p[0]), __uint_as_float(p[1]));
    }
    const float m0 = fminf(x[0], dpp_f32<kDppRowMirror>(x[0]));
    const float m1 = fminf(x[1], dpp_f32<kDppRowMirror>(x[1]));
    float y = (lane & 8) ? m1 : m0;
    y = fminf(y, dpp_f32<kDppQuad1032>(y));
    y = fminf(y, dpp_f32<kDppQuad2301>(y));
    y = fminf(y, dpp_f32<kDppRowHalfMirror>(y));
    return y;
}

// Order-preserving map of a float to 32 bits (NaN ranks below -inf).
__device__ __forceinline__ uint32_t ordered_f32(float f) {
    if (f != f) return 0u;
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

}  // namespace fmdp
