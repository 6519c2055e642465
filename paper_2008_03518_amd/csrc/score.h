// score.h -- per-action scoring arithmetic and LDS / wavefront helpers
// shared by the planner kernels (internal).  One copy of the FP64 value of
// an action (goal peak, intruder and terrain wells, box mask), so that every
// planner variant produces the same values bit for bit.
#pragma once

#include "planner.h"
#include "wave.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace fmdp {

__device__ __forceinline__ bool outside_box(const DevCfg &c, double x, double y, double z) {
    return x < c.box_lo[0] || x > c.box_hi[0] || y < c.box_lo[1] || y > c.box_hi[1] ||
           z < c.box_lo[2] || z > c.box_hi[2];
}

// Terrain height: bilinear in the vertex grid, position clamped to the grid.
static __device__ double terrain_height(const DevTable &tb, double x, double y) {
    double fx = (x - tb.tx0) / tb.tcell;
    double fy = (y - tb.ty0) / tb.tcell;
    fx = fmin(fmax(fx, 0.0), (double)(tb.tnx - 1));
    fy = fmin(fmax(fy, 0.0), (double)(tb.tny - 1));
    int i = (int)floor(fx), j = (int)floor(fy);
    i = i > tb.tnx - 2 ? tb.tnx - 2 : i;
    j = j > tb.tny - 2 ? tb.tny - 2 : j;
    const double ax = fx - i, ay = fy - j;
    const float *h = tb.terr + (size_t)j * tb.tnx + i;
    const double h00 = h[0], h10 = h[1], h01 = h[tb.tnx], h11 = h[tb.tnx + 1];
    return (1.0 - ay) * ((1.0 - ax) * h00 + ax * h10) + ay * ((1.0 - ax) * h01 + ax * h11);
}

struct Scored {
    double x, y, z;     // successor
    double G, I, T, V;  // goal term, intruder well, terrain well, value
    double clr;         // terrain clearance (inf without terrain)
};

// Per-speed step length speed*dt and per-climb altitude change climb*dt
// (FP64), kept in LDS: indexed per lane, a lookup in the kernel-argument
// block would be a vector memory load.
struct ActTab {
    const double *step, *dz;
};

// Successor of state s under action a, whose heading has unit direction
// (dx, dy).
__device__ __forceinline__ void successor(const DevCfg &c, const ActTab &at, int a, const double s[3], double dx,
                                          double dy, double &x, double &y, double &z) {
    const int v = a % c.n_speed;
    const int cl = (a / c.n_speed) % c.n_climb;
    const double step = at.step[v];
    x = s[0] + step * dx;
    y = s[1] + step * dy;
    z = s[2] + at.dz[cl];
}

// Point w of the lookahead window: action a held for w steps.
__device__ __forceinline__ void window_point(const DevCfg &c, const ActTab &at, int a, int w, const double s[3],
                                             double dx, double dy, double &x, double &y, double &z) {
    const int v = a % c.n_speed;
    const int cl = (a / c.n_speed) % c.n_climb;
    const double k = (double)w;
    const double step = k * at.step[v];
    x = s[0] + step * dx;
    y = s[1] + step * dy;
    z = s[2] + k * at.dz[cl];
}

// Goal peak r_goal * gamma^(d/ell) at a successor.  Every action's value is
// at most this term (the penalties are non-negative), the bound the
// proposal certificate rests on; both use this one function.
__device__ __forceinline__ double goal_term(const DevCfg &c, double x, double y, double z, const double g[3]) {
    const double ex = g[0] - x, ey = g[1] - y, ez = g[2] - z;
    return c.abs_r_goal * exp(c.log_gamma * (sqrt(ex * ex + ey * ey + ez * ez) / c.ell));
}

// Squared distance from action a's successor to the nearest plan, from the
// sweep's minimum m of |q|^2 - 2 Delta . q over the staged plans.
template <int NC, int NV>
__device__ __forceinline__ double nearest_d2(const ActTab &at, int a, float m) {
    const double step = at.step[a % NV];
    const double dz = at.dz[(a / NV) % NC];
    return fma(dz, dz, fma(step, step, (double)m));
}

// Score action a from state s: dx, dy is its heading's unit direction and
// d2 the squared distance from the successor to the nearest plan.
static __device__ Scored score_action(const DevCfg &c, const DevTable &tb, const ActTab &at, int a, const double s[3],
                               const double g[3], double dx, double dy, double d2, int w = 0) {
    Scored r;
    if (w > 0)
        window_point(c, at, a, w, s, dx, dy, r.x, r.y, r.z);    // lookahead window point
    else
        successor(c, at, a, s, dx, dy, r.x, r.y, r.z);
    r.G = goal_term(c, r.x, r.y, r.z, g);
    r.I = 0.0;
    if (d2 < c.R_intr * c.R_intr) r.I = c.abs_r_intr * exp(c.log_gamma_intr * (sqrt(fmax(d2, 0.0)) / c.ell));
    r.T = 0.0;
    r.clr = INFINITY;
    if (tb.terr) {
        r.clr = r.z - terrain_height(tb, r.x, r.y);
        if (r.clr < c.R_terr) r.T = c.abs_r_terr * exp(c.log_gamma_terr * (fmax(r.clr, 0.0) / c.ell));
    }
    r.V = r.G - fmax(r.I, r.T);
    if (outside_box(c, r.x, r.y, r.z)) r.V = -INFINITY;
    return r;
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its outstanding global loads (a plain __syncthreads
// fence would also drain the prefetch of the next row).  Global data written
// in the step loop is read back only after a full __syncthreads.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ double wave_max(double v) { return wave_max_f64(v); }
__device__ __forceinline__ float wave_maxf(float v) { return wave_max_f32(v); }
__device__ __forceinline__ int wave_min(int v) { return wave_min_i32(v); }

constexpr int kCachePolicyDevice = 16;    // cache-policy bits of a device-coherent load (sc1)

// 16 bytes per lane from global memory straight into LDS (lane l's bytes
// land at lds + 16 l).  The host pass never sees the gfx950 form of the
// builtin: it rejects it, silently dropping every kernel that uses it.
__device__ __forceinline__ void load_lds16(const void *g, void *lds) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0);
#endif
}

}  // namespace fmdp
