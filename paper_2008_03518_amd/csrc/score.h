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

// Commit validation of a finished OK trajectory (Sec. V: a plan enters the
// table only if it keeps R_sep from every plan it was planned against):
// each point as planned (FP64) must be at least R_sep from every visible
// entry of its row that the step scoring it counted, and clear of the
// terrain.  A point whose scored nearest-plan distance exceeds R_sep + 1 m
// cannot fail (the scored distance is within a small fraction of a
// millimetre of the exact one, and is exact near the well radius), so the
// exact check runs on the other points only.  Waves work independently:
// wave w takes points k0 + nw lane + w of each round of 64 nw points (so
// that the consecutive points of a close approach spread over the waves)
// and scans one flagged point's row at a time, four entries per lane and
// load, a box of half-width R_sep (widened by 0.1 % + 1 m + 1e-6 |point|,
// more than every FP32 rounding of the box test) picking the entries that
// get the exact FP64 test.  Returns this thread's finding (1: the plan
// fails); the caller reduces it over the workgroup.  Row bases are
// multiples of the table capacity, itself a multiple of four, so every
// four-entry group that starts below the count lies inside the row.
template <int NW>
__device__ int validate_points(const DevCfg &cfg, const DevTable &tb, const Traj &tr, size_t pt_base, int t0, int n,
                               int seq) {
    constexpr int U = 4;                                 // four-entry groups in flight per lane
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double r2 = cfg.R_sep * cfg.R_sep;
    const double clear2 = (cfg.R_sep + 1.0) * (cfg.R_sep + 1.0);
    int bad = 0;
    for (int k0 = 0; k0 < n; k0 += 64 * NW) {            // uniform
        const int k = k0 + NW * lane + wave;
        bool f = false;
        if (k < n) {
            const double *x = tr.xyz + (pt_base + k) * 3;
            if (tb.terr && x[2] - terrain_height(tb, x[0], x[1]) < 0.0) bad = 1;
            f = !(tr.nd[pt_base + k] > clear2);
        }
        uint64_t fb = __ballot(f);
        while (fb) {                                      // wave-uniform
            const int i = __builtin_ctzll(fb);
            fb &= fb - 1;
            const int kk = k0 + NW * i + wave;
            const double *x = tr.xyz + (pt_base + kk) * 3;
            const double px = x[0], py = x[1], pz = x[2];
            const int lim = tr.seen[pt_base + kk];
            const size_t rb = (size_t)(t0 + kk) * tb.cap;
            const float fx = (float)px, fy = (float)py;
            const float vb = (float)cfg.R_sep * 1.001f + 1.0f + 1e-6f * fmaxf(fabsf(fx), fabsf(fy));
            for (int j0 = 4 * lane; j0 < lim; j0 += 4 * 64 * U) {
                float4 X4[U], Y4[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = j0 + 4 * 64 * u;
                    if (j < lim) {
                        X4[u] = *reinterpret_cast<const float4 *>(tb.X + rb + j);
                        Y4[u] = *reinterpret_cast<const float4 *>(tb.Y + rb + j);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = j0 + 4 * 64 * u;
                    const float xs[4] = {X4[u].x, X4[u].y, X4[u].z, X4[u].w};
                    const float ys[4] = {Y4[u].x, Y4[u].y, Y4[u].z, Y4[u].w};
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const size_t idx = rb + j + m;
                        if (j + m < lim && fabsf(xs[m] - fx) <= vb && fabsf(ys[m] - fy) <= vb &&
                            entry_visible(tb, idx, seq) && entry_d2(px, py, pz, xs[m], ys[m], tb.Z[idx]) < r2)
                            bad = 1;
                    }
                }
            }
        }
    }
    return bad;
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
