// planner.hip -- device code of the FastMDP first-come-first-served planner
// for gfx950 (MI355X).
//
// One workgroup plans one request ("slot"), persistent over time steps.  Per
// step (the kernel pipeline of Sec. IV fused into one workgroup):
//   1. bearing to the goal and the per-heading direction cosines (FP64);
//   2. the known-plan table row of the successor's time is staged from HBM
//      into LDS in tiles, each plan as (q_x, q_y, -2 dt q_z, |q|^2) with
//      q = p - s relative to the current state (FP64 subtraction, FP32 store);
//   3. the intruder sweep (the "Process negative intruder rewards" kernel):
//      every lane owns one heading and all climb x speed actions of it and a
//      slice of the staged plans, and keeps, per action, the minimum over
//      plans of |q - Delta_a|^2 - |Delta_a|^2 = |q|^2 - 2 Delta_a . q.
//      Because gamma^d falls with d, the largest risk-well penalty over the
//      plans is the one of the nearest plan, so the per-peak maximum of the
//      paper is this minimum followed by one well evaluation per action;
//   4. per action (FP64): goal peak, intruder well from the nearest plan,
//      terrain clearance well, value = goal - max(penalties), box mask
//      (kernels "Process positive rewards", "Process negative terrain
//      rewards", "Compute value");
//   5. argmax by wavefront shuffle reductions ("Select best action");
//   6. state advance, goal capture, collision checks and trajectory append
//      ("Determine terminal state").
#include "planner.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fmdp {

__device__ __forceinline__ bool outside_box(const DevCfg &c, double x, double y, double z) {
    return x < c.box_lo[0] || x > c.box_hi[0] || y < c.box_lo[1] || y > c.box_hi[1] ||
           z < c.box_lo[2] || z > c.box_hi[2];
}

// Terrain height: bilinear in the vertex grid, position clamped to the grid.
__device__ double terrain_height(const DevTable &tb, double x, double y) {
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

// Score action a from state s: dx, dy is its heading's unit direction and
// d2 the squared distance from the successor to the nearest plan.
__device__ Scored score_action(const DevCfg &c, const DevTable &tb, int a, const double s[3], const double g[3],
                               double dx, double dy, double d2) {
    Scored r;
    const int v = a % c.n_speed;
    const int cl = (a / c.n_speed) % c.n_climb;
    const double step = c.speed[v] * c.dt;
    r.x = s[0] + step * dx;
    r.y = s[1] + step * dy;
    r.z = s[2] + c.climb[cl] * c.dt;
    const double ex = g[0] - r.x, ey = g[1] - r.y, ez = g[2] - r.z;
    r.G = c.abs_r_goal * exp(c.log_gamma * (sqrt(ex * ex + ey * ey + ez * ez) / c.ell));
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

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

template <int NT>
struct PlanGeom {
    static constexpr int NW = NT / 64;
    static constexpr int TILE = NT >= 1024 ? 4096 : 2048;   // plans staged per LDS tile
    static constexpr int PRE = TILE / NT;                    // row entries prefetched per thread
};

template <int NT, int NC, int NV, int ZC>
__global__ __launch_bounds__(NT) void planner_kernel(DevCfg cfg, DevTable tb, Slot *slots, const int *slot_list,
                                                     Traj tr, int budget, int validate, EvalOut ev) {
    using Geo = PlanGeom<NT>;
    constexpr int NW = Geo::NW, TILE = Geo::TILE, PRE = Geo::PRE;
    __shared__ float4 tile[TILE];               // staged plans; reused for the slice partial minima
    __shared__ double sV[kMaxActions];
    __shared__ double sD2[kMaxActions];         // squared nearest-plan distance per action
    __shared__ double sC0[kMaxHeads], sS0[kMaxHeads];    // cos, sin of the heading offsets 2*pi*h/H
    __shared__ double sCos[kMaxHeads], sSin[kMaxHeads];  // heading directions of the current step
    __shared__ unsigned sBand[kMaxActions / 32];
    __shared__ double st_s[3];
    __shared__ int st_n, st_status, st_flag;
    __shared__ double red_d[NW];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int slot = slot_list ? slot_list[blockIdx.x] : (int)blockIdx.x;
    Slot &S = slots[slot];
    const bool eval = ev.V != nullptr || ev.best != nullptr;

    const int H = cfg.n_head, A = cfg.n_actions;
    const int n_slices = NT / H;
    const int my_h = tid % H, my_slice = tid / H;
    const bool sweeper = tid < n_slices * H;
    const int tcap = (TILE / (2 * n_slices)) * (2 * n_slices);   // whole sweep rounds per tile
    // slice partial minima: per wave after a shuffle reduction when a wave
    // holds several lanes of one heading (H <= 64), else per slice
    const int n_part = H <= 64 ? NW : n_slices;

    const double g[3] = {S.goal[0], S.goal[1], S.goal[2]};
    const int t0 = S.t0;
    const size_t pt_base = (size_t)slot * tr.stride;

    for (int h = tid; h < H; h += NT) {
        const double th = 2.0 * M_PI * (double)h / (double)H;
        sC0[h] = cos(th);
        sS0[h] = sin(th);
    }
    if (tid == 0) {
        const int n = eval ? 0 : S.n_points;
        if (n == 0) {
            st_s[0] = S.origin[0]; st_s[1] = S.origin[1]; st_s[2] = S.origin[2];
        } else {
            const double *p = tr.xyz + (pt_base + n - 1) * 3;
            st_s[0] = p[0]; st_s[1] = p[1]; st_s[2] = p[2];
        }
        st_n = n;
        st_status = kRunning;
        st_flag = 0;
    }
    __syncthreads();

    // Origin check of a fresh request: inside the box, clear of terrain, and
    // no plan active at the departure row closer than R_sep.
    if (!eval && st_n == 0) {
        const double o[3] = {st_s[0], st_s[1], st_s[2]};
        const int n_row = t0 < tb.rows ? tb.rowN[t0] : 0;
        const size_t rb = (size_t)t0 * tb.cap;
        int hit = 0;
        for (int j = tid; j < n_row; j += NT)
            if (entry_d2(o[0], o[1], o[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < cfg.R_sep * cfg.R_sep) hit = 1;
        if (hit) st_flag = 1;        // benign race: every writer stores 1
        __syncthreads();
        if (tid == 0) {
            bool blocked = st_flag != 0 || outside_box(cfg, o[0], o[1], o[2]);
            if (tb.terr && o[2] - terrain_height(tb, o[0], o[1]) < 0.0) blocked = true;
            double *p = tr.xyz + pt_base * 3;
            p[0] = o[0]; p[1] = o[1]; p[2] = o[2];
            tr.act[pt_base] = -1;
            tr.val[pt_base] = 0.0;
            tr.seen[pt_base] = n_row;
            tr.top[pt_base] = -1;
            st_n = 1;
            if (blocked) st_status = FASTMDP_REJECT_ORIGIN;
        }
        __syncthreads();
    }

    // per-lane sweep constants
    float kv[NV], clf[NC];
#pragma unroll
    for (int v = 0; v < NV; ++v) kv[v] = cfg.kv[v];
#pragma unroll
    for (int c = 0; c < NC; ++c) clf[c] = cfg.climb_f[c];

    // first tile of the next row, prefetched into registers
    float px[PRE], py[PRE], pz[PRE];
    int pre_n = 0;
    auto prefetch = [&](int row) {
        pre_n = (row >= 0 && row < tb.rows) ? tb.rowN[row] : 0;
        const size_t rb = (size_t)(row < 0 ? 0 : row) * tb.cap;
        const int lim = min(pre_n, tcap);
#pragma unroll
        for (int i = 0; i < PRE; ++i) {
            const int j = tid + i * NT;
            if (j < lim) {
                px[i] = tb.X[rb + j];
                py[i] = tb.Y[rb + j];
                pz[i] = tb.Z[rb + j];
            }
        }
    };
    prefetch((eval ? t0 : t0 + st_n - 1) + 1);

    long long pairs = 0;
    int steps_here = 0;

    for (;;) {
        if (st_status != kRunning) break;                 // uniform (LDS, after a barrier)
        const int n = st_n;
        const int k = eval ? 0 : n - 1;                    // steps taken so far
        const int t = eval ? t0 : t0 + k;
        const double s[3] = {st_s[0], st_s[1], st_s[2]};
        if (!eval) {
            const double ex = g[0] - s[0], ey = g[1] - s[1], ez = g[2] - s[2];
            if (sqrt(ex * ex + ey * ey + ez * ez) <= cfg.ell) {
                __syncthreads();
                if (tid == 0) st_status = FASTMDP_OK;
                break;
            }
            if (k >= cfg.max_steps) {
                __syncthreads();
                if (tid == 0) st_status = FASTMDP_TIMEOUT;
                break;
            }
            if (steps_here >= budget) break;               // resumable: stays running
        }

        // 1. heading directions: the goal bearing rotated by each offset
        {
            const double bx = g[0] - s[0], by = g[1] - s[1];
            const double r = sqrt(bx * bx + by * by);
            const double cb = r > 0.0 ? bx / r : 1.0, sb = r > 0.0 ? by / r : 0.0;
            for (int h = tid; h < H; h += NT) {
                sCos[h] = cb * sC0[h] - sb * sS0[h];
                sSin[h] = sb * sC0[h] + cb * sS0[h];
            }
        }
        const int row = t + 1;
        const int n_row = pre_n;
        const size_t rb = (size_t)row * tb.cap;

        // 2. stage the first tile from the prefetched registers
        {
            const int nt = min(tcap, n_row);
            const int npad = ((nt + 2 * n_slices - 1) / (2 * n_slices)) * (2 * n_slices);
#pragma unroll
            for (int i = 0; i < PRE; ++i) {
                const int j = tid + i * NT;
                if (j < npad) {
                    float4 e = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                    if (j < nt) {
                        const float qx = (float)((double)px[i] - s[0]);
                        const float qy = (float)((double)py[i] - s[1]);
                        const float qz = (float)((double)pz[i] - s[2]);
                        e = make_float4(qx, qy, cfg.zeta_scale * qz, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
                    }
                    tile[j] = e;
                }
            }
        }
        __syncthreads();

        float ch = 0.0f, sh = 0.0f;
        if (sweeper) {
            ch = (float)sCos[my_h];
            sh = (float)sSin[my_h];
        }
        float acc[NC][NV];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[c][v] = INFINITY;

        // 3. sweep: every lane, one heading's climb x speed actions over a
        //    slice of the staged plans (two plans per round: v_min3)
        for (int base = 0; base < n_row; base += tcap) {
            const int nt = min(tcap, n_row - base);
            const int npad = ((nt + 2 * n_slices - 1) / (2 * n_slices)) * (2 * n_slices);
            if (base > 0) {
                __syncthreads();                           // previous tile fully swept
                for (int j = tid; j < npad; j += NT) {
                    float4 e = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                    if (j < nt) {
                        const size_t idx = rb + base + j;
                        const float qx = (float)((double)tb.X[idx] - s[0]);
                        const float qy = (float)((double)tb.Y[idx] - s[1]);
                        const float qz = (float)((double)tb.Z[idx] - s[2]);
                        e = make_float4(qx, qy, cfg.zeta_scale * qz, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
                    }
                    tile[j] = e;
                }
                __syncthreads();
            }
            if (sweeper) {
                for (int i = my_slice; i < npad; i += 2 * n_slices) {
                    const float4 p0 = tile[i];
                    const float4 p1 = tile[i + n_slices];
                    const float hq0 = fmaf(p0.x, ch, p0.y * sh);
                    const float hq1 = fmaf(p1.x, ch, p1.y * sh);
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const float u0 = fmaf(kv[v], hq0, p0.w);
                        const float u1 = fmaf(kv[v], hq1, p1.w);
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const float a0 = (c == ZC) ? u0 : fmaf(clf[c], p0.z, u0);
                            const float a1 = (c == ZC) ? u1 : fmaf(clf[c], p1.z, u1);
                            acc[c][v] = fminf(acc[c][v], fminf(a0, a1));
                        }
                    }
                }
            }
        }
        __syncthreads();                                   // tile is reused below

        // slice partial minima
        float *red = reinterpret_cast<float *>(tile);
        if (H <= 64) {
            // lanes l, l+H, l+2H, ... of a wave own the same heading
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    float m = acc[c][v];
                    for (int off = H; off < 64; off += H) {
                        const int src = lane + off < 64 ? lane + off : lane;
                        m = fminf(m, __shfl(m, src));
                    }
                    acc[c][v] = m;
                }
            if (lane < H) {
                const int h = (wave * 64 + lane) % H;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int v = 0; v < NV; ++v) red[wave * A + (h * NC + c) * NV + v] = acc[c][v];
            }
        } else if (sweeper) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) red[my_slice * A + (my_h * NC + c) * NV + v] = acc[c][v];
        }
        for (int w = tid; w < kMaxActions / 32; w += NT) sBand[w] = 0u;
        __syncthreads();

        // 4. per-action value.  The nearest-plan squared distance is
        //    m + |Delta|^2 with m from the FP32 sweep; actions whose distance
        //    lands within kBand of the well radius are flagged for an exact
        //    FP64 recomputation so that well membership is decided in FP64.
        int band = 0;
        for (int a = tid; a < A; a += NT) {
            float m = INFINITY;
            for (int q = 0; q < n_part; ++q) m = fminf(m, red[q * A + a]);
            const int h = a / (NC * NV);
            const double dx = sCos[h], dy = sSin[h];
            const double step = cfg.speed[a % NV] * cfg.dt;
            const double dz = cfg.climb[(a / NV) % NC] * cfg.dt;
            const double d2 = (double)m + step * step + dz * dz;
            sV[a] = score_action(cfg, tb, a, s, g, dx, dy, d2).V;
            sD2[a] = d2;
            if (fabs(sqrt(fmax(d2, 0.0)) - cfg.R_intr) < kBand) {
                atomicOr(&sBand[a >> 5], 1u << (a & 31));
                band = 1;
            }
        }
        if (__syncthreads_or(band)) {                      // uniform; almost never taken
            for (int w = 0; w < (A + 31) / 32; ++w) {
                unsigned bits = sBand[w];
                while (bits) {
                    const int a = w * 32 + __builtin_ctz(bits);
                    bits &= bits - 1;
                    const int h = a / (NC * NV);
                    const double step = cfg.speed[a % NV] * cfg.dt;
                    const double qx = s[0] + step * sCos[h], qy = s[1] + step * sSin[h];
                    const double qz = s[2] + cfg.climb[(a / NV) % NC] * cfg.dt;
                    double dmin = INFINITY;
                    for (int j = tid; j < n_row; j += NT)
                        dmin = fmin(dmin, entry_d2(qx, qy, qz, tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]));
                    dmin = -wave_max(-dmin);
                    if (lane == 0) red_d[wave] = dmin;
                    __syncthreads();
                    if (tid == 0) {
                        double d2 = red_d[0];
                        for (int q = 1; q < NW; ++q) d2 = fmin(d2, red_d[q]);
                        sD2[a] = d2;
                        sV[a] = score_action(cfg, tb, a, s, g, sCos[h], sSin[h], d2).V;
                    }
                    __syncthreads();
                }
            }
        }
        if (eval) {
            for (int a = tid; a < A; a += NT) {
                const int h = a / (NC * NV);
                const Scored r = score_action(cfg, tb, a, s, g, sCos[h], sSin[h], sD2[a]);
                if (ev.V) ev.V[a] = r.V;
                if (ev.G) ev.G[a] = r.G;
                if (ev.I) ev.I[a] = r.I;
                if (ev.T) ev.T[a] = r.T;
            }
        } else {
            prefetch(row + 1);                             // in flight during the argmax and advance
        }

        // 5-6. argmax (one wave: largest value, then the lowest index inside
        //      the tie band) and advance
        if (wave == 0) {
            double vm = -INFINITY;
            for (int a = lane; a < A; a += 64) vm = fmax(vm, sV[a]);
            vm = wave_max(vm);
            const double thr = vm - cfg.tie_rel * fabs(vm);
            int li = 0x7fffffff;
            for (int a = lane; a < A; a += 64)
                if (sV[a] >= thr) { li = a; break; }
            li = wave_min(li);
            const int best = vm == -INFINITY ? -1 : li;
            // inside the tie band the chosen action may not be the largest:
            // remember the (lowest-index) largest for the acceptance check
            int top = -1;
            if (best >= 0 && sV[best] < vm) {
                int ti = 0x7fffffff;
                for (int a = lane; a < A; a += 64)
                    if (sV[a] == vm) { ti = a; break; }
                top = wave_min(ti);
            }
            if (lane == 0) {
                if (eval) {
                    if (ev.best) *ev.best = best;
                } else if (best < 0) {
                    st_status = FASTMDP_NO_VALID_ACTION;
                } else {
                    const int h = best / (NC * NV);
                    const Scored r = score_action(cfg, tb, best, s, g, sCos[h], sSin[h], sD2[best]);
                    const size_t p = pt_base + n;
                    tr.xyz[p * 3 + 0] = r.x;
                    tr.xyz[p * 3 + 1] = r.y;
                    tr.xyz[p * 3 + 2] = r.z;
                    tr.act[p] = best;
                    tr.val[p] = r.V;
                    tr.seen[p] = n_row;
                    tr.top[p] = top;
                    st_s[0] = r.x; st_s[1] = r.y; st_s[2] = r.z;
                    st_n = n + 1;
                    if (r.I > 0.0) st_status = FASTMDP_REJECT_SEPARATION;
                    else if (r.clr < 0.0) st_status = FASTMDP_REJECT_TERRAIN;
                }
            }
        }
        pairs += (long long)A * n_row;
        steps_here += 1;
        __syncthreads();
        if (eval) break;
    }
    __syncthreads();   // st_status written by thread 0 on the way out of the loop

    // Commit validation of a finished OK trajectory against every table
    // entry it saw: each point as planned (FP64) must be at least R_sep from
    // every entry of its row that existed when the row was scored, and clear
    // of the terrain.  Entries appended later are the sequencer's
    // interaction check.
    if (!eval && validate && st_status == FASTMDP_OK) {
        const int n = st_n;
        const double r2 = cfg.R_sep * cfg.R_sep;
        int bad = 0;
        for (int k = 0; k < n; ++k) {
            const double *x = tr.xyz + (pt_base + k) * 3;
            const int lim = tr.seen[pt_base + k];
            const size_t rb = (size_t)(t0 + k) * tb.cap;
            for (int j = tid; j < lim; j += NT)
                if (entry_d2(x[0], x[1], x[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < r2) bad = 1;
            if (tb.terr && (k % NT) == tid && x[2] - terrain_height(tb, x[0], x[1]) < 0.0) bad = 1;
        }
        bad = __syncthreads_or(bad);
        if (tid == 0) S.valid = bad == 0;
    }

    if (tid == 0 && !eval) {
        S.n_points = st_n;
        S.status = st_status;
    }
    if (tid == 0) {
        S.pairs += pairs;
        S.steps += steps_here;
    }
}

// ---------------------------------------------------------------------------
// launch dispatch over the supported (climbs, speeds, zero-climb) shapes
// ---------------------------------------------------------------------------
template <int NC, int NV, int ZC>
static hipError_t launch_t(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                           const int *list, const Traj &tr, int budget, int validate, const EvalOut &ev) {
    if (nt == 1024)
        hipLaunchKernelGGL((planner_kernel<1024, NC, NV, ZC>), dim3(nblk), dim3(1024), 0, st, c, t, s, list, tr, budget,
                           validate, ev);
    else
        hipLaunchKernelGGL((planner_kernel<256, NC, NV, ZC>), dim3(nblk), dim3(256), 0, st, c, t, s, list, tr, budget,
                           validate, ev);
    return hipGetLastError();
}

#define FMDP_SHAPE(NC, NV, ZC) \
    if (c.n_climb == NC && c.n_speed == NV && zc == ZC) return launch_t<NC, NV, ZC>(nblk, nt, st, c, t, s, list, tr, budget, validate, ev);

hipError_t launch_planner(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                          const int *list, const Traj &tr, int budget, int validate, const EvalOut &ev) {
    const int zc = c.zero_climb;
    FMDP_SHAPE(1, 1, 0) FMDP_SHAPE(1, 1, -1) FMDP_SHAPE(1, 2, 0) FMDP_SHAPE(1, 2, -1)
    FMDP_SHAPE(1, 3, 0) FMDP_SHAPE(1, 3, -1)
    FMDP_SHAPE(2, 1, -1) FMDP_SHAPE(2, 2, -1) FMDP_SHAPE(2, 3, -1)
    FMDP_SHAPE(3, 1, 1) FMDP_SHAPE(3, 1, -1) FMDP_SHAPE(3, 2, 1) FMDP_SHAPE(3, 2, -1)
    FMDP_SHAPE(3, 3, 1) FMDP_SHAPE(3, 3, -1)
    FMDP_SHAPE(5, 1, 2) FMDP_SHAPE(5, 3, 2) FMDP_SHAPE(5, 3, -1)
    return hipErrorInvalidValue;
}

bool planner_shape_supported(int n_climb, int n_speed, int zc) {
    const int nc = n_climb, nv = n_speed;
#define FMDP_OK(NC, NV, ZC) if (nc == NC && nv == NV && zc == ZC) return true;
    FMDP_OK(1, 1, 0) FMDP_OK(1, 1, -1) FMDP_OK(1, 2, 0) FMDP_OK(1, 2, -1) FMDP_OK(1, 3, 0) FMDP_OK(1, 3, -1)
    FMDP_OK(2, 1, -1) FMDP_OK(2, 2, -1) FMDP_OK(2, 3, -1)
    FMDP_OK(3, 1, 1) FMDP_OK(3, 1, -1) FMDP_OK(3, 2, 1) FMDP_OK(3, 2, -1) FMDP_OK(3, 3, 1) FMDP_OK(3, 3, -1)
    FMDP_OK(5, 1, 2) FMDP_OK(5, 3, 2) FMDP_OK(5, 3, -1)
#undef FMDP_OK
    return false;
}

}  // namespace fmdp
