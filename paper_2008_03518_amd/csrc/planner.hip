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
#include "proposal.h"
#include "score.h"
#include "wave.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fmdp {

// Largest risk well, at point (x, y, z), of the peaks of the other aircraft
// of a co-simulated batch (all but slot `self`): |r_intr| gamma_intr^(d/ell)
// of the nearest peak whose radius contains the point (the wells share r and
// gamma, so the nearest such peak gives the largest), 0 if none.
__device__ double mate_well(const DevCfg &c, const MatePeaks &mp, int nm, int self, double x, double y, double z) {
    double best = INFINITY;
    for (int k = 0; k < nm; ++k) {
        if (mp.owner[k] == self) continue;
        const double *p = mp.pk + 4 * k;
        const double dx = x - p[0], dy = y - p[1], dz = z - p[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < p[3] * p[3]) best = fmin(best, d2);
    }
    return best < INFINITY ? c.abs_r_intr * exp(c.log_gamma_intr * (sqrt(best) / c.ell)) : 0.0;
}

// Relative margin that makes the FP32 goal term an upper bound of the FP64
// one: the FP32 exponent r*log2(gamma)*d/ell carries a relative error of a few
// 1e-7 (distance, constants, roundings), i.e. an absolute error below 1.2e-5
// for exponents up to 40 (over 50 km at 20 m per step), and the result a
// relative error below 1e-5; 1e-4 leaves a factor of ten.
constexpr float kGoalBoundRel = 1e-4f;
// Longest run of steps the proposal sits out after repeated fallbacks.
constexpr int kMaxBackoff = 16;

template <int NT>
struct PlanGeom {
    static constexpr int NW = NT / 64;
    static constexpr int TILE = 4096;                        // row entries per chunk (LDS tile)
    static constexpr int PRE = TILE / NT;                    // chunk entries per thread
    static constexpr int PRE4 = TILE / (4 * NT);             // 16-byte (four-entry) groups per thread
    static_assert(TILE % (4 * NT) == 0, "a chunk is a whole number of four-entry groups per thread");
};

template <int NT, int NC, int NV, int ZC, bool PROP, bool LOOK = false, bool CULL = false>
__global__ __launch_bounds__(NT) void planner_kernel(DevCfg cfg, DevTable tb, Slot *slots, const int *slot_list,
                                                     Traj tr, int budget, int validate, int epoch, EvalOut ev,
                                                     PropArgs prop, LaunchStop stop, MatePeaks mates) {
    using Geo = PlanGeom<NT>;
    constexpr int NW = Geo::NW, TILE = Geo::TILE, PRE = Geo::PRE, PRE4 = Geo::PRE4;
    constexpr int KMAX = FASTMDP_MAX_TOPK, HID = FASTMDP_MLP_HIDDEN;
    __shared__ float4 tile[TILE];               // staged plans; reused for the slice partial minima
    // the next row chunk as read from the table, and its visibility keys
    __shared__ __attribute__((aligned(16))) float rawX[TILE], rawY[TILE], rawZ[TILE];
    __shared__ __attribute__((aligned(16))) int rawK[TILE];
    __shared__ double sD2[kMaxActions];         // squared nearest-plan distance per action
    __shared__ double sC0[kMaxHeads], sS0[kMaxHeads];    // cos, sin of the heading offsets 2*pi*h/H
    __shared__ double sCos[kMaxHeads], sSin[kMaxHeads];  // heading directions of the current step
    __shared__ unsigned sBand[kMaxActions / 32];
    __shared__ double st_s[3];
    __shared__ int st_n, st_status, st_flag;
    __shared__ int st_stop[2];                  // early end: read at the top of local step i from slot i & 1
    __shared__ int sNextN[2];                   // entry count of row r + 1, slot (r + 1) & 1, loaded with row r
    __shared__ int sStopV;                      // launch stop counter as last read
    __shared__ double red_d[NW];
    __shared__ int s_wsum[NW];
    __shared__ int s_wli[NW], s_wti[NW];        // per-wave argmax partials
    __shared__ int s_any;
    __shared__ int s_nvis;                      // visible row entries counted by the DMA-buffer K sweep
    // proposal path only
    __shared__ FeatAcc sFa;                                      // traffic feature accumulators
    __shared__ __attribute__((aligned(16))) uint16_t sAct[3][HID];   // BF16 features, hidden 1, hidden 2
    __shared__ float sKey[kMaxActions];                          // ranking key per action
    __shared__ float sGu[kMaxActions];                           // goal-term upper bound per action
    __shared__ unsigned sInK[kMaxActions / 32];                  // proposed-set membership
    __shared__ int sK[KMAX];                                     // proposed actions, best first
    __shared__ float sKm[NW][KMAX];                              // per-wave nearest minima
    __shared__ int st_cert, st_best, st_top;
    __shared__ double st_r[6];                                   // chosen action's scoring: x, y, z, V, I, clearance
    // the last point taken, written to the trajectory after the next step's
    // staging (its stores then overlap that step instead of holding up the
    // wait for the row): x, y, z, value, nearest distance; index, action,
    // row entries seen, epoch, top action
    __shared__ double st_pv[5];
    __shared__ int st_pi[5], st_pend;
    __shared__ int st_seenw[kMaxLookahead], st_pseenw[kMaxLookahead];   // window rows' entry counts:
                                                                       // this step, the pending point
    __shared__ double sStep[FASTMDP_MAX_ACT_DIM], sDz[FASTMDP_MAX_ACT_DIM];   // speed*dt, climb*dt
    __shared__ float sKv[FASTMDP_MAX_ACT_DIM], sClf[FASTMDP_MAX_ACT_DIM];      // FP32 sweep constants
    const ActTab at{sStep, sDz};

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int slot = slot_list ? slot_list[blockIdx.x] : (int)blockIdx.x;
    Slot &S = slots[slot];
    const bool eval = ev.V != nullptr || ev.best != nullptr;
    if (!eval && S.status != kRunning) return;          // a finished request (uniform: one slot per workgroup)

    const int H = cfg.n_head, A = cfg.n_actions;
    const int n_mates = (!PROP && !LOOK && mates.n) ? *mates.n : 0;   // co-simulated batch peaks
    const int n_slices = NT / H;
    const int my_h = tid % H, my_slice = tid / H;
    const bool sweeper = tid < n_slices * H;
    const int tcap = TILE;                                        // row entries per chunk
    const int n_part = n_slices;                                  // slice partial minima per action

    const double g[3] = {S.goal[0], S.goal[1], S.goal[2]};
    const int t0 = S.t0;
    const int seq = S.seq;
    const size_t pt_base = (size_t)slot * tr.stride;

    for (int h = tid; h < H; h += NT) {
        const double th = 2.0 * M_PI * (double)h / (double)H;
        sC0[h] = cos(th);
        sS0[h] = sin(th);
    }
    if (tid < FASTMDP_MAX_ACT_DIM) {
        sStep[tid] = cfg.speed[tid] * cfg.dt;
        sDz[tid] = cfg.climb[tid] * cfg.dt;
        sKv[tid] = cfg.kv[tid];
        sClf[tid] = cfg.climb_f[tid];
    }
    if constexpr (PROP) feat_reset(sFa, tid);
    if (tid == 0) {
        sStopV = 0;
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
        st_stop[0] = st_stop[1] = 0;
        st_pend = 0;
        s_any = 0;
        s_nvis = 0;
    }
    __syncthreads();

    // Origin check of a fresh request: inside the box, clear of terrain, and
    // no plan active at the departure row closer than R_sep.
    if (!eval && st_n == 0) {
        const double o[3] = {st_s[0], st_s[1], st_s[2]};
        const int n_row = t0 < tb.rows ? min(tb.rowN[t0], tb.cap) : 0;
        const size_t rb = (size_t)t0 * tb.cap;
        int hit = 0;
        for (int j = tid; j < n_row; j += NT)
            if (entry_visible(tb, rb + j, seq) &&
                entry_d2(o[0], o[1], o[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < cfg.R_sep * cfg.R_sep)
                hit = 1;
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
            tr.ep[pt_base] = epoch;
            tr.top[pt_base] = -1;
            tr.col[pt_base] = -1;
            tr.nd[pt_base] = INFINITY;
            st_n = 1;
            if (blocked) st_status = FASTMDP_REJECT_ORIGIN;
        }
        __syncthreads();
    }

    // One chunk of a row (up to tcap entries) travels from the table to LDS
    // without registers (global_load_lds): entry base + j lands at raw*[j].
    // Each lane later stages exactly the entries its own loads brought, so a
    // wave only waits for its own loads (vmcnt), with no barrier, and may
    // issue the next row's loads as soon as it has staged this one.  The
    // first chunk of the next step's row is in flight during the sweep.
    int pre_n = 0, pre_lim = 0;
    auto load_chunk = [&](int row, int base, bool with_count = true) {
        const size_t rb = (size_t)row * tb.cap + base;
        const int lim = min(pre_n - base, tcap);
        pre_lim = lim;
        // the entry count of the following row travels with the first chunk,
        // so that the step does not wait for it on its own
        if (base == 0 && tid == 0 && with_count) {
            if (row + 1 < tb.rows)
                __builtin_amdgcn_global_load_lds(tb.rowN + row + 1, sNextN + ((row + 1) & 1), 4, 0, 0);
            else
                sNextN[(row + 1) & 1] = 0;
        }
        // 16 bytes (four entries) per lane and instruction: lane l of wave w
        // brings entries j0 + 4l .. j0 + 4l + 3, j0 = i*4*NT + 256w.  A group
        // that runs past the row's count stays inside the row's capacity (a
        // multiple of four), so the read is in bounds; the extra entries are
        // never staged.  The per-lane offset is made opaque so that the
        // addresses are formed here instead of being hoisted out of the step
        // loop, where they would occupy registers and be spilled.
        int ofs = 4 * tid;
        asm volatile("" : "+v"(ofs));
#pragma unroll
        for (int i = 0; i < PRE4; ++i) {
            const int j0 = i * 4 * NT + wave * 256;        // wave-uniform LDS destination
            const int j = ofs + i * 4 * NT;
            if (j < lim) {
                load_lds16(tb.X + rb + j, rawX + j0);
                load_lds16(tb.Y + rb + j, rawY + j0);
                load_lds16(tb.Z + rb + j, rawZ + j0);
                load_lds16(tb.vis + rb + j, rawK + j0);
            }
        }
    };
    auto row_count = [&](int row) { return (row >= 0 && row < tb.rows) ? min(tb.rowN[row], tb.cap) : 0; };
    // Stage the chunk into the tile, compacted to the entries this request
    // sees, as (q_x, q_y, -2 dt q_z, |q|^2) with q = p - s.  Returns the
    // count.
    int steps_here = 0;
    // Early end of the launch (thread 0): the flag for the next step from
    // the counter value read during the previous step, then the next read,
    // device-coherent and straight into LDS, so that nothing waits for it
    // until the next step's staging
    auto take_stop = [&]() {
        if (tid == 0 && stop.target > 0 && !eval) {
            st_stop[(steps_here + 1) & 1] = sStopV >= stop.target;
            __builtin_amdgcn_global_load_lds(stop.ctr, &sStopV, 4, 0, kCachePolicyDevice);
        }
    };
    auto stage_chunk = [&](const double s[3], bool cull = true) -> int {
        // wave-level compaction with ballots: entry i of this lane goes after
        // the wave's visible entries of lower i and of lower lanes at i
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's loads of the chunk landed
        take_stop();
        if (CULL && cull) {
            // range query: of the visible entries only those within the
            // staging radius of the state (farther plans cannot reach any
            // scored point's well), so the offsets come before the ballots
            float4 e[PRE4][4];
            bool pv[PRE4][4];
            uint64_t bal[PRE4][4];
            int wcnt = 0;
#pragma unroll
            for (int i = 0; i < PRE4; ++i) {
                const int j = 4 * tid + i * 4 * NT;
                const int4 k4 = *reinterpret_cast<const int4 *>(rawK + j);
                const float4 x4 = *reinterpret_cast<const float4 *>(rawX + j);
                const float4 y4 = *reinterpret_cast<const float4 *>(rawY + j);
                const float4 z4 = *reinterpret_cast<const float4 *>(rawZ + j);
                const int kv4[4] = {k4.x, k4.y, k4.z, k4.w};
                const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
                const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
                const float zs[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float qx = (float)((double)xs[m] - s[0]);
                    const float qy = (float)((double)ys[m] - s[1]);
                    const float qz = (float)((double)zs[m] - s[2]);
                    const float w = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
                    e[i][m] = make_float4(qx, qy, cfg.zeta_scale * qz, w);
                    pv[i][m] = j + m < pre_lim && kv4[m] < seq && w < cfg.cull_r2;
                    bal[i][m] = __ballot(pv[i][m]);
                    wcnt += __popcll(bal[i][m]);
                }
            }
            if (lane == 0) s_wsum[wave] = wcnt;
            lds_barrier();
            int pos = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int t = s_wsum[w];
                pos += w < wave ? t : 0;
                total += t;
            }
#pragma unroll
            for (int i = 0; i < PRE4; ++i)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (pv[i][m]) {
                        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[i][m] >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bal[i][m], 0));
                        tile[pos + below] = e[i][m];
                    }
                    pos += __popcll(bal[i][m]);
                }
            return total;
        }
        // each lane stages the four-entry groups its own loads brought
        bool pv[PRE4][4];
        uint64_t bal[PRE4][4];
        int wcnt = 0;
#pragma unroll
        for (int i = 0; i < PRE4; ++i) {
            const int j = 4 * tid + i * 4 * NT;
            const int4 k4 = *reinterpret_cast<const int4 *>(rawK + j);
            const int kv4[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                pv[i][m] = j + m < pre_lim && kv4[m] < seq;
                bal[i][m] = __ballot(pv[i][m]);
                wcnt += __popcll(bal[i][m]);
            }
        }
        if (lane == 0) s_wsum[wave] = wcnt;
        lds_barrier();
        int pos = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int t = s_wsum[w];
            pos += w < wave ? t : 0;
            total += t;
        }
#pragma unroll
        for (int i = 0; i < PRE4; ++i) {
            const int j = 4 * tid + i * 4 * NT;
            const float4 x4 = *reinterpret_cast<const float4 *>(rawX + j);
            const float4 y4 = *reinterpret_cast<const float4 *>(rawY + j);
            const float4 z4 = *reinterpret_cast<const float4 *>(rawZ + j);
            const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
            const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
            const float zs[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (pv[i][m]) {
                    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[i][m] >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal[i][m], 0));
                    const float qx = (float)((double)xs[m] - s[0]);
                    const float qy = (float)((double)ys[m] - s[1]);
                    const float qz = (float)((double)zs[m] - s[2]);
                    tile[pos + below] =
                        make_float4(qx, qy, cfg.zeta_scale * qz, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
                }
                pos += __popcll(bal[i][m]);
            }
        }
        return total;
    };
    // Actions whose FP32 nearest distance lies within kBand of the well
    // radius (flagged in sBand) get it recomputed exactly in FP64 over the
    // visible entries of the row.  Uniform: every thread calls it.
    auto band_recheck = [&](const double s[3], int n_row, size_t rb, int win = 0) {
        for (int w = 0; w < (A + 31) / 32; ++w) {
            unsigned bits = sBand[w];
            while (bits) {
                const int a = w * 32 + __builtin_ctz(bits);
                bits &= bits - 1;
                const int h = a / (NC * NV);
                double qx, qy, qz;
                if (win > 0)
                    window_point(cfg, at, a, win, s, sCos[h], sSin[h], qx, qy, qz);
                else
                    successor(cfg, at, a, s, sCos[h], sSin[h], qx, qy, qz);
                double dmin = INFINITY;
                for (int j = tid; j < n_row; j += NT)
                    if (entry_visible(tb, rb + j, seq))
                        dmin = fmin(dmin, entry_d2(qx, qy, qz, tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]));
                dmin = -wave_max(-dmin);
                if (lane == 0) red_d[wave] = dmin;
                lds_barrier();
                if (tid == 0) {
                    double d2 = red_d[0];
                    for (int q = 1; q < NW; ++q) d2 = fmin(d2, red_d[q]);
                    sD2[a] = d2;
                }
                lds_barrier();
            }
        }
    };
    {
        const int row = (eval ? t0 : t0 + st_n - 1) + 1;
        pre_n = row_count(row);
        if (pre_n > 0) load_chunk(row, 0);
    }

    auto flush_point = [&]() {                                  // thread 0
        if (!st_pend) return;
        const size_t p = pt_base + st_pi[0];
        tr.xyz[p * 3 + 0] = st_pv[0];
        tr.xyz[p * 3 + 1] = st_pv[1];
        tr.xyz[p * 3 + 2] = st_pv[2];
        tr.val[p] = st_pv[3];
        tr.nd[p] = st_pv[4];
        tr.act[p] = st_pi[1];
        tr.seen[p] = st_pi[2];
        tr.ep[p] = st_pi[3];
        tr.top[p] = st_pi[4];
        tr.col[p] = -1;
        if constexpr (LOOK) {
            for (int w = 0; w < cfg.lookahead; ++w) tr.seenw[p * cfg.lookahead + w] = st_pseenw[w];
        }
        st_pend = 0;
    };

    long long pairs = 0, entries = 0;
    int hits = 0, misses = 0;
    int since = 1 << 30;                                         // steps since the last ranking
    // after a step that fell back, the proposal sits out `skip` steps (the
    // full sweep runs directly), doubling up to kMaxBackoff while it keeps
    // failing: inside traffic the certificate rarely holds and the attempt
    // would only add to the full sweep's cost
    int skip = 0, backoff = 1;

    for (;;) {
        if (st_status != kRunning) break;                 // uniform (LDS, after a barrier)
        const int n = st_n;
        const int k = eval ? 0 : n - 1;                    // steps taken so far
        const int t = eval ? t0 : t0 + k;
        const double s[3] = {st_s[0], st_s[1], st_s[2]};
        if (!eval) {
            const double ex = g[0] - s[0], ey = g[1] - s[1], ez = g[2] - s[2];
            if (sqrt(ex * ex + ey * ey + ez * ez) <= cfg.ell) {
                lds_barrier();
                if (tid == 0) st_status = FASTMDP_OK;
                break;
            }
            if (k >= cfg.max_steps) {
                lds_barrier();
                if (tid == 0) st_status = FASTMDP_TIMEOUT;
                break;
            }
            if (steps_here >= budget || st_stop[steps_here & 1]) break;   // resumable: stays running
        }

        // 1. heading directions: the goal bearing rotated by each offset
        const double bx = g[0] - s[0], by = g[1] - s[1];
        const double br = sqrt(bx * bx + by * by);
        const double cb = br > 0.0 ? bx / br : 1.0, sb = br > 0.0 ? by / br : 0.0;
        for (int h = tid; h < H; h += NT) {
            sCos[h] = cb * sC0[h] - sb * sS0[h];
            sSin[h] = sb * sC0[h] + cb * sS0[h];
        }
        const int row = t + 1;
        const int n_row = pre_n;
        entries += n_row;                                 // (thread 0's count is the one kept)
        const size_t rb = (size_t)row * tb.cap;
        const bool single = n_row <= tcap;
        // entry count of the next row: it came with this row's first chunk
        // (read after that chunk's staging), else it is read directly
        auto next_count = [&]() -> int {
            if (eval) return 0;
            return n_row > 0 ? min(sNextN[(row + 1) & 1], tb.cap) : row_count(row + 1);
        };

        int n_vis = 0;
        bool staged = false;
        int cert = 0;
        // Proposal path (rows that fit one tile): rank the actions, score the
        // top k exactly with the full sweep's arithmetic, and take the step
        // from them when the certificate holds.
        if constexpr (PROP) {
            if (prop.mode != FASTMDP_PROPOSE_NONE && single && (skip == 0 || eval)) {
                // the ranking (and the proposed set) is refreshed every
                // prop.refresh steps and after every fallback; the certificate
                // is decided at every step
                const bool rank = eval || since >= prop.refresh;
                // Unless the network's features need the staged tile, the K
                // actions are swept straight from the row's DMA buffers, and
                // the row is staged only if the step falls back to the full
                // sweep (the buffers still hold it until the next row's loads
                // are issued, after the certificate).
                const bool fused = !eval && !(rank && prop.mode == FASTMDP_PROPOSE_MLP);
                if (!fused) {
                    if (n_row > 0) n_vis = stage_chunk(s, false);   // the features see every plan
                    if (!eval) {                           // next row in flight meanwhile
                        pre_n = next_count();
                        if (pre_n > 0) load_chunk(row + 1, 0);
                    }
                    staged = true;
                }
                const int K = min(prop.k, A);
                if (n_row == 0 || fused) lds_barrier();    // headings visible (staging has its own barrier)
                // upper bound of every action's goal term (FP32 with a margin;
                // -inf outside the box, decided in FP64)
                {
                    const float gx32 = (float)(g[0] - s[0]), gy32 = (float)(g[1] - s[1]);
                    const float gz32 = (float)(g[2] - s[2]);
                    for (int a = tid; a < A; a += NT) {
                        const int h = a / (NC * NV);
                        double x, y, z;
                        successor(cfg, at, a, s, sCos[h], sSin[h], x, y, z);
                        float gu = -INFINITY;
                        if (!outside_box(cfg, x, y, z)) {
                            const float ex = gx32 - (float)(x - s[0]), ey = gy32 - (float)(y - s[1]);
                            const float ez = gz32 - (float)(z - s[2]);
                            gu = cfg.abs_r_goal_f *
                                 exp2f(cfg.log2_gamma_f * (sqrtf(ex * ex + ey * ey + ez * ez) * cfg.inv_ell_f)) *
                                 (1.0f + kGoalBoundRel);
                        }
                        sGu[a] = gu;
                        if (rank && prop.mode == FASTMDP_PROPOSE_GOAL) sKey[a] = gu;
                    }
                }
                if (rank)
                    for (int w = tid; w < kMaxActions / 32; w += NT) sInK[w] = 0u;
                lds_barrier();                             // tile staged, headings visible
                if (tid == 0 && !fused) flush_point();
                if (rank && prop.mode == FASTMDP_PROPOSE_MLP) {
                    const float ux = (float)cb, uy = (float)sb;
                    for (int j = tid; j < n_vis; j += NT) {
                        const float4 p = tile[j];
                        feat_point(sFa, p.x, p.y, p.z <= 0.0f, p.w, ux, uy);
                    }
                    lds_barrier();
                    if (tid < FASTMDP_N_FEAT) {
                        const float f = feat_value(sFa, tid, s, g, cfg.box_lo, cfg.box_hi, cfg.ell);
                        sAct[0][tid] = f2bf(f);
                        if (ev.feat) ev.feat[tid] = f;
                    }
                    lds_barrier();
                    feat_reset(sFa, tid);                  // next use is several barriers away
                    // three layers, one 16-neuron tile per wave at a time:
                    // the state vector is broadcast to every row of the MFMA A
                    // operand, the weights [out][in] are the B operand, row 0
                    // of the result (lanes 0-15, register 0) is the layer.  All
                    // of a tile's weight loads are issued before its MFMAs.
                    const PropNet &W = prop.net;
                    for (int layer = 0; layer < 3; ++layer) {
                        const int kin = layer == 0 ? FASTMDP_N_FEAT : HID;
                        const int nk = kin / 32;
                        const int nout = layer == 2 ? A : HID;
                        const uint16_t *Wl = layer == 0 ? W.W1 : (layer == 1 ? W.W2 : W.W3);
                        const float *bl = layer == 0 ? W.b1 : (layer == 1 ? W.b2 : W.b3);
                        const uint16_t *in = sAct[layer];
                        const int kofs = 8 * (lane >> 4);
                        for (int tl = wave; tl * 16 < nout; tl += NW) {
                            const int nn = tl * 16 + (lane & 15);
                            const uint4 *wrow = reinterpret_cast<const uint4 *>(Wl + (size_t)nn * kin + kofs);
                            uint4 wv[HID / 32];
#pragma unroll
                            for (int q = 0; q < HID / 32; ++q)
                                if (q < nk) wv[q] = wrow[4 * q];
                            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                            for (int q = 0; q < HID / 32; ++q)
                                if (q < nk)
                                    acc = mfma_bf16(*reinterpret_cast<const uint4 *>(in + 32 * q + kofs), wv[q], acc);
                            if (lane < 16 && nn < nout) {
                                const float z = acc[0] + bl[nn];
                                if (layer < 2) {
                                    sAct[layer + 1][nn] = f2bf(fmaxf(z, 0.0f));
                                } else {
                                    sKey[nn] = z;
                                    if (ev.logit) ev.logit[nn] = z;
                                }
                            }
                        }
                        lds_barrier();
                    }
                }
                // top K by key (largest first, lowest index on ties; NaN
                // ranks last), one wave: keys packed with the complement of
                // the index into 64 bits and sorted within each lane once;
                // each round takes the wave maximum of the lanes' heads
                if (rank && wave == 0) {
                    constexpr int KPL = kMaxActions / 64;
                    uint64_t kk[KPL];
#pragma unroll
                    for (int i = 0; i < KPL; ++i) {
                        const int a = lane + 64 * i;
                        kk[i] = a < A ? ((uint64_t)ordered_f32(sKey[a]) << 32) | (0xffffffffu - (uint32_t)a) : 0u;
                    }
                    auto cas = [&](int i, int j) {         // descending
                        const uint64_t x = kk[i], y = kk[j];
                        kk[i] = x > y ? x : y;
                        kk[j] = x > y ? y : x;
                    };
                    // Batcher's odd-even merge network for 8 keys
                    cas(0, 1); cas(2, 3); cas(4, 5); cas(6, 7);
                    cas(0, 2); cas(1, 3); cas(4, 6); cas(5, 7);
                    cas(1, 2); cas(5, 6);
                    cas(0, 4); cas(1, 5); cas(2, 6); cas(3, 7);
                    cas(2, 4); cas(3, 5);
                    cas(1, 2); cas(3, 4); cas(5, 6);
                    for (int r = 0; r < K; ++r) {
                        const uint64_t m = wave_max_u64(kk[0]);
                        const int a = (int)(0xffffffffu - (uint32_t)m);
                        if (kk[0] == m) {
#pragma unroll
                            for (int i = 0; i + 1 < KPL; ++i) kk[i] = kk[i + 1];
                            kk[KPL - 1] = 0u;
                        }
                        if (lane == 0) {
                            sK[r] = a;
                            if (ev.topk) ev.topk[r] = a;
                        }
                    }
                }
                if (rank) {
                    lds_barrier();
                    if (wave == 0 && lane < K) {
                        const int a = sK[lane];
                        atomicOr(&sInK[a >> 5], 1u << (a & 31));
                    }
                    since = 0;
                }
                since += 1;
                // exact nearest distances of the K actions: the sweep's FP32
                // expression over the same staged plans (min is exact, so
                // the result does not depend on the order).  Lane r holds the
                // constants of action r; each round broadcasts them.
                {
                    // (the zero climb's constant is 0, so fmaf(0, z, u) = u: the
                    // full sweep's skipped term)
                    float kch = 0.0f, ksh = 0.0f, kkv = 0.0f, kclf = 0.0f;
                    if (lane < K) {
                        const int a = sK[lane];
                        const int h = a / (NC * NV), c = (a / NV) % NC, v = a % NV;
                        kch = (float)sCos[h];
                        ksh = (float)sSin[h];
                        kkv = sKv[v];
                        kclf = sClf[c];
                    }
                    // the thread's staged plans in registers (slots past the
                    // row's visible plans skipped), all K minima, then the K
                    // wave reductions side by side
                    float4 pe[PRE];
                    int n_pre;
                    if (!fused) {
#pragma unroll
                        for (int i = 0; i < PRE; ++i) {
                            const int j = tid + i * NT;
                            pe[i] = j < n_vis ? tile[j] : make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                        }
                        n_pre = min(PRE, (n_vis + NT - 1) / NT + 1) & ~1;   // uniform, even (pe beyond n_vis is far)
                    } else {
                        // this lane's four-entry groups as its loads brought
                        // them, in the staging's arithmetic; entries the
                        // request does not see and slots past the row read as
                        // a plan at infinity
                        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                        take_stop();
                        const int lim = n_row > 0 ? pre_lim : 0;
                        int seen_w = 0;
#pragma unroll
                        for (int gi = 0; gi < PRE4; ++gi) {
                            const int j = 4 * tid + gi * 4 * NT;
                            const int4 k4 = *reinterpret_cast<const int4 *>(rawK + j);
                            const float4 x4 = *reinterpret_cast<const float4 *>(rawX + j);
                            const float4 y4 = *reinterpret_cast<const float4 *>(rawY + j);
                            const float4 z4 = *reinterpret_cast<const float4 *>(rawZ + j);
                            const int kv4[4] = {k4.x, k4.y, k4.z, k4.w};
                            const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
                            const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
                            const float zs[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
                            for (int m = 0; m < 4; ++m) {
                                bool vis = j + m < lim && kv4[m] < seq;
                                float4 p = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                                if (vis) {
                                    const float qx = (float)((double)xs[m] - s[0]);
                                    const float qy = (float)((double)ys[m] - s[1]);
                                    const float qz = (float)((double)zs[m] - s[2]);
                                    p = make_float4(qx, qy, cfg.zeta_scale * qz, fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
                                    if constexpr (CULL) {        // range query: farther plans read as far
                                        if (!(p.w < cfg.cull_r2)) {
                                            vis = false;
                                            p = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                                        }
                                    }
                                }
                                pe[gi * 4 + m] = p;
                                seen_w += __popcll(__ballot(vis));
                            }
                        }
                        if (lane == 0) atomicAdd(&s_nvis, seen_w);
                        n_pre = min(PRE, 4 * ((lim + 4 * NT - 1) / (4 * NT)));   // uniform
                    }
                    float mk[KMAX];
#pragma unroll
                    for (int r = 0; r < KMAX; ++r) {
                        float m = INFINITY;
                        if (r < K) {                                     // uniform
                            const float ch = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kch), r));
                            const float sh = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ksh), r));
                            const float kvv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kkv), r));
                            const float clv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kclf), r));
#pragma unroll
                            for (int i = 0; i < PRE; i += 2) {
                                if (i < n_pre) {                         // uniform; n_pre is even
                                    const float hq0 = fmaf(pe[i].x, ch, pe[i].y * sh);
                                    const float hq1 = fmaf(pe[i + 1].x, ch, pe[i + 1].y * sh);
                                    const float u0 = fmaf(kvv, hq0, pe[i].w);
                                    const float u1 = fmaf(kvv, hq1, pe[i + 1].w);
                                    m = fminf(m, fminf(fmaf(clv, pe[i].z, u0), fmaf(clv, pe[i + 1].z, u1)));
                                }
                            }
                        }
                        mk[r] = m;
                    }
                    // the K wave minima, eight at a time
                    static_assert(KMAX % 8 == 0, "minima are reduced in groups of eight");
#pragma unroll
                    for (int r0 = 0; r0 < KMAX; r0 += 8) {
                        if (r0 < K) {                                    // uniform
                            const float m = wave_min8_f32(mk + r0, lane);
                            const int r = r0 + 2 * (lane >> 4) + ((lane >> 3) & 1);
                            if ((lane & 7) == 0 && r < K) sKm[wave][r] = m;
                        }
                    }
                }
                for (int w = tid; w < kMaxActions / 32; w += NT) sBand[w] = 0u;
                lds_barrier();
                if (fused) n_vis = s_nvis;                     // reset by thread 0 two barriers on
                int band = 0;
                if (wave == 0 && lane < K) {
                    const int a = sK[lane];
                    float m = INFINITY;
                    for (int w = 0; w < NW; ++w) m = fminf(m, sKm[w][lane]);
                    const double d2 = nearest_d2<NC, NV>(at, a, m);
                    sD2[a] = d2;
                    if (d2 > cfg.band_lo2 && d2 < cfg.band_hi2) {
                        atomicOr(&sBand[a >> 5], 1u << (a & 31));
                        band = 1;
                    }
                }
                if (band) s_any = 1;
                lds_barrier();
                const int any_band = s_any;
                lds_barrier();
                if (tid == 0) {
                    s_any = 0;
                    s_nvis = 0;
                }
                if (any_band) band_recheck(s, n_row, rb);
                // certificate: the best exact value among the K, less the tie
                // band, must exceed an upper bound of every other action's
                // goal term, hence of its value
                if (wave == 0) {
                    double v = -INFINITY;
                    int a = 0x7fffffff;
                    Scored sc{};
                    if (lane < K) {
                        a = sK[lane];
                        const int h = a / (NC * NV);
                        sc = score_action(cfg, tb, at, a, s, g, sCos[h], sSin[h], sD2[a]);
                        v = sc.V;
                    }
                    const double vm = wave_max(v);
                    const double thr = vm - cfg.tie_rel * fabs(vm);
                    float tau = -INFINITY;
#pragma unroll
                    for (int j = 0; j < kMaxActions / 64; ++j) {   // every read issued at once
                        const int b = j * 64 + lane;               // below kMaxActions: in bounds
                        const float gu = sGu[b];
                        const unsigned inK = sInK[b >> 5] >> (b & 31) & 1u;
                        if (b < A && !inK) tau = fmaxf(tau, gu);
                    }
                    tau = wave_maxf(tau);
                    int ok = vm > -INFINITY && (double)tau < thr;
                    // the FP32 bound is loose by up to 1e-4: where it does not
                    // clear the threshold but the exact goal term might, decide
                    // with the exact term (the one the value is computed from)
                    if (!ok && vm > -INFINITY && (double)tau * (1.0 - 4.0 * kGoalBoundRel) < thr) {
                        int bad = 0;
                        for (int b = lane; b < A; b += 64)
                            if (!(sInK[b >> 5] >> (b & 31) & 1u) && (double)sGu[b] >= thr) {
                                const int h = b / (NC * NV);
                                double x, y, z;
                                successor(cfg, at, b, s, sCos[h], sSin[h], x, y, z);
                                if (!(goal_term(cfg, x, y, z, g) < thr)) bad = 1;
                            }
                        ok = __ballot(bad) == 0;
                    }
                    const int best = wave_min(lane < K && v >= thr ? a : 0x7fffffff);
                    const int top1 = wave_min(lane < K && v == vm ? a : 0x7fffffff);
                    const double vb = wave_max(lane < K && a == best ? v : -INFINITY);
                    if (ok && lane < K && a == best) {             // the advance reuses the scoring
                        st_r[0] = sc.x; st_r[1] = sc.y; st_r[2] = sc.z;
                        st_r[3] = sc.V; st_r[4] = sc.I; st_r[5] = sc.clr;
                    }
                    if (lane == 0) {
                        st_cert = ok;
                        st_best = best;
                        st_top = vb < vm ? top1 : -1;
                        pairs += (long long)(K + (rank && prop.mode == FASTMDP_PROPOSE_MLP ? 1 : 0)) * n_vis;
                        if (eval) {
                            if (ev.cert) *ev.cert = ok;
                            if (ev.pbest) *ev.pbest = ok ? best : -1;
                        }
                    }
                }
                lds_barrier();
                cert = eval ? 0 : st_cert;                 // eval always runs the full sweep too
                if (fused) {
                    // a fallback needs the staged tile: the row is still in the
                    // DMA buffers; then the next row's loads
                    if (!cert && n_row > 0) n_vis = stage_chunk(s);
                    staged = !cert;
                    pre_n = next_count();
                    if (pre_n > 0) load_chunk(row + 1, 0);
                    if (tid == 0) flush_point();
                }
                if (!eval) {
                    if (cert) {
                        backoff = 1;
                    } else {
                        since = prop.refresh;              // re-rank at the next attempt
                        skip = backoff;
                        backoff = min(2 * backoff, kMaxBackoff);
                    }
                }
                if (tid == 0 && !eval) {
                    if (cert) ++hits;
                    else ++misses;
                }
            } else if (prop.mode != FASTMDP_PROPOSE_NONE && !eval) {
                if (skip > 0) --skip;
                if (tid == 0) ++misses;                    // backing off, or a row larger than one tile
            }
        }

        // the step's point and state from the chosen action's scoring (one
        // thread); a point still pending (row without plans) is written first
        auto advance = [&](const Scored &r, int best, int top) {
            flush_point();
            st_pv[0] = r.x; st_pv[1] = r.y; st_pv[2] = r.z;
            st_pv[3] = r.V; st_pv[4] = sD2[best];
            st_pi[0] = n; st_pi[1] = best; st_pi[2] = n_row; st_pi[3] = epoch; st_pi[4] = top;
            st_pend = 1;
            st_s[0] = r.x; st_s[1] = r.y; st_s[2] = r.z;
            st_n = n + 1;
            if (r.I > 0.0) st_status = FASTMDP_REJECT_SEPARATION;
            else if (r.clr < 0.0) st_status = FASTMDP_REJECT_TERRAIN;
        };

        if constexpr (LOOK) {
            // Lookahead window (Alg. 1's forward projections; "Forward
            // project": W points per action; "Compute value": the largest
            // value along them).  Point w of action a is s + w * Delta_a,
            // scored against row t + w: the same staging and sweep with the
            // action constants scaled by w (|q - w Delta|^2 - w^2 |Delta|^2 =
            // |q|^2 + w * (-2 Delta . q)).  Thread a keeps action a's running
            // maximum; its successor (w = 1) decides the advance, the recorded
            // nearest distance and the rejections.
            const int W = cfg.lookahead;
            const int a = tid;                                   // A <= kMaxActions <= NT
            Scored r1{}, rbest{};
            double vbest = -INFINITY, d2_1 = INFINITY;
            float *red = reinterpret_cast<float *>(tile);
            for (int w = 1; w <= W; ++w) {
                const int roww = row + w - 1;                    // t + w
                const int nw = w == 1 ? n_row : row_count(roww);
                const size_t rbw = (size_t)roww * tb.cap;
                const float fw = (float)w;
                float ch = 0.0f, sh = 0.0f;
                float kv[NV], clf[NC];
#pragma unroll
                for (int v = 0; v < NV; ++v) kv[v] = fw * sKv[v];
#pragma unroll
                for (int c = 0; c < NC; ++c) clf[c] = fw * sClf[c];
                float acc[NC][NV];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[c][v] = INFINITY;
                int nvis_w = 0;
                for (int base = 0; base < nw; base += tcap) {
                    if (w > 1 || base > 0) {                     // row t+1's first chunk came by prefetch
                        lds_barrier();                           // the tile is free
                        pre_n = nw;
                        load_chunk(roww, base, false);
                    }
                    const int nv = stage_chunk(s);
                    nvis_w += nv;
                    lds_barrier();
                    if (w == 1 && base == 0 && tid == 0) flush_point();
                    if (base == 0 && sweeper) {
                        ch = (float)sCos[my_h];
                        sh = (float)sSin[my_h];
                    }
                    auto sweep2 = [&](const float4 p0, const float4 p1) {
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
                    };
                    const int full = (nv / (2 * n_slices)) * (2 * n_slices);
                    if (sweeper) {
                        for (int i = my_slice; i < full; i += 2 * n_slices) sweep2(tile[i], tile[i + n_slices]);
                        if (full < nv) {
                            const float4 far = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                            const int i = full + my_slice;
                            sweep2(i < nv ? tile[i] : far, i + n_slices < nv ? tile[i + n_slices] : far);
                        }
                    }
                }
                if (tid == 0) {
                    st_seenw[w - 1] = nw;
                    pairs += (long long)A * nvis_w;
                    if (w > 1) entries += nw;
                }
                lds_barrier();                                   // the tile becomes the partials
                if (sweeper) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int v = 0; v < NV; ++v) red[my_slice * A + (my_h * NC + c) * NV + v] = acc[c][v];
                }
                for (int q = tid; q < kMaxActions / 32; q += NT) sBand[q] = 0u;
                lds_barrier();
                bool myband = false;
                if (a < A) {
                    float m = INFINITY;
                    for (int q = 0; q < n_part; ++q) m = fminf(m, red[q * A + a]);
                    const double stepw = w * at.step[a % NV], dzw = w * at.dz[(a / NV) % NC];
                    const double d2 = fma(dzw, dzw, fma(stepw, stepw, (double)m));
                    sD2[a] = d2;
                    if (d2 > cfg.band_lo2 && d2 < cfg.band_hi2) {
                        atomicOr(&sBand[a >> 5], 1u << (a & 31));
                        myband = true;
                    }
                }
                if (myband) s_any = 1;
                lds_barrier();
                const int any_band = s_any;
                if (any_band) {                                  // uniform; rare
                    lds_barrier();                               // every thread has read the flag
                    if (tid == 0) s_any = 0;
                    band_recheck(s, nw, rbw, w);
                }
                if (a < A) {
                    const int h = a / (NC * NV);
                    const Scored rw = score_action(cfg, tb, at, a, s, g, sCos[h], sSin[h], sD2[a], w);
                    if (w == 1) {
                        r1 = rw;
                        rbest = rw;
                        vbest = rw.V;
                        d2_1 = sD2[a];
                    } else if (rw.V > vbest) {
                        rbest = rw;
                        vbest = rw.V;
                    }
                }
                lds_barrier();                                   // partials and distances read
            }
            // the next step's first row (t + 2) while the argmax runs
            if (!eval) {
                pre_n = row_count(row + 1);
                if (pre_n > 0) load_chunk(row + 1, 0, false);
            }
            const double myV = (a < A && r1.V > -INFINITY) ? vbest : -INFINITY;
            const double wv = wave_max(myV);
            if (lane == 0) red_d[wave] = wv;
            lds_barrier();
            double vm = -INFINITY;
#pragma unroll
            for (int q = 0; q < NW; ++q) vm = fmax(vm, red_d[q]);
            const double thr = vm - cfg.tie_rel * fabs(vm);
            const int li = wave_min(a < A && myV >= thr ? a : 0x7fffffff);
            const int ti = wave_min(a < A && myV == vm ? a : 0x7fffffff);
            if (lane == 0) {
                s_wli[wave] = li;
                s_wti[wave] = ti;
            }
            if (eval && a < A) {
                if (ev.V) ev.V[a] = myV;
                if (ev.G) ev.G[a] = rbest.G;
                if (ev.I) ev.I[a] = rbest.I;
                if (ev.T) ev.T[a] = rbest.T;
            }
            lds_barrier();
            int best = 0x7fffffff, top = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                best = min(best, s_wli[q]);
                top = min(top, s_wti[q]);
            }
            if (vm == -INFINITY) best = -1;
            if (tid == 0) {
                if (eval && ev.best) *ev.best = best;
                if (!eval && best < 0) st_status = FASTMDP_NO_VALID_ACTION;
                if (!eval && n_row == 0) take_stop();
            }
            if (!eval && best >= 0 && a == best) {
                // the successor's scoring with the window's value
                Scored adv = r1;
                adv.V = myV;
                sD2[best] = d2_1;
                flush_point();                                   // the previous point keeps its counts
                for (int q = 0; q < W; ++q) st_pseenw[q] = st_seenw[q];
                advance(adv, best, top != best ? top : -1);
            }
        }
        if (!LOOK && !cert) {
            // 2-3. stage (compacted) and sweep the row chunk by chunk: every
            //      lane, one heading's climb x speed actions over a slice of the
            //      staged plans (two plans per round: v_min3)
            float ch = 0.0f, sh = 0.0f;
            float kv[NV], clf[NC];                           // per-lane sweep constants
#pragma unroll
            for (int v = 0; v < NV; ++v) kv[v] = sKv[v];
#pragma unroll
            for (int c = 0; c < NC; ++c) clf[c] = sClf[c];
            float acc[NC][NV];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[c][v] = INFINITY;
            for (int base = 0; base < n_row; base += tcap) {
                int nv;
                if (base == 0 && staged) {
                    nv = n_vis;                            // staged by the proposal path
                } else {
                    if (base > 0) {
                        lds_barrier();                     // previous chunk fully swept
                        load_chunk(row, base);
                    }
                    nv = stage_chunk(s);
                    if (base == 0 && single && !eval) {    // next row in flight during the sweep
                        pre_n = next_count();
                        if (pre_n > 0) load_chunk(row + 1, 0);
                    }
                    n_vis += nv;
                    lds_barrier();
                    if (base == 0 && tid == 0) flush_point();
                }
                if (base == 0 && sweeper) {
                    ch = (float)sCos[my_h];
                    sh = (float)sSin[my_h];
                }
                // whole rounds of 2 * n_slices plans, then one round with the
                // ragged tail (missing plans read as a plan at infinity)
                auto sweep2 = [&](const float4 p0, const float4 p1) {
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
                };
                const int full = (nv / (2 * n_slices)) * (2 * n_slices);
                if (sweeper) {
                    for (int i = my_slice; i < full; i += 2 * n_slices) sweep2(tile[i], tile[i + n_slices]);
                    if (full < nv) {
                        const float4 far = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                        const int i = full + my_slice;
                        sweep2(i < nv ? tile[i] : far, i + n_slices < nv ? tile[i + n_slices] : far);
                    }
                }
            }
            lds_barrier();                                   // tile is reused below
            if (n_row == 0 && !eval && !staged) {
                pre_n = next_count();
                if (pre_n > 0) load_chunk(row + 1, 0);
            }

            // slice partial minima, one row of A per slice
            float *red = reinterpret_cast<float *>(tile);
            if (sweeper) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int v = 0; v < NV; ++v) red[my_slice * A + (my_h * NC + c) * NV + v] = acc[c][v];
            }
            for (int w = tid; w < kMaxActions / 32; w += NT) sBand[w] = 0u;
            lds_barrier();

            // 4. per-action value, one action per thread, in FP64 (the
            //    scoring the oracle does): the nearest-plan squared distance is
            //    m + |Delta|^2 with m from the FP32 sweep.  Actions whose
            //    nearest distance lands within kBand of the well radius get it
            //    recomputed exactly in FP64 first, so that well membership is
            //    decided in FP64.  The chosen action's scoring stays in its
            //    thread's registers for the advance.
            const int a = tid;                                   // A <= kMaxActions <= NT
            Scored myr{};
            double myV = -INFINITY;
            bool myband = false;
            // a co-simulated batch: the other aircraft's wells at this
            // action's successor
            double myM = 0.0;
            if (n_mates > 0 && a < A) {
                const int h = a / (NC * NV);
                double x, y, z;
                successor(cfg, at, a, s, sCos[h], sSin[h], x, y, z);
                myM = mate_well(cfg, mates, n_mates, slot, x, y, z);
            }
            if (a < A) {
                // eight independent chains, so that eight LDS reads are in
                // flight instead of one
                float m8[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) m8[j] = INFINITY;
                // (with the range query, slices at or past the staged count
                // swept nothing)
                const int n_fold = CULL ? min(n_part, n_vis) : n_part;
                int q = 0;
                for (; q + 8 <= n_fold; q += 8) {
                    float r8[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) r8[j] = red[(q + j) * A + a];
                    // all eight values live at once: the reads are issued
                    // back to back rather than each after the previous one
                    asm volatile("" ::"v"(r8[0]), "v"(r8[1]), "v"(r8[2]), "v"(r8[3]), "v"(r8[4]), "v"(r8[5]),
                                 "v"(r8[6]), "v"(r8[7]));
#pragma unroll
                    for (int j = 0; j < 8; ++j) m8[j] = fminf(m8[j], r8[j]);
                }
                for (; q < n_fold; ++q) m8[0] = fminf(m8[0], red[q * A + a]);
                const float m = fminf(fminf(fminf(m8[0], m8[1]), fminf(m8[2], m8[3])),
                                      fminf(fminf(m8[4], m8[5]), fminf(m8[6], m8[7])));
                const double d2 = nearest_d2<NC, NV>(at, a, m);
                sD2[a] = d2;
                if (d2 > cfg.band_lo2 && d2 < cfg.band_hi2) {
                    atomicOr(&sBand[a >> 5], 1u << (a & 31));
                    myband = true;
                } else {
                    const int h = a / (NC * NV);
                    myr = score_action(cfg, tb, at, a, s, g, sCos[h], sSin[h], d2);
                    if (n_mates > 0 && myr.V > -INFINITY)       // the batch's wells join the penalties
                        myr.V = myr.G - fmax(fmax(myr.I, myM), myr.T);
                    myV = myr.V;
                }
            }

            // 5. argmax over the workgroup: the largest value vm, then the
            //    lowest index inside the tie band [vm - tie |vm|, vm], and the
            //    lowest-index largest action (kept when the choice is not the
            //    largest, for the acceptance check); DPP wave reductions, one
            //    partial per wave in LDS
            double wv = wave_max(myV);
            if (lane == 0) red_d[wave] = wv;
            if (myband) s_any = 1;
            lds_barrier();
            const int any_band = s_any;
            if (any_band) {                                      // uniform; almost never taken
                lds_barrier();                                   // every thread has read the flag
                if (tid == 0) s_any = 0;
                band_recheck(s, n_row, rb);
                if (myband) {
                    const int h = a / (NC * NV);
                    myr = score_action(cfg, tb, at, a, s, g, sCos[h], sSin[h], sD2[a]);
                    if (n_mates > 0 && myr.V > -INFINITY) myr.V = myr.G - fmax(fmax(myr.I, myM), myr.T);
                    myV = myr.V;
                }
                wv = wave_max(myV);
                if (lane == 0) red_d[wave] = wv;
                lds_barrier();
            }
            double vm = -INFINITY;
#pragma unroll
            for (int w = 0; w < NW; ++w) vm = fmax(vm, red_d[w]);
            const double thr = vm - cfg.tie_rel * fabs(vm);
            const int li = wave_min(a < A && myV >= thr ? a : 0x7fffffff);
            const int ti = wave_min(a < A && myV == vm ? a : 0x7fffffff);
            if (lane == 0) {
                s_wli[wave] = li;
                s_wti[wave] = ti;
            }
            if (eval) {
                if (a < A) {
                    if (ev.V) ev.V[a] = myr.V;
                    if (ev.G) ev.G[a] = myr.G;
                    if (ev.I) ev.I[a] = myr.I;
                    if (ev.T) ev.T[a] = myr.T;
                }
            } else if (!single) {
                pre_n = next_count();                            // in flight during the advance
                if (pre_n > 0) load_chunk(row + 1, 0);
            }
            lds_barrier();
            int best = 0x7fffffff, top = 0x7fffffff;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                best = min(best, s_wli[w]);
                top = min(top, s_wti[w]);
            }
            if (vm == -INFINITY) best = -1;
            if (tid == 0) {
                pairs += (long long)A * n_vis;                   // pairs with the plans this request sees
                if (eval && ev.best) *ev.best = best;
                if (!eval && best < 0) st_status = FASTMDP_NO_VALID_ACTION;
                if (!eval && n_row == 0) take_stop();            // no staging in this step
            }
            // top is kept when the choice is not the largest
            if constexpr (!PROP) {
                // 6. advance, by the chosen action's thread (its scoring is in
                //    its registers)
                if (!eval && best >= 0 && a == best) advance(myr, best, top != best ? top : -1);
            } else {
                // (with the proposal, thread 0 advances on every path: one
                // copy of the advance keeps that variant's registers down)
                if (best >= 0 && a == best) {
                    st_r[0] = myr.x; st_r[1] = myr.y; st_r[2] = myr.z;
                    st_r[3] = myr.V; st_r[4] = myr.I; st_r[5] = myr.clr;
                }
                if (tid == 0) {
                    st_best = best;
                    st_top = top != best ? top : -1;
                }
                lds_barrier();
            }
        }
        if constexpr (PROP) {
            // 6. advance (thread 0), from the scoring the certificate or the
            //    argmax left in st_r
            if (tid == 0 && !eval && st_best >= 0) {
                Scored r;
                r.x = st_r[0]; r.y = st_r[1]; r.z = st_r[2];
                r.V = st_r[3]; r.I = st_r[4]; r.clr = st_r[5];
                if (cert && n_row == 0) take_stop();             // no staging in this step
                advance(r, st_best, st_top);
            }
        }
        steps_here += 1;
        lds_barrier();
        if (eval) break;
    }
    if (tid == 0) flush_point();
    __syncthreads();   // st_status written by thread 0 on the way out of the loop; trajectory complete

    // Commit validation (shared with the range-query planner)
    if (!eval && validate && st_status == FASTMDP_OK) {
        const int bad = __syncthreads_or(validate_points<NT / 64>(cfg, tb, tr, pt_base, t0, st_n, seq));
        if (tid == 0) S.valid = bad == 0;
    }

    if (tid == 0 && !eval) {
        S.n_points = st_n;
        S.status = st_status;
        if (stop.target > 0 && st_status != kRunning) atomicAdd(stop.ctr, 1);
    }
    if (tid == 0) {
        S.pairs += pairs;
        S.entries += entries;
        S.steps += steps_here;
        S.cert_hit += hits;
        S.cert_miss += misses;
    }
}

// ---------------------------------------------------------------------------
// launch dispatch over the supported (climbs, speeds, zero-climb) shapes
// ---------------------------------------------------------------------------
template <int NC, int NV, int ZC>
static hipError_t launch_t(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                           const int *list, const Traj &tr, int budget, int validate, int epoch, const EvalOut &ev,
                           const PropArgs &prop, const LaunchStop &stop, const MatePeaks &mates) {
    (void)nt;
    if (c.lookahead > 1 && c.range_query)
        hipLaunchKernelGGL((planner_kernel<kPlanThreads, NC, NV, ZC, false, true, true>), dim3(nblk),
                           dim3(kPlanThreads), 0, st, c, t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);
    else if (c.lookahead > 1)
        hipLaunchKernelGGL((planner_kernel<kPlanThreads, NC, NV, ZC, false, true>), dim3(nblk), dim3(kPlanThreads), 0,
                           st, c, t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);
    else if (prop.mode == FASTMDP_PROPOSE_NONE && c.range_query)
        hipLaunchKernelGGL((planner_kernel<kPlanThreads, NC, NV, ZC, false, false, true>), dim3(nblk),
                           dim3(kPlanThreads), 0, st, c, t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);
    else if (prop.mode == FASTMDP_PROPOSE_NONE)
        hipLaunchKernelGGL((planner_kernel<kPlanThreads, NC, NV, ZC, false>), dim3(nblk), dim3(kPlanThreads), 0, st, c,
                           t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);
    else if (c.range_query)
        hipLaunchKernelGGL((planner_kernel<kPropThreads, NC, NV, ZC, true, false, true>), dim3(nblk),
                           dim3(kPropThreads), 0, st, c, t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);
    else
        hipLaunchKernelGGL((planner_kernel<kPropThreads, NC, NV, ZC, true>), dim3(nblk), dim3(kPropThreads), 0, st, c,
                           t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);
    return hipGetLastError();
}

#define FMDP_SHAPE(NC, NV, ZC) \
    if (c.n_climb == NC && c.n_speed == NV && zc == ZC) \
        return launch_t<NC, NV, ZC>(nblk, nt, st, c, t, s, list, tr, budget, validate, epoch, ev, prop, stop, mates);

hipError_t launch_planner(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                          const int *list, const Traj &tr, int budget, int validate, int epoch, const EvalOut &ev,
                          const PropArgs &prop, const LaunchStop &stop, const MatePeaks &mates) {
    const int zc = c.zero_climb;
    if (prop.mode != FASTMDP_PROPOSE_NONE && (prop.k < 1 || prop.k > FASTMDP_MAX_TOPK || prop.k > c.n_actions))
        return hipErrorInvalidValue;
    if (c.lookahead > 1 && (prop.mode != FASTMDP_PROPOSE_NONE || c.lookahead > kMaxLookahead || !tr.seenw))
        return hipErrorInvalidValue;
    const bool eval = ev.V != nullptr || ev.best != nullptr;
    if (!eval && !mates.n && uses_range_planner(c, prop.mode))
        return launch_range_planner(nblk, st, c, t, s, list, tr, budget, validate, epoch, stop);
    FMDP_PLANNER_SHAPES(FMDP_SHAPE)
    return hipErrorInvalidValue;
}

bool planner_shape_supported(int n_climb, int n_speed, int zc) {
    const int nc = n_climb, nv = n_speed;
#define FMDP_OK(NC, NV, ZC) if (nc == NC && nv == NV && zc == ZC) return true;
    FMDP_PLANNER_SHAPES(FMDP_OK)
#undef FMDP_OK
    return false;
}

}  // namespace fmdp
