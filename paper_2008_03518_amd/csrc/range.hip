// range.hip -- the range-query planner for gfx950: up to four requests per
// compute unit on 256-thread workgroups, or one on a 512-thread workgroup.
//
// With the range query (Sec. VII: only the trajectories within reach of the
// state are considered) most steps find no plan within reach, and the work
// of a step is the FP64 valuation of every action, the argmax and the
// advance: a chain of short phases separated by barriers and memory round
// trips.  One request on a 1024-thread workgroup leaves the compute unit
// idle through most of that chain; here two to four requests share a compute
// unit, so that one request's waits overlap the others' work, or a request
// alone on a compute unit runs the chain on 512 threads without spilled
// registers; a step has three workgroup barriers.  Per step:
//   1. x and y of the row's entries (up to 4096 per chunk) arrive in LDS by
//      DMA while the previous step runs (with 512 threads z and visibility
//      too), and a box test against the state
//      marks candidate entries.  Its half-width exceeds the staging radius
//      by a margin that covers every rounding of the exact test, so each
//      entry the exact test keeps is a candidate;
//   2. each lane takes its candidates one per round: z and visibility are
//      read (from the table, or from LDS) and the exact test of the range query (FP64
//      offset from the state, FP32 squared distance against the staging
//      radius, visible to this request) stages the same entries as the
//      1024-thread range query, as (q_x, q_y, -2 dt q_z, |q|^2), which every
//      thread sweeps for its actions;
//   3. FP64 scoring, tie-band argmax and the trajectory record are those of
//      the 1024-thread kernel (the same functions and expressions, each
//      thread holding up to two actions, one with 512 threads), so plans,
//      values and records are
//      identical bit for bit.  Every wave publishes its candidate choice
//      with the value, flags and nearest distance, and every thread then
//      takes the step itself: the state lives in registers, and the heading
//      directions alternate between two LDS buffers, so no barrier closes
//      the step.
#include "planner.h"
#include "score.h"
#include "wave.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fmdp {

namespace {

constexpr int RAW = 4096;                    // row entries per chunk (x and y in LDS)
constexpr int HMAX = kRangeMaxHeads;

__device__ __forceinline__ int lanes_below(uint64_t bal) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
}

// NT threads per request: kRangeThreads with OCC requests resident per CU
// (kRangePerCU: up to 128 VGPRs each; 2: up to 256, no register spills), or
// kRangeThreadsSolo with one per CU (no register spills) for launches that
// hold at most one request per CU.
template <int NT, int OCC, int NC, int NV, int ZC>
__global__ __attribute__((amdgpu_flat_work_group_size(NT, NT),
                          amdgpu_waves_per_eu(NT == kRangeThreads ? OCC : 2))) void range_planner_kernel(
    DevCfg cfg, DevTable tb, Slot *slots, const int *slot_list, Traj tr, int budget, int validate, int epoch,
    LaunchStop stop) {
    constexpr int NW = NT / 64;
    constexpr int G4 = RAW / (4 * NT);           // four-entry groups per lane and chunk
    constexpr int TILE = NT;                     // staged entries per round: one candidate per thread
    constexpr int APT = kMaxActions / NT;        // actions per thread
    static_assert(RAW % (4 * NT) == 0, "a chunk is a whole number of four-entry groups per lane");
    static_assert(4 * G4 <= 32, "a lane's candidates of a chunk fit one 32-bit mask");
    static_assert(kMaxActions % NT == 0, "actions are dealt to threads in whole rounds");
    static_assert(HMAX <= NT, "one thread per heading");
    // the row chunk's x, y by DMA; alone on its CU (LDS to spare) also z
    // and visibility, so that a candidate's exact test reads no memory
    constexpr bool ZV = NT == kRangeThreadsSolo;
    __shared__ __attribute__((aligned(16))) float rawX[RAW], rawY[RAW];
    __shared__ __attribute__((aligned(16))) float rawZ[ZV ? RAW : 4];
    __shared__ __attribute__((aligned(16))) int rawV[ZV ? RAW : 4];
    __shared__ float4 tile[TILE];               // staged entries of one round; validation point list
    __shared__ double sCos[2][HMAX], sSin[2][HMAX];      // heading directions, alternate steps
    __shared__ double sStep[FASTMDP_MAX_ACT_DIM], sDz[FASTMDP_MAX_ACT_DIM];   // speed*dt, climb*dt
    __shared__ float sKv[FASTMDP_MAX_ACT_DIM], sClf[FASTMDP_MAX_ACT_DIM];      // FP32 sweep constants
    __shared__ unsigned sBand[kMaxActions / 32];
    __shared__ double red_d[NW];
    __shared__ int s_wsum[NW], s_rem[2][NW];
    __shared__ int s_wli[NW], s_wti[NW], s_wfl[NW];      // per wave: choice, largest, choice's flags
    __shared__ double s_wv[NW], s_wd2[NW];               // per wave: choice's value, nearest distance
    __shared__ int s_any, s_flag, s_stop;
    const ActTab at{sStep, sDz};

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int slot = slot_list ? slot_list[blockIdx.x] : (int)blockIdx.x;
    Slot &S = slots[slot];
    if (S.status != kRunning) return;           // a finished request (uniform: one slot per workgroup)

    const int H = cfg.n_head, A = cfg.n_actions;
    const double g[3] = {S.goal[0], S.goal[1], S.goal[2]};
    const int t0 = S.t0;
    const int seq = S.seq;
    const size_t pt_base = (size_t)slot * tr.stride;

    // this thread's heading offset 2*pi*h/H (h = tid < H)
    double c0 = 0.0, s0 = 0.0;
    if (tid < H) {
        const double th = 2.0 * M_PI * (double)tid / (double)H;
        c0 = cos(th);
        s0 = sin(th);
    }
    if (tid < FASTMDP_MAX_ACT_DIM) {
        sStep[tid] = cfg.speed[tid] * cfg.dt;
        sDz[tid] = cfg.climb[tid] * cfg.dt;
        sKv[tid] = cfg.kv[tid];
        sClf[tid] = cfg.climb_f[tid];
    }
    for (int w = tid; w < kMaxActions / 32; w += NT) sBand[w] = 0u;
    if (tid == 0) {
        s_any = 0;
        s_flag = 0;
        s_stop = 0;
    }
    // the state, the point count and the status live in every thread's
    // registers (the same values in all)
    int n = S.n_points;
    double s[3];
    if (n == 0) {
        s[0] = S.origin[0]; s[1] = S.origin[1]; s[2] = S.origin[2];
    } else {
        const double *p = tr.xyz + (pt_base + n - 1) * 3;
        s[0] = p[0]; s[1] = p[1]; s[2] = p[2];
    }
    int status = kRunning;
    __syncthreads();

    // Origin check of a fresh request: inside the box, clear of terrain, and
    // no plan active at the departure row closer than R_sep.
    if (n == 0) {
        const int n_row = t0 < tb.rows ? min(tb.rowN[t0], tb.cap) : 0;
        const size_t rb = (size_t)t0 * tb.cap;
        int hit = 0;
        for (int j = tid; j < n_row; j += NT)
            if (entry_visible(tb, rb + j, seq) &&
                entry_d2(s[0], s[1], s[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < cfg.R_sep * cfg.R_sep)
                hit = 1;
        if (hit) s_flag = 1;        // benign race: every writer stores 1
        __syncthreads();
        bool blocked = s_flag != 0 || outside_box(cfg, s[0], s[1], s[2]);
        if (tb.terr && s[2] - terrain_height(tb, s[0], s[1]) < 0.0) blocked = true;
        if (tid == 0) {
            double *p = tr.xyz + pt_base * 3;
            p[0] = s[0]; p[1] = s[1]; p[2] = s[2];
            tr.act[pt_base] = -1;
            tr.val[pt_base] = 0.0;
            tr.seen[pt_base] = n_row;
            tr.ep[pt_base] = epoch;
            tr.top[pt_base] = -1;
            tr.col[pt_base] = -1;
            tr.nd[pt_base] = INFINITY;
        }
        n = 1;
        if (blocked) status = FASTMDP_REJECT_ORIGIN;
    }

    auto row_count = [&](int row) { return (row >= 0 && row < tb.rows) ? min(tb.rowN[row], tb.cap) : 0; };
    // Entries [base, base + min(cnt - base, RAW)) of a row: x and y (and z
    // and visibility with ZV) travel
    // from the table to LDS without registers (global_load_lds), 16 bytes
    // (four entries) per lane and instruction; entry base + j lands at
    // raw*[j], in the slots of the lane that later tests it, so a wave waits
    // only for its own loads and a lane may refill its slots once it has
    // read them.  A group that runs past the row's count stays inside the
    // row's capacity (a multiple of four), so every read is in bounds.
    auto load_xy = [&](int row, int base, int cnt) {
        const size_t rb = (size_t)row * tb.cap + base;
        const int lim = min(cnt - base, RAW);
        int ofs = 4 * tid;
        asm volatile("" : "+v"(ofs));
#pragma unroll
        for (int i = 0; i < G4; ++i) {
            const int j0 = i * 4 * NT + wave * 256;        // wave-uniform LDS destination
            const int j = ofs + i * 4 * NT;
            if (j < lim) {
                load_lds16(tb.X + rb + j, rawX + j0);
                load_lds16(tb.Y + rb + j, rawY + j0);
                if constexpr (ZV) {
                    load_lds16(tb.Z + rb + j, rawZ + j0);
                    load_lds16(tb.vis + rb + j, rawV + j0);
                }
            }
        }
    };

    // rows in flight: pre_n entries of the next step's row (its x, y loading
    // into LDS) and nn, the count of the row after it
    int pre_n = 0, nn = 0;
    {
        const int row = t0 + n;
        pre_n = row_count(row);
        if (pre_n > 0) load_xy(row, 0, pre_n);
        nn = row_count(row + 1);
    }

    long long pairs = 0, entries = 0;
    int steps_here = 0, stop_v = 0, buf = 0;
    const float cbox = cfg.cull_box;
    // The point taken by a step is written to the trajectory during the
    // next step's valuation, by the last wave, which scores no action in at
    // least one round (with 360 actions or fewer) and so waits there: its
    // coordinates are the state, its value and nearest distance stay in
    // s_wv / s_wd2 of the winning wave until the next argmax, the rest in
    // registers (the same in every thread).  pend: a point is not yet written.
    int pend = 0, p_act = 0, p_seen = 0, p_top = 0, p_bw = 0;
    auto write_point = [&]() {                        // one thread
        const size_t p = pt_base + n - 1;
        tr.xyz[p * 3 + 0] = s[0];
        tr.xyz[p * 3 + 1] = s[1];
        tr.xyz[p * 3 + 2] = s[2];
        tr.val[p] = s_wv[p_bw];
        tr.nd[p] = s_wd2[p_bw];
        tr.act[p] = p_act;
        tr.seen[p] = p_seen;
        tr.top[p] = p_top;
        tr.ep[p] = epoch;
        tr.col[p] = -1;
    };
    // scoring rounds q that hold an action of this wave (wave-uniform)
    const int nq = min(APT, max(0, (A - wave * 64 + NT - 1) / NT));

    for (;;) {
        if (status != kRunning) break;                    // uniform (registers)
        const int k = n - 1;                              // steps taken so far
        const int t = t0 + k;
        {
            const double ex = g[0] - s[0], ey = g[1] - s[1], ez = g[2] - s[2];
            if (sqrt(ex * ex + ey * ey + ez * ez) <= cfg.ell) {
                status = FASTMDP_OK;
                break;
            }
            if (k >= cfg.max_steps) {
                status = FASTMDP_TIMEOUT;
                break;
            }
            if (steps_here >= budget || s_stop) break;    // resumable: stays running
        }

        // heading directions: the goal bearing rotated by each offset
        {
            const double bx = g[0] - s[0], by = g[1] - s[1];
            const double br = sqrt(bx * bx + by * by);
            const double cb = br > 0.0 ? bx / br : 1.0, sb = br > 0.0 ? by / br : 0.0;
            if (tid < H) {
                sCos[buf][tid] = cb * c0 - sb * s0;
                sSin[buf][tid] = sb * c0 + cb * s0;
            }
        }
        const double *hc = sCos[buf], *hs = sSin[buf];
        const int row = t + 1;
        const int n_row = pre_n;
        entries += n_row;                                 // (thread 0's count is the one kept)
        const size_t rb = (size_t)row * tb.cap;
        int n_vis = 0;
        float mA[APT];
#pragma unroll
        for (int i = 0; i < APT; ++i) mA[i] = INFINITY;
        const float sx = (float)s[0], sy = (float)s[1];
        // the count of the row after next and the launch stop counter, read
        // once this wave's loads of the row have landed (the wait for them
        // then does not include these reads) and in flight through the rest
        // of the step
        int nn_after = 0;
        auto read_ahead = [&]() {
            nn_after = row_count(row + 2);
            if (tid == 0 && stop.target > 0)
                stop_v = __hip_atomic_load(stop.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        if (n_row == 0) read_ahead();

        int par = 0;                                      // alternate s_rem buffer (see below)
        for (int base = 0; base < n_row; base += RAW) {  // uniform
            if (base > 0) load_xy(row, base, n_row);     // chunks after the first: loaded here
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's loads of the chunk landed
            if (base == 0) read_ahead();
            const int lim = min(n_row - base, RAW);
            // 1. box test of this lane's entries: bit 4 i + m of cm marks
            //    entry 4 tid + 4 NT i + m of the chunk
            uint32_t cm = 0u;
#pragma unroll
            for (int i = 0; i < G4; ++i) {
                const int j = 4 * tid + i * 4 * NT;
                const float4 x4 = *reinterpret_cast<const float4 *>(rawX + j);
                const float4 y4 = *reinterpret_cast<const float4 *>(rawY + j);
                const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
                const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
                uint32_t g4 = 0u;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    g4 |= (fmaxf(fabsf(xs[m] - sx), fabsf(ys[m] - sy)) <= cbox ? 1u : 0u) << m;
                const int r = lim - j;                    // entries of the group inside the chunk
                cm |= (r >= 4 ? g4 : (r > 0 ? g4 & ((1u << r) - 1u) : 0u)) << (4 * i);
            }
            // the flags of remaining candidates alternate between two
            // buffers: a buffer is rewritten only after a barrier that
            // follows every read of its previous contents
            const uint64_t any0 = __ballot(cm != 0u);
            par ^= 1;
            if (lane == 0) s_rem[par][wave] = any0 != 0;
            lds_barrier();                                // also: this step's heading directions visible
            bool more = false;
#pragma unroll
            for (int w = 0; w < NW; ++w) more = more || s_rem[par][w];
            // 2. the candidates, one per lane and round: exact test, staging,
            //    sweep of the staged entries
            while (more) {                                // uniform
                bool keep = false;
                float4 e = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
                if (cm) {
                    const int bit = __builtin_ctz(cm);
                    cm &= cm - 1u;
                    const int jj = 4 * tid + (bit >> 2) * 4 * NT + (bit & 3);
                    const size_t idx = rb + base + jj;
                    const float xs = rawX[jj], ys = rawY[jj];   // the DMA's copy of X, Y at idx
                    float zs;
                    int kv;
                    if constexpr (ZV) {
                        zs = rawZ[jj];
                        kv = rawV[jj];
                    } else {
                        zs = tb.Z[idx];
                        kv = tb.vis[idx];
                    }
                    const float qx = (float)((double)xs - s[0]);
                    const float qy = (float)((double)ys - s[1]);
                    const float qz = (float)((double)zs - s[2]);
                    const float w = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
                    e = make_float4(qx, qy, cfg.zeta_scale * qz, w);
                    keep = kv < seq && w < cfg.cull_r2;
                }
                const uint64_t kb = __ballot(keep);
                const uint64_t rem = __ballot(cm != 0u);
                par ^= 1;
                if (lane == 0) {
                    s_wsum[wave] = __popcll(kb);
                    s_rem[par][wave] = rem != 0;
                }
                lds_barrier();
                int tp = 0, tn = 0;
                more = false;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const int c = s_wsum[w];
                    tp += w < wave ? c : 0;
                    tn += c;
                    more = more || s_rem[par][w];
                }
                if (keep) tile[tp + lanes_below(kb)] = e;
                lds_barrier();
                n_vis += tn;
                // every thread's actions over the staged entries: the
                // 1024-thread sweep's FP32 expression, minimum over plans
#pragma unroll
                for (int q = 0; q < APT; ++q) {
                    const int a = tid + q * NT;
                    if (a < A && tn > 0) {
                        const int h = a / (NC * NV), c = (a / NV) % NC, v = a % NV;
                        const float ch = (float)hc[h], sh = (float)hs[h];
                        const float kvv = sKv[v], clv = sClf[c];
                        float m = mA[q];
                        for (int u = 0; u < tn; ++u) {
                            const float4 p = tile[u];
                            const float hq = fmaf(p.x, ch, p.y * sh);
                            const float uu = fmaf(kvv, hq, p.w);
                            m = fminf(m, (c == ZC) ? uu : fmaf(clv, p.z, uu));
                        }
                        mA[q] = m;
                    }
                }
                // (the next round writes the tile after its first barrier,
                // which every thread reaches after this sweep)
            }
        }
        if (n_row == 0) lds_barrier();                    // heading directions visible
        // the next step's row, in flight during the valuation (this lane's
        // slots of the chunk are read)
        pre_n = nn;
        if (pre_n > 0) load_xy(row + 1, 0, pre_n);
        nn = nn_after;

        // 3. per-action value in FP64 (the 1024-thread kernel's scoring);
        //    actions whose nearest distance lies within kBand of the well
        //    radius get it recomputed exactly first.  Kept per action: value,
        //    nearest distance and whether the successor is inside a well or
        //    below the terrain.  The rounds of a wave that holds an action in
        //    each are scored unconditionally (a past the last action reads
        //    the last one), so that their FP64 chains interleave; a round
        //    with no action of the wave is skipped.
        auto flags = [](const Scored &c) { return (c.I > 0.0 ? 1 : 0) | (c.clr < 0.0 ? 2 : 0); };
        double V[APT], d2v[APT];
        int fl[APT];
        bool band[APT];
        double vloc = -INFINITY;
        bool mine_band = false;
        auto score_rounds = [&](auto nq_c) {
            constexpr int NQ = decltype(nq_c)::value;
#pragma unroll
            for (int q = 0; q < APT; ++q) {
                const int a = tid + q * NT;
                if (q >= NQ) {                            // every action of the round is past the last
                    V[q] = -INFINITY;
                    d2v[q] = INFINITY;
                    fl[q] = 0;
                    band[q] = false;
                    continue;
                }
                const int ac = a < A ? a : A - 1;
                const int h = ac / (NC * NV);
                const double d2 = nearest_d2<NC, NV>(at, ac, mA[q]);
                d2v[q] = d2;
                band[q] = a < A && d2 > cfg.band_lo2 && d2 < cfg.band_hi2;
                const Scored c = score_action(cfg, tb, at, ac, s, g, hc[h], hs[h], d2);
                V[q] = (a < A && !band[q]) ? c.V : -INFINITY;
                fl[q] = flags(c);
                if (band[q]) atomicOr(&sBand[a >> 5], 1u << (a & 31));
                mine_band = mine_band || band[q];
                vloc = fmax(vloc, V[q]);
            }
        };
        static_assert(APT <= 2, "one or two scoring rounds");
        if (nq >= APT) score_rounds(std::integral_constant<int, APT>());
        else if (nq == 1) score_rounds(std::integral_constant<int, 1>());
        else score_rounds(std::integral_constant<int, 0>());
        if (pend) {                                       // uniform
            if (tid == NT - 64) write_point();            // the previous step's point (see above)
            pend = 0;
        }
        double wv = wave_max(vloc);
        if (lane == 0) red_d[wave] = wv;
        if (mine_band) s_any = 1;
        lds_barrier();
        if (s_any) {                                      // uniform; almost never taken
            lds_barrier();                                // every thread has read the flag
            if (tid == 0) s_any = 0;
            // exact FP64 nearest distance over the row's visible entries for
            // each flagged action; its owner thread takes the result
            for (int w = 0; w < (A + 31) / 32; ++w) {
                unsigned bits = sBand[w];
                while (bits) {
                    const int a = w * 32 + __builtin_ctz(bits);
                    bits &= bits - 1;
                    const int h = a / (NC * NV);
                    double qx, qy, qz;
                    successor(cfg, at, a, s, hc[h], hs[h], qx, qy, qz);
                    double dmin = INFINITY;
                    for (int j = tid; j < n_row; j += NT)
                        if (entry_visible(tb, rb + j, seq))
                            dmin = fmin(dmin, entry_d2(qx, qy, qz, tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]));
                    dmin = -wave_max(-dmin);
                    if (lane == 0) red_d[wave] = dmin;
                    lds_barrier();
                    if (a % NT == tid) {
                        double d2 = red_d[0];
#pragma unroll
                        for (int q = 1; q < NW; ++q) d2 = fmin(d2, red_d[q]);
#pragma unroll
                        for (int q = 0; q < APT; ++q)
                            if (q == a / NT) d2v[q] = d2;
                    }
                    lds_barrier();
                }
            }
            vloc = -INFINITY;
#pragma unroll
            for (int q = 0; q < APT; ++q) {
                const int a = tid + q * NT;
                if (band[q]) {
                    const int h = a / (NC * NV);
                    const Scored c = score_action(cfg, tb, at, a, s, g, hc[h], hs[h], d2v[q]);
                    V[q] = c.V;
                    fl[q] = flags(c);
                }
                vloc = fmax(vloc, V[q]);
            }
            wv = wave_max(vloc);
            if (lane == 0) red_d[wave] = wv;
            lds_barrier();
        }
        // argmax: the largest value vm, then the lowest index inside the tie
        // band [vm - tie |vm|, vm], and the lowest-index largest action; each
        // wave publishes its lowest candidate with what the step needs of it
        double vm = -INFINITY;
#pragma unroll
        for (int w = 0; w < NW; ++w) vm = fmax(vm, red_d[w]);
        const double thr = vm - cfg.tie_rel * fabs(vm);
        int li = 0x7fffffff, ti = 0x7fffffff;
#pragma unroll
        for (int q = APT - 1; q >= 0; --q) {              // lowest index last
            const int a = tid + q * NT;
            if (a < A && V[q] >= thr) li = a;
            if (a < A && V[q] == vm) ti = a;
        }
        li = wave_min(li);
        ti = wave_min(ti);
        if (lane == 0) {
            s_wli[wave] = li;
            s_wti[wave] = ti;
        }
#pragma unroll
        for (int q = 0; q < APT; ++q)
            if (tid + q * NT == li) {
                s_wv[wave] = V[q];
                s_wd2[wave] = d2v[q];
                s_wfl[wave] = fl[q];
            }
        if (tid == 0 && stop.target > 0) s_stop = stop_v >= stop.target;
        lds_barrier();
        int best = 0x7fffffff, top = 0x7fffffff, bw = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int l = s_wli[w];
            if (l < best) {
                best = l;
                bw = w;
            }
            top = min(top, s_wti[w]);
        }
        if (vm == -INFINITY) best = -1;
        if (best < 0) {
            status = FASTMDP_NO_VALID_ACTION;
        } else {
            // every thread takes the step: the chosen action's successor (the
            // point its scoring was computed at), recorded as the pending point
            const int h = best / (NC * NV);
            double x, y, z;
            successor(cfg, at, best, s, hc[h], hs[h], x, y, z);
            const int flb = s_wfl[bw];
            if (tid == 0) pairs += (long long)A * n_vis;  // pairs with the plans this request sees
            pend = 1;
            p_act = best;
            p_seen = n_row;
            p_top = top != best ? top : -1;
            p_bw = bw;
            s[0] = x; s[1] = y; s[2] = z;
            n += 1;
            if (flb & 1) status = FASTMDP_REJECT_SEPARATION;
            else if (flb & 2) status = FASTMDP_REJECT_TERRAIN;
        }
        // (the band bits were last read before the barrier above; the next
        // step sets them after its first barrier)
        for (int w = tid; w < kMaxActions / 32; w += NT) sBand[w] = 0u;
        buf ^= 1;
        steps_here += 1;
    }
    if (pend && tid == NT - 64) write_point();      // the last step's point
    __syncthreads();   // the trajectory complete for every thread

    // Commit validation (shared with the 1024-thread kernel)
    if (validate && status == FASTMDP_OK) {
        const int bad = __syncthreads_or(validate_points<NW>(cfg, tb, tr, pt_base, t0, n, seq));
        if (tid == 0) S.valid = bad == 0;
    }

    if (tid == 0) {
        S.n_points = n;
        S.status = status;
        if (stop.target > 0 && status != kRunning) atomicAdd(stop.ctr, 1);
        S.pairs += pairs;
        S.entries += entries;
        S.steps += steps_here;
    }
}

template <int NC, int NV, int ZC>
hipError_t launch_t(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s, const int *list,
                    const Traj &tr, int budget, int validate, int epoch, const LaunchStop &stop) {
    if (nt == kRangeThreadsSolo)
        hipLaunchKernelGGL((range_planner_kernel<kRangeThreadsSolo, 1, NC, NV, ZC>), dim3(nblk), dim3(nt), 0, st, c,
                           t, s, list, tr, budget, validate, epoch, stop);
    else if (nt == kRangeThreads && nblk <= 2 * c.n_cu)        // two per CU: no spilled registers
        hipLaunchKernelGGL((range_planner_kernel<kRangeThreads, 2, NC, NV, ZC>), dim3(nblk), dim3(nt), 0, st, c, t,
                           s, list, tr, budget, validate, epoch, stop);
    else if (nt == kRangeThreads)
        hipLaunchKernelGGL((range_planner_kernel<kRangeThreads, kRangePerCU, NC, NV, ZC>), dim3(nblk), dim3(nt), 0,
                           st, c, t, s, list, tr, budget, validate, epoch, stop);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_range_planner(int nblk, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                                const int *list, const Traj &tr, int budget, int validate, int epoch,
                                const LaunchStop &stop) {
    if (!c.range_query || c.lookahead > 1 || c.n_head > kRangeMaxHeads) return hipErrorInvalidValue;
    const int zc = c.zero_climb;
    const int nt = range_planner_threads(c, nblk);
#define FMDP_RANGE_SHAPE(NC, NV, ZC) \
    if (c.n_climb == NC && c.n_speed == NV && zc == ZC) \
        return launch_t<NC, NV, ZC>(nblk, nt, st, c, t, s, list, tr, budget, validate, epoch, stop);
    FMDP_PLANNER_SHAPES(FMDP_RANGE_SHAPE)
#undef FMDP_RANGE_SHAPE
    return hipErrorInvalidValue;
}

}  // namespace fmdp
