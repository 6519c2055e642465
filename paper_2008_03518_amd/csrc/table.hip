// table.hip -- known-plan table kernels: load scatter, commit validation and
// append (the accepted-plan database of Sec. V), and the first-come-first-
// served sequencer that accepts concurrently planned trajectories strictly in
// request order.
#include "planner.h"
#include "wave.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>

namespace fmdp {

namespace {

__device__ double table_terrain_height(const DevTable &tb, double x, double y) {
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

// Order-preserving map of floats to ints (LDS integer minima of floats).
__device__ __forceinline__ int ordered_key(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float ordered_value(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

__global__ void fill_int_kernel(int *p, int value, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void copy_int_kernel(int *dst, const int *src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void scatter_points_kernel(DevTable tb, const float *pts, const int *rows, const int *cols, int n,
                                      int own) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t idx = (size_t)rows[i] * tb.cap + cols[i];
    tb.X[idx] = pts[3 * i + 0];
    tb.Y[idx] = pts[3 * i + 1];
    tb.Z[idx] = pts[3 * i + 2];
    tb.vis[idx] = own;
    tb.own[idx] = own;
    tb.dead[idx] = kAlive;
}

// Plans appended in order from one staging buffer, by one workgroup: plan j
// (t0[j], len[j] points from xyz + 3 * off) takes the next column of each row
// it spans.  A plan spans a row at most once, so its points take their
// columns independently; plans follow one another behind a barrier, which
// gives every row its entries in plan order (the columns the host-computed
// scatter of fastmdp_load_plans gives).  The row counts move by device
// atomics, which the next plan reads after the barrier.
__global__ __launch_bounds__(1024) void append_plans_kernel(DevTable tb, const int *t0, const int *len, int n,
                                                            const float *xyz) {
    long long off = 0;
    for (int j = 0; j < n; ++j) {
        const int t = t0[j], L = len[j];
        for (int k = threadIdx.x; k < L; k += blockDim.x) {
            const int row = t + k;
            const int col = atomicAdd(&tb.rowN[row], 1);
            const size_t idx = (size_t)row * tb.cap + col;
            const float *p = xyz + 3 * (off + k);
            tb.X[idx] = p[0];
            tb.Y[idx] = p[1];
            tb.Z[idx] = p[2];
            tb.vis[idx] = -1;
            tb.own[idx] = -1;
            tb.dead[idx] = kAlive;
        }
        off += L;
        __syncthreads();
    }
}

// Commit validation of one trajectory point as planned (FP64) against every
// entry of its row visible to `seq`, as stored (FP32), in FP64; terrain
// clearance; capacity.  flag bit 0: conflict, bit 1: capacity.
__device__ int check_point(const DevCfg &c, const DevTable &tb, const double p[3], int row, int seq, int tid,
                           int nthr) {
    if (row >= tb.rows) return 2;
    const int n_row = tb.rowN[row];
    int f = n_row >= tb.cap ? 2 : 0;
    const double r2 = c.R_sep * c.R_sep;
    const size_t rb = (size_t)row * tb.cap;
    for (int j = tid; j < n_row; j += nthr)
        if (entry_visible(tb, rb + j, seq) && entry_d2(p[0], p[1], p[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < r2)
            f |= 1;
    if (tid == 0 && tb.terr && p[2] - table_terrain_height(tb, p[0], p[1]) < 0.0) f |= 1;
    return f;
}

__global__ void commit_check_kernel(DevCfg c, DevTable tb, const double *pts, int t0, int n, int seq, int *flag) {
    const int k = blockIdx.x;
    if (k >= n) return;
    const double p[3] = {pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]};
    const int f = check_point(c, tb, p, t0 + k, seq, threadIdx.x, blockDim.x);
    if (f) atomicOr(flag, f);
}

// Append the trajectory rounded to FP32 (the table's storage format).
__global__ void commit_append_kernel(DevTable tb, const double *pts, int t0, int n, int own, const int *flag) {
    if (*flag) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int row = t0 + k;
    const int col = tb.rowN[row];
    const size_t idx = (size_t)row * tb.cap + col;
    tb.X[idx] = (float)pts[3 * k + 0];
    tb.Y[idx] = (float)pts[3 * k + 1];
    tb.Z[idx] = (float)pts[3 * k + 2];
    tb.vis[idx] = own;
    tb.own[idx] = own;
    tb.dead[idx] = kAlive;
    tb.rowN[row] = col + 1;
}

// ---------------------------------------------------------------------------
// First-come-first-served with concurrent requests and tentative plans.
//
// Request q (sequence number q) plans against the live table entries of
// every earlier request: plans accepted before it and the tentative
// trajectories of earlier requests that finished planning.  A finished
// trajectory with status OK enters the table at once as tentative entries
// owned by q; when q is re-planned from step k its entries from step k on are
// withdrawn (dead = epoch, logged).  Passes run between planner launches; in
// pass e (epoch e):
//   1. insert: every finished OK trajectory enters the table (missing entries);
//   2. check: every finished, not yet accepted trajectory is tested against
//      the events since it scored each row:
//        - added entries visible to it (entries [seen[k], rowN) of the row
//          that produced point k): an added plan only adds a penalty, so
//          every value at that step can only fall and the chosen action
//          stays chosen with the same value unless the plan lands within the
//          well radius of the chosen successor (or of the largest action's
//          successor when the choice was made inside the tie band);
//        - withdrawn entries it saw (logged deaths with epoch in
//          (ep[k], e-1], column < seen[k], owner < q): a withdrawal can raise
//          any successor's value, so it matters when within the well radius
//          of any successor, i.e. within `reach_state` of the scored state;
//        - for the origin (k = 0) the test is the origin check.
//      The first affected step is recorded; clean steps take seen = rowN and
//      ep = e - 1;
//   3. withdraw: an affected trajectory drops its points from the first
//      affected step on (their entries die with epoch e) and goes back to
//      planning; a finished trajectory that is not OK (or failed its commit
//      validation) withdraws all its entries.
// Acceptance (host side) walks the requests in order: a finished request
// whose checks are clean and all of whose predecessors are accepted is
// final; its tentative entries simply stay.  A request that withdrew entries
// in this pass ends the walk, because later requests have not yet been
// checked against the withdrawal.
// ---------------------------------------------------------------------------
constexpr int kPassThreads = 256;

__global__ __launch_bounds__(kPassThreads) void fcfs_insert_kernel(DevTable tb, Slot *slots, const int *list,
                                                                   Traj tr, PassBufs pb) {
    __shared__ int s_key[kRowBlocks][4];                     // the boxes as ordered keys: x, -x, y, -y minima
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;                        // still planning: not in this pass
    if (threadIdx.x == 0) S.first = 0x7fffffff;             // opened here for the checks that follow
    if (S.status != FASTMDP_OK || !S.valid) return;
    const int n = S.n_points, t0 = S.t0, own = S.seq;
    const size_t base = (size_t)slot * tr.stride;
    int err = 0, added = 0;
    for (int k = threadIdx.x; k < n; k += kPassThreads) {
        if (tr.col[base + k] >= 0) continue;
        added = 1;
        const int row = t0 + k;
        if (row >= tb.rows) { err = 1; continue; }
        const int col = atomicAdd(&tb.rowN[row], 1);
        if (col >= tb.cap) {                          // row full: undo and report
            atomicSub(&tb.rowN[row], 1);
            err = 1;
            continue;
        }
        const double *x = tr.xyz + (base + k) * 3;
        const size_t idx = (size_t)row * tb.cap + col;
        tb.X[idx] = (float)x[0];
        tb.Y[idx] = (float)x[1];
        tb.Z[idx] = (float)x[2];
        tb.vis[idx] = own;
        tb.own[idx] = own;
        tb.dead[idx] = kAlive;
        tr.col[base + k] = col;
    }
    if (err) S.err = 1;
    // a trajectory that entered entries: its row-block boxes, for the check
    // of the entries entered in this pass
    if (!__syncthreads_or(added) || n == 0) return;
    const int b0 = t0 / kRowBlock, nb = (t0 + n - 1) / kRowBlock - b0 + 1;
    for (int i = threadIdx.x; i < nb * 4; i += kPassThreads) s_key[i >> 2][i & 3] = 0x7fffffff;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += kPassThreads) {
        const double *x = tr.xyz + (base + k) * 3;
        const float fx = (float)x[0], fy = (float)x[1];            // the values the table stores
        int *key = s_key[(t0 + k) / kRowBlock - b0];
        atomicMin(&key[0], ordered_key(fx));
        atomicMin(&key[1], ordered_key(-fx));
        atomicMin(&key[2], ordered_key(fy));
        atomicMin(&key[3], ordered_key(-fy));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kPassThreads)
        pb.box[(size_t)slot * kRowBlocks + b] = make_float4(ordered_value(s_key[b][0]), -ordered_value(s_key[b][1]),
                                                            ordered_value(s_key[b][2]), -ordered_value(s_key[b][3]));
    if (threadIdx.x == 0) pb.ins_list[atomicAdd(pb.ins_n, 1)] = slot;
}

// Check, part 1: withdrawn entries the request saw; the log range is split
// over the workgroups of the request (blockIdx.y, at most kDeadSplit: one
// per kDeadPerGroup logged deaths), which fold their finds into the
// request's first-affected-step minimum (Slot::first, opened by the insert
// kernel).  The log holds each withdrawn entry's x, y and owner, so that a
// death is tested against the request's trajectory without reading the
// table: first against the bounding box (in LDS) of the block of kBoxPoints
// points holding the scored state, widened by the test radius and a margin
// above every rounding of the FP32 box (coordinates up to 1e6 m), and only
// inside it by the exact rule.
constexpr int kDeadSplit = 16;
constexpr int kDeadPerGroup = 4096;
constexpr int kBoxPoints = 64;                              // points per bounding box: one wave's round
constexpr int kMaxBoxes = kMaxPoints / kBoxPoints;
static_assert(kBoxPoints == 64 && kPassThreads % 64 == 0, "a wave's points of a round form one box");

__global__ __launch_bounds__(kPassThreads) void fcfs_check_dead_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                       const int *list, Traj tr, DeathLog dl,
                                                                       int epoch) {
    __shared__ int s_first, s_minep;
    __shared__ float s_box[kMaxBoxes][4];                   // min x, max x, min y, max y
    const int tid = threadIdx.x, lane = tid & 63;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;                        // still planning: not in this pass
    const int n = S.n_points, t0 = S.t0, q = S.seq;
    const size_t base = (size_t)slot * tr.stride;
    if (tid == 0) { s_first = 0x7fffffff; s_minep = 0x7fffffff; }
    // the oldest consistency epoch of the trajectory: a trajectory found
    // consistent throughout by the last pass has every point at epoch - 2
    if (S.clean_ep == epoch - 1) {
        if (tid == 0) s_minep = epoch - 2;
    } else {
        int mine = 0x7fffffff;
        for (int k = tid; k < n; k += kPassThreads) mine = min(mine, tr.ep[base + k]);
        atomicMin(&s_minep, mine);
    }
    __syncthreads();
    const int minep = s_minep;
    if (minep >= epoch) return;                              // uniform: nothing withdrawn since
    const int lo = dl.start[minep + 1], hi = dl.start[epoch];
    if (lo + (int)blockIdx.y * kPassThreads >= hi) return;  // uniform: no logged death for this workgroup
    // the boxes
    for (int k0 = 0; k0 < n; k0 += kPassThreads) {          // uniform
        const int k = k0 + tid;
        float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        if (k < n) {
            const double *p = tr.xyz + (base + k) * 3;
            x0 = x1 = (float)p[0];
            y0 = y1 = (float)p[1];
        }
        x0 = wave_min_f32(x0);
        x1 = wave_max_f32(x1);
        y0 = wave_min_f32(y0);
        y1 = wave_max_f32(y1);
        const int b = (k - lane) / kBoxPoints;
        if (lane == 0 && b < kMaxBoxes) {
            s_box[b][0] = x0;
            s_box[b][1] = x1;
            s_box[b][2] = y0;
            s_box[b][3] = y1;
        }
    }
    __syncthreads();
    {
        const double rs2 = c.reach_state * c.reach_state;
        const double ro2 = (c.R_sep + 1.0) * (c.R_sep + 1.0);
        const float rs = (float)c.reach_state + 1.0f, ro = (float)c.R_sep + 2.0f;
        for (int i = lo + blockIdx.y * kPassThreads + tid; i < hi; i += kPassThreads * gridDim.y) {
            const int k = dl.row[i] - t0;
            const float ex = dl.x[i], ey = dl.y[i];
            if (k < 0 || k >= n) continue;
            const float *bx = s_box[(k == 0 ? 0 : k - 1) / kBoxPoints];
            const float m = (k == 0 ? ro : rs) + 1e-6f * (fabsf(ex) + fabsf(ey));
            if (ex < bx[0] - m || ex > bx[1] + m || ey < bx[2] - m || ey > bx[3] + m) continue;
            const int col = dl.col[i], e = dl.ep[i];
            if (col >= tr.seen[base + k] || e <= tr.ep[base + k] || dl.own[i] >= q) continue;
            const size_t idx = (size_t)dl.row[i] * tb.cap + col;
            const double *sp = tr.xyz + (base + (k == 0 ? 0 : k - 1)) * 3;
            if (entry_d2(sp[0], sp[1], sp[2], ex, ey, tb.Z[idx]) < (k == 0 ? ro2 : rs2))
                atomicMin(&s_first, k);
        }
    }
    __syncthreads();
    if (tid == 0 && s_first != 0x7fffffff) atomicMin(&S.first, s_first);
}

// Check, part 2: added entries.  Those entered before this pass (entries
// [seen[k], rowN_pre) of row t0 + k, for each point k: the part a request
// that was checked in the last pass no longer has) are scanned here; those
// entered in this pass are checked trajectory against trajectory below.
// kCheckPoints points of one request at a time
// per workgroup (blockIdx.y picks the first chunk of points, then every
// gridDim.y-th).  Each wave takes one point at a time; its lanes read x and
// y of kAddLoads x 64 of the row's new entries at once and test them
// against boxes around the point's one or two successors (half-width reach,
// widened by a margin above every rounding of the FP32 box for coordinates
// up to 1e6 m); only entries inside a box are read further and tested
// exactly.  The wave stops at the first point with an entry in reach (its
// later points cannot be the first affected one).
constexpr int kCheckPoints = 64;
constexpr int kAddSplit = 8;
constexpr int kAddLoads = 4;

// The successor the added-entry rule tests besides the chosen one x_k
// (point k): the largest action's, when the step to point k chose inside
// the tie band (top_k >= 0), else x_k itself.
__device__ __forceinline__ void top_successor(const DevCfg &c, const Slot &S, const Traj &tr, size_t base, int k,
                                              int top_k, double y[3]) {
    const double *x = tr.xyz + (base + k) * 3;
    y[0] = x[0];
    y[1] = x[1];
    y[2] = x[2];
    if (top_k < 0) return;
    const double *sp = tr.xyz + (base + k - 1) * 3;
    const double bx = S.goal[0] - sp[0], by = S.goal[1] - sp[1];
    const double r = sqrt(bx * bx + by * by);
    const double cb = r > 0.0 ? bx / r : 1.0, sb = r > 0.0 ? by / r : 0.0;
    const int h = top_k / (c.n_climb * c.n_speed);
    const int cl = (top_k / c.n_speed) % c.n_climb;
    const int v = top_k % c.n_speed;
    const double th = 2.0 * M_PI * (double)h / (double)c.n_head;
    const double c0 = cos(th), s0 = sin(th);
    const double step = c.speed[v] * c.dt;
    y[0] = sp[0] + step * (cb * c0 - sb * s0);
    y[1] = sp[1] + step * (sb * c0 + cb * s0);
    y[2] = sp[2] + c.climb[cl] * c.dt;
}

__global__ __launch_bounds__(kPassThreads) void fcfs_check_add_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                      const int *list, Traj tr, PassBufs pb,
                                                                      int epoch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;                        // still planning: not in this pass
    // checked throughout in the last pass: it saw every entry entered before
    // this one (its rows' counts then are this pass's counts before insertion)
    if (S.clean_ep == epoch - 1) return;
    const int n = S.n_points, t0 = S.t0, q = S.seq;
    const size_t base = (size_t)slot * tr.stride;
    const double r2 = c.reach * c.reach;
    const float reach_f = (float)c.reach + 1.0f;
    constexpr int per_wave = kCheckPoints / (kPassThreads / 64);
    static_assert(per_wave <= 64, "one lane per point of the wave");
    for (int k0 = blockIdx.y * kCheckPoints; k0 < n; k0 += gridDim.y * kCheckPoints) {
        // the bookkeeping of the wave's points, one lane each, read at once;
        // then only the points whose row gained entries are scanned, in order
        const int kl = k0 + wave * per_wave + lane;
        int lo = 0, hi = 0, top = -1;
        if (lane < per_wave && kl < n && t0 + kl < tb.rows) {
            hi = min(pb.rowN_pre[t0 + kl], tb.cap);
            lo = tr.seen[base + kl];
            top = kl > 0 ? tr.top[base + kl] : -1;
        }
        uint64_t todo = __ballot(lane < per_wave && lo < hi);
        while (todo) {                                        // wave-uniform
            const int i = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int k = k0 + wave * per_wave + i;
            const int row = t0 + k;
            const int lo_k = __builtin_amdgcn_readlane(lo, i), hi_k = __builtin_amdgcn_readlane(hi, i);
            const int top_k = __builtin_amdgcn_readlane(top, i);
            const double *x = tr.xyz + (base + k) * 3;         // chosen successor (the origin for k = 0)
            double y[3];                                       // largest action's successor, if different
            top_successor(c, S, tr, base, k, top_k, y);
            const float ax = (float)x[0], ay = (float)x[1], bx = (float)y[0], by = (float)y[1];
            const float m = reach_f + 1e-6f * fmaxf(fmaxf(fabsf(ax), fabsf(ay)), fmaxf(fabsf(bx), fabsf(by)));
            const size_t rb = (size_t)row * tb.cap;
            int hit = 0;
            for (int jb = lo_k; jb < hi_k; jb += 64 * kAddLoads) {   // uniform
                float ex[kAddLoads], ey[kAddLoads];
#pragma unroll
                for (int u = 0; u < kAddLoads; ++u) {
                    const int j = jb + 64 * u + lane;
                    ex[u] = INFINITY;
                    ey[u] = INFINITY;
                    if (j < hi_k) {
                        ex[u] = tb.X[rb + j];
                        ey[u] = tb.Y[rb + j];
                    }
                }
                bool cand[kAddLoads], any = false;
#pragma unroll
                for (int u = 0; u < kAddLoads; ++u) {
                    cand[u] = (fabsf(ex[u] - ax) <= m && fabsf(ey[u] - ay) <= m) ||
                              (fabsf(ex[u] - bx) <= m && fabsf(ey[u] - by) <= m);
                    any = any || cand[u];
                }
                if (__ballot(any)) {                            // uniform; rare
#pragma unroll
                    for (int u = 0; u < kAddLoads; ++u) {
                        const size_t idx = rb + jb + 64 * u + lane;
                        if (cand[u] && entry_visible(tb, idx, q)) {
                            const float ez = tb.Z[idx];
                            hit |= entry_d2(x[0], x[1], x[2], ex[u], ey[u], ez) < r2 ||
                                   entry_d2(y[0], y[1], y[2], ex[u], ey[u], ez) < r2;
                        }
                    }
                    if (__ballot(hit)) break;
                }
            }
            if (__ballot(hit)) {
                if (lane == 0) atomicMin(&S.first, k);
                return;                                         // later points of this wave cannot be first
            }
        }
    }
}

// Check, part 2b: the entries entered in this pass, trajectory against
// trajectory.  Each entered a point of a trajectory in the pass's list of
// inserting slots, at a column at or past the row's count before the pass.
// The request's scored states are boxed per block of kRowBlock rows (in
// LDS); a block of an inserted trajectory of an earlier request whose box
// comes within reach + the longest step (+ 1 m and 1e-6 |coordinate| for
// the FP32 boxes) of the request's box is a candidate, and a wave then
// tests its rows, one per lane, by the added-entry rule: the entry in reach
// of the chosen successor or of the largest action's.  Outside such blocks
// no entry can be in reach of a successor of the request.
constexpr int kNewCand = 4 * kPassThreads;             // (trajectory, block) pairs tested per round

__global__ __launch_bounds__(kPassThreads) void fcfs_check_new_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                      const int *list, Traj tr, PassBufs pb) {
    __shared__ int s_key[kRowBlocks][4];                  // scored states' boxes as ordered keys
    __shared__ float s_box[kRowBlocks][4];                // x min, x max, y min, y max
    __shared__ int2 s_cand[kNewCand];                     // (inserting slot, block)
    __shared__ int s_nc, s_first;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;                        // still planning: not in this pass
    const int n_ins = *pb.ins_n;
    const int n = S.n_points, t0 = S.t0, q = S.seq;
    if (n_ins == 0 || n == 0) return;                        // uniform
    const size_t base = (size_t)slot * tr.stride;
    const int b0 = t0 / kRowBlock, nb = (t0 + n - 1) / kRowBlock - b0 + 1;
    for (int i = tid; i < nb * 4; i += kPassThreads) s_key[i >> 2][i & 3] = 0x7fffffff;
    if (tid == 0) {
        s_nc = 0;
        s_first = 0x7fffffff;
    }
    __syncthreads();
    for (int k = tid; k < n; k += kPassThreads) {
        const double *x = tr.xyz + (base + (k == 0 ? 0 : k - 1)) * 3;   // the state point k was scored from
        const float fx = (float)x[0], fy = (float)x[1];
        int *key = s_key[(t0 + k) / kRowBlock - b0];
        atomicMin(&key[0], ordered_key(fx));
        atomicMin(&key[1], ordered_key(-fx));
        atomicMin(&key[2], ordered_key(fy));
        atomicMin(&key[3], ordered_key(-fy));
    }
    __syncthreads();
    for (int b = tid; b < nb; b += kPassThreads) {
        s_box[b][0] = ordered_value(s_key[b][0]);
        s_box[b][1] = -ordered_value(s_key[b][1]);
        s_box[b][2] = ordered_value(s_key[b][2]);
        s_box[b][3] = -ordered_value(s_key[b][3]);
    }
    __syncthreads();
    const double r2 = c.reach * c.reach;
    const float reach_f = (float)(c.reach + c.max_step) + 1.0f;
    const int total = n_ins * nb;
    for (int c0 = 0; c0 < total; c0 += kNewCand) {            // uniform
        // 1. box against box
        for (int i = c0 + tid; i < min(total, c0 + kNewCand); i += kPassThreads) {
            const int pi = i / nb, b = i - pi * nb;
            const int ps = pb.ins_list[pi];
            const Slot &P = slots[ps];
            if (P.seq >= q) continue;                          // not visible to this request
            const int pb0 = P.t0 / kRowBlock, pnb = (P.t0 + P.n_points - 1) / kRowBlock - pb0 + 1;
            const int bb = b0 + b - pb0;
            if (bb < 0 || bb >= pnb) continue;
            const float4 e = pb.box[(size_t)ps * kRowBlocks + bb];
            const float *qb = s_box[b];
            if (!(qb[0] <= qb[1])) continue;                   // no point of the request in this block
            const float m = reach_f + 1e-6f * fmaxf(fmaxf(fabsf(qb[0]), fabsf(qb[1])), fmaxf(fabsf(qb[2]), fabsf(qb[3])));
            if (e.x > qb[1] + m || e.y < qb[0] - m || e.z > qb[3] + m || e.w < qb[2] - m) continue;
            s_cand[atomicAdd(&s_nc, 1)] = make_int2(ps, b);
        }
        __syncthreads();
        // 2. the candidate blocks' rows, one per lane
        const int nc = s_nc;
        for (int ci = wave; ci < nc; ci += kPassThreads / 64) {
            const int ps = s_cand[ci].x;
            const int r = (b0 + s_cand[ci].y) * kRowBlock + lane;
            const Slot &P = slots[ps];
            const int k = r - t0, kp = r - P.t0;
            if (k < 0 || k >= n || kp < 0 || kp >= P.n_points || r >= tb.rows) continue;
            const int col = tr.col[(size_t)ps * tr.stride + kp];
            if (col < pb.rowN_pre[r] || col >= tb.cap) continue;      // entered before this pass (or none)
            const size_t idx = (size_t)r * tb.cap + col;
            if (!entry_visible(tb, idx, q)) continue;
            const double *x = tr.xyz + (base + k) * 3;
            double y[3];
            top_successor(c, S, tr, base, k, k > 0 ? tr.top[base + k] : -1, y);
            const float px = tb.X[idx], py = tb.Y[idx], pz = tb.Z[idx];
            if (entry_d2(x[0], x[1], x[2], px, py, pz) < r2 || entry_d2(y[0], y[1], y[2], px, py, pz) < r2)
                atomicMin(&s_first, k);
        }
        __syncthreads();
        if (tid == 0) s_nc = 0;
        __syncthreads();
    }
    if (tid == 0 && s_first != 0x7fffffff) atomicMin(&S.first, s_first);
}

// Lookahead window W > 1: the step to point k (from point k-1 at row
// t0 + k - 1) scored rows t0 + k - 1 + w, w = 1..W, and recorded the entry
// counts it saw in seenw.  The same two rules per window row: an added entry
// matters within reach of the chosen action's window point w (or of the
// largest action's, when the choice was made inside the tie band), a
// withdrawn one within reach of any action's point w, i.e. within
// reach + w * max_step of point k - 1.  The origin (k = 0) is the origin
// check, as without the window.

// Window point w of action a from state sp (the action's heading is an
// offset from the goal bearing at sp).
__device__ void table_window_point(const DevCfg &c, const double sp[3], const double goal[3], int a, int w,
                                   double y[3]) {
    const double bx = goal[0] - sp[0], by = goal[1] - sp[1];
    const double r = sqrt(bx * bx + by * by);
    const double cb = r > 0.0 ? bx / r : 1.0, sb = r > 0.0 ? by / r : 0.0;
    const int h = a / (c.n_climb * c.n_speed);
    const int cl = (a / c.n_speed) % c.n_climb;
    const int v = a % c.n_speed;
    const double th = 2.0 * M_PI * (double)h / (double)c.n_head;
    const double c0 = cos(th), s0 = sin(th);
    const double k = (double)w;
    const double step = k * (c.speed[v] * c.dt);
    y[0] = sp[0] + step * (cb * c0 - sb * s0);
    y[1] = sp[1] + step * (sb * c0 + cb * s0);
    y[2] = sp[2] + k * (c.climb[cl] * c.dt);
}

__global__ __launch_bounds__(kPassThreads) void fcfs_check_dead_window_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                              const int *list, Traj tr, DeathLog dl,
                                                                              int epoch) {
    __shared__ int s_first, s_minep;
    const int tid = threadIdx.x;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;
    const int n = S.n_points, t0 = S.t0, q = S.seq, W = c.lookahead;
    const size_t base = (size_t)slot * tr.stride;
    if (tid == 0) { s_first = 0x7fffffff; s_minep = 0x7fffffff; }
    __syncthreads();
    int mine = 0x7fffffff;
    for (int k = tid; k < n; k += kPassThreads) mine = min(mine, tr.ep[base + k]);
    atomicMin(&s_minep, mine);
    __syncthreads();
    const int minep = s_minep;
    if (minep < epoch) {
        const int lo = dl.start[minep + 1], hi = dl.start[epoch];
        const double ro2 = (c.R_sep + 1.0) * (c.R_sep + 1.0);
        for (int i = lo + blockIdx.y * kPassThreads + tid; i < hi; i += kPassThreads * gridDim.y) {
            const int row = dl.row[i], col = dl.col[i], e = dl.ep[i];
            const size_t idx = (size_t)row * tb.cap + col;
            if (tb.own[idx] >= q) continue;
            const int r = row - t0;
            if (r == 0 && n > 0 && col < tr.seen[base] && e > tr.ep[base]) {      // the origin check
                const double *o = tr.xyz + base * 3;
                if (entry_d2(o[0], o[1], o[2], tb.X[idx], tb.Y[idx], tb.Z[idx]) < ro2) atomicMin(&s_first, 0);
            }
            for (int w = 1; w <= W; ++w) {
                const int k = r - w + 1;                  // the step to point k scored this row as point w
                if (k < 1 || k >= n) continue;
                if (col >= tr.seenw[(base + k) * W + w - 1] || e <= tr.ep[base + k]) continue;
                const double *sp = tr.xyz + (base + k - 1) * 3;
                const double rw = c.reach + w * c.max_step;
                if (entry_d2(sp[0], sp[1], sp[2], tb.X[idx], tb.Y[idx], tb.Z[idx]) < rw * rw) atomicMin(&s_first, k);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && s_first != 0x7fffffff) atomicMin(&S.first, s_first);
}

// Added entries, window W > 1: one wave per point at a time, its lanes over
// the new entries of each window row; the wave stops at the first entry in
// reach.
__global__ __launch_bounds__(kPassThreads) void fcfs_check_add_window_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                             const int *list, Traj tr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;
    const int n = S.n_points, t0 = S.t0, q = S.seq, W = c.lookahead;
    const int k0 = blockIdx.y * kCheckPoints;
    if (k0 >= n) return;
    const size_t base = (size_t)slot * tr.stride;
    const double r2 = c.reach * c.reach;
    constexpr int per_wave = kCheckPoints / (kPassThreads / 64);
    for (int i = 0; i < per_wave; ++i) {
        const int k = k0 + wave * per_wave + i;
        if (k >= n) break;
        int hit = 0;
        if (k == 0) {                                     // the origin check: row t0 against R_sep + 1 m
            const int row = t0;
            if (row < tb.rows) {
                const int lo = tr.seen[base], hi = min(tb.rowN[row], tb.cap);
                const double *x = tr.xyz + base * 3;
                const size_t rb = (size_t)row * tb.cap;
                for (int j = lo + lane; j < hi && !hit; j += 64)
                    hit = entry_visible(tb, rb + j, q) &&
                          entry_d2(x[0], x[1], x[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < r2;
            }
        } else {
            const double *sp = tr.xyz + (base + k - 1) * 3, *sk = tr.xyz + (base + k) * 3;
            const int top = tr.top[base + k];
            for (int w = 1; w <= W && !__ballot(hit); ++w) {
                const int row = t0 + k - 1 + w;
                if (row >= tb.rows) break;
                const int lo = tr.seenw[(base + k) * W + w - 1], hi = min(tb.rowN[row], tb.cap);
                if (lo >= hi) continue;
                // the chosen action's point w lies on the line through points k-1 and k
                const double y[3] = {sp[0] + w * (sk[0] - sp[0]), sp[1] + w * (sk[1] - sp[1]),
                                     sp[2] + w * (sk[2] - sp[2])};
                double u[3] = {y[0], y[1], y[2]};
                if (top >= 0) table_window_point(c, sp, S.goal, top, w, u);
                const size_t rb = (size_t)row * tb.cap;
                for (int j = lo + lane; j < hi && !hit; j += 64) {
                    if (!entry_visible(tb, rb + j, q)) continue;
                    const float px = tb.X[rb + j], py = tb.Y[rb + j], pz = tb.Z[rb + j];
                    hit = entry_d2(y[0], y[1], y[2], px, py, pz) < r2 || entry_d2(u[0], u[1], u[2], px, py, pz) < r2;
                }
            }
        }
        if (__ballot(hit)) {
            if (lane == 0) atomicMin(&S.first, k);
            break;                                        // later points of this wave cannot be first
        }
    }
}

__global__ __launch_bounds__(kPassThreads) void fcfs_check_finish_window_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                                const int *list, Traj tr, int epoch) {
    const int tid = threadIdx.x;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;
    const int n = S.n_points, t0 = S.t0, first = S.first, W = c.lookahead;
    const size_t base = (size_t)slot * tr.stride;
    for (int k = tid; k < min(n, first); k += kPassThreads) {
        const int row = t0 + k;
        if (row < tb.rows) tr.seen[base + k] = min(tb.rowN[row], tb.cap);
        if (k > 0)
            for (int w = 1; w <= W; ++w) {
                const int rw = t0 + k - 1 + w;
                tr.seenw[(base + k) * W + w - 1] = rw < tb.rows ? min(tb.rowN[rw], tb.cap) : 0;
            }
        tr.ep[base + k] = epoch - 1;
    }
    if (tid == 0) {
        S.resume_at = first == 0x7fffffff ? -1 : first;
        S.clean_ep = first == 0x7fffffff ? epoch : -1;
    }
}

// Check, part 3 (one workgroup per request): steps before the first
// affected one are consistent with the table now.
__global__ __launch_bounds__(kPassThreads) void fcfs_check_finish_kernel(DevTable tb, Slot *slots, const int *list,
                                                                         Traj tr, int epoch) {
    const int tid = threadIdx.x;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;                        // still planning: not in this pass
    const int n = S.n_points, t0 = S.t0, first = S.first;
    const size_t base = (size_t)slot * tr.stride;
    for (int k = tid; k < min(n, first); k += kPassThreads) {
        const int row = t0 + k;
        if (row < tb.rows) tr.seen[base + k] = min(tb.rowN[row], tb.cap);
        tr.ep[base + k] = epoch - 1;
    }
    if (tid == 0) {
        S.resume_at = first == 0x7fffffff ? -1 : first;
        S.clean_ep = first == 0x7fffffff ? epoch : -1;
    }
}

__global__ __launch_bounds__(kPassThreads) void fcfs_withdraw_kernel(DevTable tb, Slot *slots, const int *list,
                                                                     Traj tr, DeathLog dl, int epoch) {
    __shared__ int s_killed;
    const int tid = threadIdx.x;
    const int slot = list[blockIdx.x];
    Slot &S = slots[slot];
    if (S.status == kRunning) return;                        // still planning: not in this pass
    const int n = S.n_points, t0 = S.t0;
    const size_t base = (size_t)slot * tr.stride;
    int from = n;
    if (S.resume_at >= 0) from = S.resume_at;
    else if (S.status != FASTMDP_OK || !S.valid) from = 0;
    if (tid == 0) s_killed = 0;
    __syncthreads();
    int killed = 0, err = 0;
    for (int k = from + tid; k < n; k += kPassThreads) {
        const int col = tr.col[base + k];
        if (col < 0) continue;
        const int row = t0 + k;
        tb.dead[(size_t)row * tb.cap + col] = epoch;
        tb.vis[(size_t)row * tb.cap + col] = kAlive;
        const int i = atomicAdd(dl.len, 1);
        if (i < dl.cap) {
            const size_t idx = (size_t)row * tb.cap + col;
            dl.row[i] = row;
            dl.col[i] = col;
            dl.ep[i] = epoch;
            dl.x[i] = tb.X[idx];
            dl.y[i] = tb.Y[idx];
            dl.own[i] = tb.own[idx];
        } else {
            err = 1;
        }
        tr.col[base + k] = -1;
        killed = 1;
    }
    if (killed) s_killed = 1;
    __syncthreads();
    if (tid == 0) {
        S.killed = s_killed;
        if (err) S.err = 1;
        if (S.resume_at >= 0) {
            S.n_points = S.resume_at;   // keep points 0..resume_at-1; re-score from the last kept point
            S.status = kRunning;
            S.valid = 0;
            S.resumes += 1;
            S.clean_ep = -1;
        }
    }
}

// An interrupted call: every table entry of the listed slots (requests that
// were admitted but not accepted) is withdrawn, whatever their state, so
// that only accepted plans stay visible.  Only entries owned by sequence
// numbers from min_own on (the unaccepted requests) are touched.
__global__ __launch_bounds__(kPassThreads) void fcfs_abort_kernel(DevTable tb, Slot *slots, const int *list, Traj tr,
                                                                  int min_own, int epoch) {
    const int slot = list[blockIdx.x];
    const Slot &S = slots[slot];
    const int n = min(S.n_points, tr.stride), t0 = S.t0;
    const size_t base = (size_t)slot * tr.stride;
    for (int k = threadIdx.x; k < n; k += kPassThreads) {
        const int col = tr.col[base + k];
        const int row = t0 + k;
        if (col < 0 || col >= tb.cap || row >= tb.rows) continue;
        if (tb.own[(size_t)row * tb.cap + col] < min_own) continue;
        tb.dead[(size_t)row * tb.cap + col] = epoch;
        tb.vis[(size_t)row * tb.cap + col] = kAlive;
        tr.col[base + k] = -1;
    }
}

// Pack the trajectories of the listed slots into one buffer for a single
// device-to-host copy: slot list[i]'s n_points points go to point offset
// off[i]; xyz (3 doubles), then action, then value per point, in three
// contiguous sections of `total` points each.
__global__ void gather_traj_kernel(const Slot *slots, const int *list, const long long *off, long long total, Traj tr,
                                   double *xyz, int *act, double *val) {
    const int slot = list[blockIdx.x];
    const int n = slots[slot].n_points;
    const long long o = off[blockIdx.x];
    const size_t base = (size_t)slot * tr.stride;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        xyz[(o + k) * 3 + 0] = tr.xyz[(base + k) * 3 + 0];
        xyz[(o + k) * 3 + 1] = tr.xyz[(base + k) * 3 + 1];
        xyz[(o + k) * 3 + 2] = tr.xyz[(base + k) * 3 + 2];
        act[o + k] = tr.act[base + k];
        val[o + k] = tr.val[base + k];
    }
}

}  // namespace

hipError_t launch_gather_traj(const Slot *slots, const int *list, int n_list, const long long *off, long long total,
                              const Traj &tr, void *dst, hipStream_t st) {
    if (n_list <= 0) return hipSuccess;
    double *xyz = static_cast<double *>(dst);
    double *val = xyz + 3 * total;
    int *act = reinterpret_cast<int *>(val + total);
    hipLaunchKernelGGL(gather_traj_kernel, dim3(n_list), dim3(256), 0, st, slots, list, off, total, tr, xyz, act, val);
    return hipGetLastError();
}

hipError_t launch_fcfs_abort(const DevTable &t, Slot *slots, const int *list, int n_list, const Traj &tr, int min_own,
                             int epoch, hipStream_t st) {
    if (n_list <= 0) return hipSuccess;
    hipLaunchKernelGGL(fcfs_abort_kernel, dim3(n_list), dim3(kPassThreads), 0, st, t, slots, list, tr, min_own, epoch);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int value, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_append_plans(const DevTable &t, const int *t0, const int *len, int n, const float *xyz,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(append_plans_kernel, dim3(1), dim3(1024), 0, st, t, t0, len, n, xyz);
    return hipGetLastError();
}

hipError_t launch_scatter_points(const DevTable &t, const float *pts, const int *rows, const int *cols, int n,
                                 int own, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_points_kernel, dim3((n + 255) / 256), dim3(256), 0, st, t, pts, rows, cols, n, own);
    return hipGetLastError();
}

hipError_t launch_commit_check(const DevCfg &c, const DevTable &t, const double *pts, int t0, int n, int seq,
                               int *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(commit_check_kernel, dim3(n), dim3(256), 0, st, c, t, pts, t0, n, seq, flag);
    return hipGetLastError();
}

hipError_t launch_commit_append(const DevTable &t, const double *pts, int t0, int n, int own, const int *flag,
                                hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(commit_append_kernel, dim3((n + 255) / 256), dim3(256), 0, st, t, pts, t0, n, own, flag);
    return hipGetLastError();
}

hipError_t launch_fcfs_pass(const DevCfg &c, const DevTable &t, Slot *slots, const int *list, int n_list,
                            const Traj &tr, const DeathLog &dl, const PassBufs &pb, int epoch, int dl_len,
                            hipStream_t st) {
    if (n_list <= 0) return hipSuccess;
    const int dead_split = std::min(kDeadSplit, std::max(1, (dl_len + kDeadPerGroup - 1) / kDeadPerGroup));
    // the row counts before this pass's insertions; no slot inserted yet
    hipLaunchKernelGGL(copy_int_kernel, dim3((t.rows + 255) / 256), dim3(256), 0, st, pb.rowN_pre, t.rowN, t.rows);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(256), 0, st, pb.ins_n, 0, 1);
    hipLaunchKernelGGL(fcfs_insert_kernel, dim3(n_list), dim3(kPassThreads), 0, st, t, slots, list, tr, pb);
    if (c.lookahead > 1) {
        if (!tr.seenw) return hipErrorInvalidValue;
        hipLaunchKernelGGL(fcfs_check_dead_window_kernel, dim3(n_list, dead_split), dim3(kPassThreads), 0, st, c, t,
                           slots, list, tr, dl, epoch);
        hipLaunchKernelGGL(fcfs_check_add_window_kernel, dim3(n_list, (tr.stride + kCheckPoints - 1) / kCheckPoints),
                           dim3(kPassThreads), 0, st, c, t, slots, list, tr);
        hipLaunchKernelGGL(fcfs_check_finish_window_kernel, dim3(n_list), dim3(kPassThreads), 0, st, c, t, slots, list,
                           tr, epoch);
    } else {
        hipLaunchKernelGGL(fcfs_check_dead_kernel, dim3(n_list, dead_split), dim3(kPassThreads), 0, st, c, t, slots,
                           list, tr, dl, epoch);
        hipLaunchKernelGGL(fcfs_check_add_kernel, dim3(n_list, kAddSplit), dim3(kPassThreads), 0, st, c, t, slots,
                           list, tr, pb, epoch);
        hipLaunchKernelGGL(fcfs_check_new_kernel, dim3(n_list), dim3(kPassThreads), 0, st, c, t, slots, list, tr, pb);
        hipLaunchKernelGGL(fcfs_check_finish_kernel, dim3(n_list), dim3(kPassThreads), 0, st, t, slots, list, tr,
                           epoch);
    }
    hipLaunchKernelGGL(fcfs_withdraw_kernel, dim3(n_list), dim3(kPassThreads), 0, st, t, slots, list, tr, dl, epoch);
    return hipGetLastError();
}

}  // namespace fmdp
