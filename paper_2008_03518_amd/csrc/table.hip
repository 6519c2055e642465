// table.hip -- known-plan table kernels: load scatter, commit validation and
// append (the accepted-plan database of Sec. V), and the first-come-first-
// served sequencer that accepts concurrently planned trajectories strictly in
// request order.
#include "planner.h"

#include <hip/hip_runtime.h>
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

__global__ void fill_int_kernel(int *p, int value, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void scatter_points_kernel(DevTable tb, const float *pts, const int *rows, const int *cols, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t idx = (size_t)rows[i] * tb.cap + cols[i];
    tb.X[idx] = pts[3 * i + 0];
    tb.Y[idx] = pts[3 * i + 1];
    tb.Z[idx] = pts[3 * i + 2];
}

// Commit validation of one trajectory point as planned (FP64) against every
// entry of its row as stored (FP32), in FP64; terrain clearance; capacity.
// flag bit 0: conflict, bit 1: capacity.
__device__ int check_point(const DevCfg &c, const DevTable &tb, const double p[3], int row, int tid, int nthr) {
    if (row >= tb.rows) return 2;
    const int n_row = tb.rowN[row];
    int f = n_row >= tb.cap ? 2 : 0;
    const double r2 = c.R_sep * c.R_sep;
    const size_t rb = (size_t)row * tb.cap;
    for (int j = tid; j < n_row; j += nthr)
        if (entry_d2(p[0], p[1], p[2], tb.X[rb + j], tb.Y[rb + j], tb.Z[rb + j]) < r2) f |= 1;
    if (tid == 0 && tb.terr && p[2] - table_terrain_height(tb, p[0], p[1]) < 0.0) f |= 1;
    return f;
}

__global__ void commit_check_kernel(DevCfg c, DevTable tb, const double *pts, int t0, int n, int *flag) {
    const int k = blockIdx.x;
    if (k >= n) return;
    const double p[3] = {pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]};
    const int f = check_point(c, tb, p, t0 + k, threadIdx.x, blockDim.x);
    if (f) atomicOr(flag, f);
}

// Append the trajectory rounded to FP32 (the table's storage format).
__global__ void commit_append_kernel(DevTable tb, const double *pts, int t0, int n, const int *flag) {
    if (*flag) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int row = t0 + k;
    const int col = tb.rowN[row];
    const size_t idx = (size_t)row * tb.cap + col;
    tb.X[idx] = (float)pts[3 * k + 0];
    tb.Y[idx] = (float)pts[3 * k + 1];
    tb.Z[idx] = (float)pts[3 * k + 2];
    tb.rowN[row] = col + 1;
}

constexpr int kSeqThreads = 1024;
constexpr int kCheckThreads = 256;

// Interaction check of one finished trajectory against the table entries
// appended after it scored their rows.  A plan committed after a row was
// scored can only add penalties, so every action's value at that step can
// only fall: the chosen action stays chosen, with the same value, unless the
// new plan changes the chosen successor's own value (or, when the choice was
// made inside the tie band, the largest action's value).  A new entry
// (entries [seen[k], rowN) of the row that produced point k) can change a
// successor's value only within the well radius of it; `reach` adds 1 m to
// cover the planner's FP32 arithmetic.  For the origin (k = 0) the test is
// the origin check.  Clean steps record the checked entries as seen.
// Returns (through *first) the first affected point, untouched if none.
__device__ void check_interactions(const DevCfg &c, const DevTable &tb, const Slot &S, const Traj &tr,
                                   size_t base, int tid, int nthr, int *first) {
    const double r2 = c.reach * c.reach;
    const int n = S.n_points, t0 = S.t0;
    for (int k = tid; k < n; k += nthr) {
        const int row = t0 + k;
        if (row >= tb.rows) continue;
        const int hi = tb.rowN[row];
        const int lo = tr.seen[base + k];
        if (lo >= hi) continue;
        const double *x = tr.xyz + (base + k) * 3;     // chosen successor (the origin for k = 0)
        double y[3] = {x[0], x[1], x[2]};              // largest action's successor, if different
        const int top = k > 0 ? tr.top[base + k] : -1;
        if (top >= 0) {
            const double *sp = tr.xyz + (base + k - 1) * 3;
            const double bx = S.goal[0] - sp[0], by = S.goal[1] - sp[1];
            const double r = sqrt(bx * bx + by * by);
            const double cb = r > 0.0 ? bx / r : 1.0, sb = r > 0.0 ? by / r : 0.0;
            const int h = top / (c.n_climb * c.n_speed);
            const int cl = (top / c.n_speed) % c.n_climb;
            const int v = top % c.n_speed;
            const double th = 2.0 * M_PI * (double)h / (double)c.n_head;
            const double c0 = cos(th), s0 = sin(th);
            const double step = c.speed[v] * c.dt;
            y[0] = sp[0] + step * (cb * c0 - sb * s0);
            y[1] = sp[1] + step * (sb * c0 + cb * s0);
            y[2] = sp[2] + c.climb[cl] * c.dt;
        }
        const size_t rb = (size_t)row * tb.cap;
        bool hit = false;
        for (int j = lo; j < hi; ++j) {
            const float px = tb.X[rb + j], py = tb.Y[rb + j], pz = tb.Z[rb + j];
            if (entry_d2(x[0], x[1], x[2], px, py, pz) < r2 || entry_d2(y[0], y[1], y[2], px, py, pz) < r2) {
                hit = true;
                break;
            }
        }
        if (hit) atomicMin(first, k);
        else tr.seen[base + k] = hi;
    }
}

__device__ void resume_from(Slot &S, int first) {
    S.resume_at = first;
    S.n_points = first;          // keep points 0..first-1; re-score from point first-1
    S.status = kRunning;
    S.committed = 0;
}

// Every finished, not yet accepted slot against everything committed so far
// (one workgroup per slot, in parallel).  An affected slot goes back to
// planning from its first affected step at once, so that re-plans overlap.
__global__ __launch_bounds__(kCheckThreads) void fcfs_check_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                   const int *order, Traj tr) {
    __shared__ int s_first;
    const int slot = order[blockIdx.x];
    Slot &S = slots[slot];
    if (threadIdx.x == 0) s_first = 0x7fffffff;
    __syncthreads();
    check_interactions(c, tb, S, tr, (size_t)slot * tr.stride, threadIdx.x, kCheckThreads, &s_first);
    __syncthreads();
    if (threadIdx.x == 0 && s_first != 0x7fffffff) resume_from(S, s_first);
}

// Acceptance in request order of the leading slots (the first n_prefix
// listed are consecutive requests; all were just checked against the table)
// up to the first one that must be re-planned.  Each is checked against the
// plans accepted earlier in this pass, then an OK trajectory that the
// planning workgroup validated against the entries it saw (Slot::valid) is
// appended if its rows have room.
__global__ __launch_bounds__(kSeqThreads) void fcfs_accept_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                  const int *order, int n_prefix, Traj tr,
                                                                  int *n_done) {
    __shared__ int s_first, s_flag;
    const int tid = threadIdx.x;
    int accepted = 0;                                      // uniform
    for (int q = 0; q < n_prefix; ++q) {
        Slot &S = slots[order[q]];
        if (S.status == kRunning) break;                  // re-planned by the check pass
        const int n = S.n_points;
        const int t0 = S.t0;
        const size_t base = (size_t)order[q] * tr.stride;
        if (tid == 0) { s_first = 0x7fffffff; s_flag = 0; }
        __syncthreads();
        check_interactions(c, tb, S, tr, base, tid, kSeqThreads, &s_first);
        __syncthreads();
        if (s_first != 0x7fffffff) {
            if (tid == 0) resume_from(S, s_first);
            break;
        }
        if (S.status == FASTMDP_OK && S.valid) {
            // entries [0, seen[k]) were validated by the planning workgroup and
            // the interaction checks cleared the rest; only capacity is left
            if (tid == 0) s_flag = (t0 + n > tb.rows) ? 2 : 0;
            __syncthreads();
            for (int k = tid; k < n && s_flag == 0; k += kSeqThreads)
                if (tb.rowN[t0 + k] >= tb.cap) atomicOr(&s_flag, 2);
            __syncthreads();
            const bool ok = s_flag == 0;
            if (ok) {
                for (int k = tid; k < n; k += kSeqThreads) {
                    const int row = t0 + k;
                    const int col = tb.rowN[row];
                    const double *x = tr.xyz + (base + k) * 3;
                    const size_t idx = (size_t)row * tb.cap + col;
                    tb.X[idx] = (float)x[0];
                    tb.Y[idx] = (float)x[1];
                    tb.Z[idx] = (float)x[2];
                    tb.rowN[row] = col + 1;
                }
            }
            if (tid == 0) {
                S.committed = ok ? 1 : 0;
                S.resume_at = ok ? -1 : -3;   // -3: table capacity
            }
        } else if (S.status == FASTMDP_OK) {
            if (tid == 0) {
                S.committed = 0;
                S.resume_at = -2;             // -2: refused by the commit validation
            }
        } else if (tid == 0) {
            S.committed = 0;
            S.resume_at = -1;
        }
        accepted = q + 1;
        __syncthreads();
    }
    if (tid == 0) *n_done = accepted;
}

}  // namespace

hipError_t launch_fill_int(int *p, int value, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_scatter_points(const DevTable &t, const float *pts, const int *rows, const int *cols, int n,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_points_kernel, dim3((n + 255) / 256), dim3(256), 0, st, t, pts, rows, cols, n);
    return hipGetLastError();
}

hipError_t launch_commit_check(const DevCfg &c, const DevTable &t, const double *pts, int t0, int n, int *flag,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(commit_check_kernel, dim3(n), dim3(256), 0, st, c, t, pts, t0, n, flag);
    return hipGetLastError();
}

hipError_t launch_commit_append(const DevTable &t, const double *pts, int t0, int n, const int *flag,
                                hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(commit_append_kernel, dim3((n + 255) / 256), dim3(256), 0, st, t, pts, t0, n, flag);
    return hipGetLastError();
}

hipError_t launch_fcfs_sequencer(const DevCfg &c, const DevTable &t, Slot *slots, const int *order, int n_order,
                                 int n_prefix, const Traj &tr, int *n_done, hipStream_t st) {
    if (n_order > 0)
        hipLaunchKernelGGL(fcfs_check_kernel, dim3(n_order), dim3(kCheckThreads), 0, st, c, t, slots, order, tr);
    hipLaunchKernelGGL(fcfs_accept_kernel, dim3(1), dim3(kSeqThreads), 0, st, c, t, slots, order, n_prefix, tr,
                       n_done);
    return hipGetLastError();
}

}  // namespace fmdp
