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

// Accept finished slots in the given (request) order.  For each slot:
//   1. Interaction check: every table entry appended after the slot scored a
//      row (entries [seen[k], rowN) of the row that produced point k) is
//      compared with the state the row was scored from.  An entry farther
//      than `reach` cannot change any successor's value, so if none is
//      closer the trajectory equals the one planned against the full table.
//      Otherwise the slot keeps its first k points and is re-planned from
//      there (status back to running) and the sequencer stops: later
//      requests wait for it.  For the origin (k = 0) the test is the origin
//      check itself (R_sep) and the request restarts.
//   2. An OK trajectory that the planning workgroup validated against the
//      entries it saw (Slot::valid) is appended if its rows have room.
__global__ __launch_bounds__(kSeqThreads) void fcfs_sequencer_kernel(DevCfg c, DevTable tb, Slot *slots,
                                                                     const int *order, int n_order, Traj tr,
                                                                     int *n_done) {
    __shared__ int s_first, s_flag;
    const int tid = threadIdx.x;
    int q = 0;
    for (; q < n_order; ++q) {
        Slot &S = slots[order[q]];
        const int n = S.n_points;
        const int t0 = S.t0;
        const size_t base = (size_t)order[q] * tr.stride;
        if (tid == 0) { s_first = 0x7fffffff; s_flag = 0; }
        __syncthreads();

        for (int k = tid; k < n; k += kSeqThreads) {
            const int row = t0 + k;
            if (row >= tb.rows) continue;
            const int hi = tb.rowN[row];
            const int lo = tr.seen[base + k];
            if (lo >= hi) continue;
            // state the row was scored from: the origin for k = 0 (origin
            // check), else point k-1
            const double *sp = tr.xyz + (base + (k == 0 ? 0 : k - 1)) * 3;
            const double r = k == 0 ? c.R_sep + 1.0 : c.reach;
            const size_t rb = (size_t)row * tb.cap;
            for (int j = lo; j < hi; ++j) {
                const double dx = (double)tb.X[rb + j] - sp[0];
                const double dy = (double)tb.Y[rb + j] - sp[1];
                const double dz = (double)tb.Z[rb + j] - sp[2];
                if (sqrt(dx * dx + dy * dy + dz * dz) < r) {
                    atomicMin(&s_first, k);
                    break;
                }
            }
        }
        __syncthreads();
        const int first = s_first;
        if (first != 0x7fffffff) {
            if (tid == 0) {
                S.resume_at = first;
                S.n_points = first;          // keep points 0..first-1; re-score from point first-1
                S.status = kRunning;
                S.committed = 0;
            }
            break;
        }

        if (S.status == FASTMDP_OK && S.valid) {
            // entries [0, seen[k]) were validated by the planning workgroup and
            // the interaction check above clears the rest; only capacity is left
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
        __syncthreads();
    }
    if (tid == 0) *n_done = q;
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
                                 const Traj &tr, int *n_done, hipStream_t st) {
    hipLaunchKernelGGL(fcfs_sequencer_kernel, dim3(1), dim3(kSeqThreads), 0, st, c, t, slots, order, n_order, tr,
                       n_done);
    return hipGetLastError();
}

}  // namespace fmdp
