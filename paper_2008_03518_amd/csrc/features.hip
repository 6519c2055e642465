// features.hip -- proposal features of a batch of states (training data and
// checks of the planner's in-loop features, which use the same helpers).
#include <hip/hip_runtime.h>

#include "planner.h"
#include "proposal.h"

namespace fmdp {

// One workgroup per state: the entries of row rows[i] + 1 visible to
// sequence number seqs[i], as offsets q = p - s rounded to FP32 exactly as the
// planner stages them.
__global__ __launch_bounds__(256) void features_kernel(DevCfg c, DevTable tb, int n, const double *__restrict__ states,
                                                       const double *__restrict__ goals, const int *__restrict__ rows,
                                                       const int *__restrict__ seqs, float *__restrict__ feat) {
    __shared__ FeatAcc fa;
    const int i = blockIdx.x, tid = threadIdx.x;
    if (i >= n) return;
    feat_reset(fa, tid);
    __syncthreads();
    const double s[3] = {states[3 * i], states[3 * i + 1], states[3 * i + 2]};
    const double g[3] = {goals[3 * i], goals[3 * i + 1], goals[3 * i + 2]};
    const int row = rows[i] + 1, seq = seqs[i];
    const double bx = g[0] - s[0], by = g[1] - s[1];
    const double r = sqrt(bx * bx + by * by);
    const float ux = (float)(r > 0.0 ? bx / r : 1.0), uy = (float)(r > 0.0 ? by / r : 0.0);
    const int n_row = (row >= 0 && row < tb.rows) ? min(tb.rowN[row], tb.cap) : 0;
    const size_t rb = (size_t)(row >= 0 ? row : 0) * tb.cap;
    for (int j = tid; j < n_row; j += 256) {
        const size_t idx = rb + j;
        if (!entry_visible(tb, idx, seq)) continue;
        const float qx = (float)((double)tb.X[idx] - s[0]);
        const float qy = (float)((double)tb.Y[idx] - s[1]);
        const float qz = (float)((double)tb.Z[idx] - s[2]);
        feat_point(fa, qx, qy, qz >= 0.0f, fmaf(qx, qx, fmaf(qy, qy, qz * qz)), ux, uy);
    }
    __syncthreads();
    for (int f = tid; f < FASTMDP_N_FEAT; f += 256)
        feat[(size_t)i * FASTMDP_N_FEAT + f] = feat_value(fa, f, s, g, c.box_lo, c.box_hi, c.ell);
}

hipError_t launch_features(const DevCfg &c, const DevTable &t, int n, const double *states, const double *goals,
                           const int *rows, const int *seqs, float *feat, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(n), dim3(256), 0, st, c, t, n, states, goals, rows, seqs, feat);
    return hipGetLastError();
}

}  // namespace fmdp
