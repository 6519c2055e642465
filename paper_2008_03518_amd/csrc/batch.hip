// batch.hip -- co-simulated batches: several aircraft planned together, in
// lockstep, each aware of the others and of every accepted plan (Sec. V,
// batch sizes greater than one).  Between two planner steps one wavefront
// applies the batch's own rules: the separation between the aircraft that
// just moved ("Determine terminal state"), goal capture and the step limit,
// and the peaks every aircraft still flying places along its extrapolated
// track for the others ("Build peaks"; the peak table: five risk wells at
// p + v*tau, tau in {-5, 0, 5, 10, 15} s, radius R_intr + growth*tau).
#include "planner.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace fmdp {

namespace {

__global__ __launch_bounds__(64) void batch_step_kernel(DevCfg c, Slot *slots, int n, Traj tr, BatchState bs,
                                                       int first) {
    const int i = threadIdx.x;
    __shared__ double sx[64][3];
    __shared__ int smoved[64];
    double x[3] = {0.0, 0.0, 0.0}, xp[3] = {0.0, 0.0, 0.0};
    int np = 0;
    bool moved = false;
    if (i < n) {
        np = slots[i].n_points;
        if (np > 0) {
            const double *p = tr.xyz + ((size_t)i * tr.stride + np - 1) * 3;
            x[0] = p[0]; x[1] = p[1]; x[2] = p[2];
            if (np > 1) { xp[0] = p[-3]; xp[1] = p[-2]; xp[2] = p[-1]; }
        }
        moved = !first && bs.active[i] && np > bs.prev_n[i];
    }
    sx[i][0] = x[0]; sx[i][1] = x[1]; sx[i][2] = x[2];
    smoved[i] = moved;
    __syncthreads();
    bool running = false;
    if (i < n) {
        Slot &S = slots[i];
        // two aircraft that moved in this step closer than R_sep collide
        bool hit = false;
        if (moved)
            for (int j = 0; j < n; ++j) {
                if (j == i || !smoved[j]) continue;
                const double dx = x[0] - sx[j][0], dy = x[1] - sx[j][1], dz = x[2] - sx[j][2];
                if (sqrt(dx * dx + dy * dy + dz * dz) < c.R_sep) hit = true;
            }
        if (hit) S.status = FASTMDP_REJECT_SEPARATION;
        // the start of the next step: goal capture and the step limit (the
        // planner's own tests), so that the peaks leave these aircraft out
        if (S.status == kRunning) {
            const double ex = S.goal[0] - x[0], ey = S.goal[1] - x[1], ez = S.goal[2] - x[2];
            if (sqrt(ex * ex + ey * ey + ez * ez) <= c.ell) S.status = FASTMDP_OK;
            else if (np - 1 >= c.max_steps) S.status = FASTMDP_TIMEOUT;
        }
        running = S.status == kRunning;
        bs.active[i] = running;
        bs.prev_n[i] = np;
    }
    // peaks of the aircraft still flying, in slot order
    const uint64_t bal = __ballot(running);
    if (running) {
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
        const double tau[kMatePeaks] = {-5.0, 0.0, 5.0, 10.0, 15.0};
        double v[3] = {0.0, 0.0, 0.0};
        if (np > 1)
            for (int a = 0; a < 3; ++a) v[a] = (x[a] - xp[a]) / c.dt;
        for (int m = 0; m < kMatePeaks; ++m) {
            double *pk = bs.pk + 4 * (kMatePeaks * rank + m);
            for (int a = 0; a < 3; ++a) pk[a] = x[a] + v[a] * tau[m];
            pk[3] = c.R_intr + c.peak_growth * tau[m];
            bs.owner[kMatePeaks * rank + m] = i;
        }
    }
    if (i == 0) {
        *bs.n = kMatePeaks * __popcll(bal);
        *bs.any = bal != 0;
    }
}

}  // namespace

hipError_t launch_batch_step(const DevCfg &c, Slot *slots, int n, const Traj &tr, const BatchState &bs, int first,
                             hipStream_t st) {
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_step_kernel, dim3(1), dim3(64), 0, st, c, slots, n, tr, bs, first);
    return hipGetLastError();
}

}  // namespace fmdp
