// planner.h -- device-side data layout shared by the HIP translation units of
// libfastmdp (internal; the public boundary is include/fastmdp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastmdp.h"

namespace fmdp {

constexpr int kMaxActions = 1024;
constexpr int kMaxHeads = 128;
constexpr int kRunning = -1;        // slot status while a request is being planned
constexpr double kBand = 1e-3;      // metres: FP32 nearest distances this close to the well
                                    // radius are recomputed exactly in FP64

// Problem constants as the kernels use them (passed by value).
struct DevCfg {
    double box_lo[3], box_hi[3];
    double dt, ell;
    double gamma, r_goal, r_intr, R_intr, gamma_intr, R_sep, r_terr, R_terr, gamma_terr;
    double log_gamma, log_gamma_intr, log_gamma_terr;   // discounts as exp(log_gamma * distance/ell)
    double abs_r_goal, abs_r_intr, abs_r_terr;
    double climb[FASTMDP_MAX_ACT_DIM], speed[FASTMDP_MAX_ACT_DIM];
    float kv[FASTMDP_MAX_ACT_DIM];       // -2 * speed * dt
    float climb_f[FASTMDP_MAX_ACT_DIM];  // climb rates
    float zeta_scale;                    // -2 * dt
    double tie_rel;
    double reach;                        // max(R_intr, R_sep) + 1 m: a plan farther than this from
                                         // a successor cannot change its value
    int n_head, n_climb, n_speed, n_actions;
    int zero_climb;                      // index of the zero climb rate in the middle, else -1
    int max_steps;
};

// Time-major structure-of-arrays known-plan table.  Entry j of row t is at
// [t * cap + j] in X, Y, Z; rowN[t] entries are in use, in commit order.
struct DevTable {
    float *X, *Y, *Z;
    int *rowN;
    int cap, rows;
    const float *terr;                   // nullptr without terrain
    int tnx, tny;
    double tx0, ty0, tcell;
};

// One request being planned.
struct Slot {
    double origin[3], goal[3];
    int t0;
    int n_points;     // points already in the trajectory (0 = fresh request)
    int status;       // kRunning or a FASTMDP_* plan status
    int req;          // request index (host bookkeeping)
    long long pairs;  // pair evaluations, accumulated
    int steps;        // steps taken, accumulated
    int resume_at;    // FCFS check: first affected point, -1 if none
    int committed;    // FCFS sequencer: 1 once appended to the table
    int valid;        // OK trajectory passed the commit validation against the entries it saw
};

// Per-slot trajectory buffers, `stride` points per slot.  seen[k] is the
// number of entries of the row scored to produce point k (for k = 0: the
// departure row of the origin check).  top[k] is the action with the largest
// value at that step when the chosen action (the lowest index inside the
// tie band) is not itself the largest, else -1.
struct Traj {
    double *xyz;
    int *act;
    double *val;
    int *seen;
    int *top;
    int stride;
};

// Outputs of a single evaluated step (all device pointers, any may be null).
struct EvalOut {
    double *V, *G, *I, *T;
    int *best;
};

// Squared distance, in FP64, between an FP64 point and an FP32 table entry:
// the one separation arithmetic of the planner's exact checks and of commit.
__device__ __forceinline__ double entry_d2(double x, double y, double z, float px, float py, float pz) {
    const double dx = (double)px - x, dy = (double)py - y, dz = (double)pz - z;
    return dx * dx + dy * dy + dz * dz;
}

// nt: workgroup size, 256 (several requests per CU) or 1024 (one request per CU)
hipError_t launch_planner(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                          const int *list, const Traj &tr, int budget, int validate, const EvalOut &ev);
bool planner_shape_supported(int n_climb, int n_speed, int zero_climb);

// table.hip
hipError_t launch_fill_int(int *p, int value, int n, hipStream_t st);
hipError_t launch_scatter_points(const DevTable &t, const float *pts, const int *rows, const int *cols, int n,
                                 hipStream_t st);
hipError_t launch_commit_check(const DevCfg &c, const DevTable &t, const double *pts, int t0, int n, int *flag,
                               hipStream_t st);
hipError_t launch_commit_append(const DevTable &t, const double *pts, int t0, int n, const int *flag,
                                hipStream_t st);
hipError_t launch_fcfs_sequencer(const DevCfg &c, const DevTable &t, Slot *slots, const int *order, int n_order,
                                 int n_prefix, const Traj &tr, int *n_done, hipStream_t st);

}  // namespace fmdp
