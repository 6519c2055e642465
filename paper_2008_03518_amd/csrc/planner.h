// planner.h -- device-side data layout shared by the HIP translation units of
// libfastmdp (internal; the public boundary is include/fastmdp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastmdp.h"

namespace fmdp {

constexpr int kPlanThreads = 1024;  // planning workgroup: one request per CU, 16 wave64
constexpr int kPropThreads = 512;   // with the proposal path: 8 wave64, twice the registers per lane
constexpr int kRangeThreads = 256;  // range-query planner: 4 wave64, up to four requests per CU
constexpr int kRangePerCU = 4;      // range-query workgroups resident per CU (LDS and registers)
constexpr int kRangeLaunchPerCU = 2;  // FCFS requests per CU in a range-query planner launch
constexpr int kRangeThreadsSolo = 512;  // range-query planner alone on a CU: 8 wave64, one action per thread
constexpr int kRangeMaxHeads = 64;  // headings the range-query planner takes (its LDS budget)
constexpr int kMaxActions = 512;
constexpr int kMaxPoints = 4 * 4096;  // trajectory points per request (max_steps + 1)
constexpr int kMaxHeads = 128;
constexpr int kMaxLookahead = 16;   // longest scoring window W (steps)
constexpr int kRunning = -1;        // slot status while a request is being planned
constexpr int kAlive = 0x7fffffff;  // table entry death epoch of a live entry
constexpr double kBand = 1e-3;      // metres: FP32 nearest distances this close to the well
                                    // radius are recomputed exactly in FP64

// Problem constants as the kernels use them (passed by value).
struct DevCfg {
    double box_lo[3], box_hi[3];
    double dt, ell;
    double gamma, r_goal, r_intr, R_intr, gamma_intr, R_sep, r_terr, R_terr, gamma_terr;
    double log_gamma, log_gamma_intr, log_gamma_terr;   // discounts as exp(log_gamma * distance/ell)
    double abs_r_goal, abs_r_intr, abs_r_terr;
    float log2_gamma_f, inv_ell_f, abs_r_goal_f;        // FP32 goal-term bound of the proposal
    double climb[FASTMDP_MAX_ACT_DIM], speed[FASTMDP_MAX_ACT_DIM];
    float kv[FASTMDP_MAX_ACT_DIM];       // -2 * speed * dt
    float climb_f[FASTMDP_MAX_ACT_DIM];  // climb rates
    float zeta_scale;                    // -2 * dt
    double tie_rel;
    double reach;                        // max(R_intr, R_sep) + 1 m: a plan farther than this from
                                         // a successor cannot change its value
    double band_lo2, band_hi2;           // (R_intr -+ kBand)^2: squared distances recomputed exactly
    double reach_state;                  // reach + longest action step: a plan farther than this
                                         // from a state cannot change any of its successors' values
    int n_head, n_climb, n_speed, n_actions;
    int zero_climb;                      // index of the zero climb rate in the middle, else -1
    int max_steps;
    int lookahead;                       // scoring window W >= 1 (Alg. 1 forward projections)
    int range_query;                     // 1: stage only the row entries within cull_r2 of the state
    float cull_r2;                       // squared staging radius of the range query (FP32, 1 m margin)
    double max_step;                     // longest action step [m]: window point w lies within
                                         // w * max_step of the state
    double peak_growth;                  // co-simulated batch: peak radius R_intr + peak_growth * tau
    float cull_box;                      // half-width of the range-query box test on x and y: the
                                         // staging radius plus a margin for every rounding of the
                                         // exact test (FP32 offsets of coordinates up to max_abs)
    int planner_threads;                 // full-sweep path: 0 (automatic), kRangeThreads, kRangeThreadsSolo,
                                         // kPlanThreads
    int n_cu;                            // compute units of the device
};

// Time-major structure-of-arrays known-plan table.  Entry j of row t is at
// [t * cap + j] in X, Y, Z, vis, own, dead; rowN[t] entries are in use, in
// append order.  own is the sequence number of the request that owns the
// entry (-1 for loaded plans); dead is the epoch at which a tentative entry
// was withdrawn (kAlive while it stands); vis is own while the entry stands
// and kAlive once withdrawn, so that a request with sequence number q sees
// exactly the entries with vis < q (the planner reads X, Y, Z, vis only).
struct DevTable {
    float *X, *Y, *Z;
    int *vis, *own, *dead;
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
    long long entries;  // table row entries read (16 bytes each), accumulated
    int steps;        // steps taken, accumulated
    int resume_at;    // FCFS check: first affected point, -1 if none
    int seq;          // sequence number: sees live table entries with own < seq
    int valid;        // OK trajectory passed the commit validation against the entries it saw
    int killed;       // FCFS: withdrew tentative entries in the current pass
    int err;          // FCFS: table or log capacity exceeded
    int cert_hit;     // proposal steps certified, accumulated
    int cert_miss;    // proposal steps that fell back to the full sweep, accumulated
    int first;        // FCFS check: first affected point found so far (INT_MAX if none)
    int resumes;      // FCFS: times the request went back to planning, accumulated
    int clean_ep;     // FCFS: the pass whose check found the whole trajectory consistent (-1: none since
                      // it last finished planning)
};

// Per-slot trajectory buffers, `stride` points per slot.  seen[k] is the
// number of entries of the row scored to produce point k (for k = 0: the
// departure row of the origin check) and ep[k] the withdrawal epoch up to
// which that scoring is known to be consistent.  top[k] is the action with
// the largest value at that step when the chosen action (the lowest index
// inside the tie band) is not itself the largest, else -1.  col[k] is the
// column of point k's tentative table entry, -1 if none.  nd[k] is the
// nearest-plan squared distance of point k as the step scored it.
struct Traj {
    double *xyz;
    int *act;
    double *val;
    int *seen;
    int *ep;
    int *top;
    int *col;
    double *nd;      // squared distance from point k to the nearest plan of its row, as scored
                     // (infinity for the origin, which the origin check validated exactly)
    int *seenw;      // window W > 1: seenw[k * W + w - 1] is the number of entries of row
                     // t0 + k - 1 + w scored for window point w of the step to point k
    int stride;
};

// Log of withdrawn table entries (row, column, epoch), in epoch order.
struct DeathLog {
    int *row, *col, *ep;
    int *len;          // device counter
    int cap;
    const int *start;  // start[e]: log length when epoch e's withdrawals began
    float *x, *y;      // the withdrawn entry's stored x, y
    int *own;          // and its owner (sequence number)
};

// Work buffers of the FCFS acceptance pass: the row counts before the
// pass's insertions, the slots whose trajectories entered entries in it, and
// per slot the bounding box (FP32 x min, x max, y min, y max) of its points
// in each block of kRowBlock rows, from the block of its first row on.
constexpr int kRowBlock = 64;
constexpr int kRowBlocks = kMaxPoints / kRowBlock + 1;   // row blocks a trajectory can touch
struct PassBufs {
    int *rowN_pre;     // [rows]
    int *ins_list;     // [max_slots]
    int *ins_n;        // [1]
    float4 *box;       // [max_slots * kRowBlocks]
};

// Outputs of a single evaluated step (all device pointers, any may be null).
// feat, logit, topk, cert and pbest are written only with a proposal.
struct EvalOut {
    double *V, *G, *I, *T;
    int *best;
    float *feat, *logit;
    int *topk, *cert, *pbest;
};

// Proposal network weights as the planner reads them: BF16 [out][in]
// (W3 zero-padded to a multiple of 32 rows), FP32 biases.
struct PropNet {
    const uint16_t *W1, *W2, *W3;
    const float *b1, *b2, *b3;
    int n_in, n_hid, n_out;
};

// Proposal selection of a planner launch (mode FASTMDP_PROPOSE_*): the top
// k of the ranking, re-ranked every `refresh` steps and after a fallback.
struct PropArgs {
    int mode, k, refresh;
    PropNet net;
};

// Entry j of a row (absolute index idx) is visible to the request with
// sequence number seq.
__device__ __forceinline__ bool entry_visible(const DevTable &tb, size_t idx, int seq) {
    return tb.vis[idx] < seq;
}

// Squared distance, in FP64, between an FP64 point and an FP32 table entry:
// the one separation arithmetic of the planner's exact checks and of commit.
__device__ __forceinline__ double entry_d2(double x, double y, double z, float px, float py, float pz) {
    const double dx = (double)px - x, dy = (double)py - y, dz = (double)pz - z;
    return dx * dx + dy * dy + dz * dz;
}

// Early end of a launch: every workgroup whose request finishes adds one to
// *ctr; once it reaches target the others stop at their next step (they stay
// resumable).  target 0: run the full budget.
struct LaunchStop {
    int *ctr;
    int target;
};

// Peaks of the other aircraft of a co-simulated batch (Sec. V; the peak
// table: five risk wells per aircraft along its extrapolated track): pk[4k ..
// 4k+3] = x, y, z, radius of peak k, owner[k] its aircraft's slot, *n the
// number of peaks (device memory, written between planner launches).
// n == nullptr: no batch.
constexpr int kMaxBatch = 32;       // aircraft of one co-simulated batch
constexpr int kMatePeaks = 5;       // peaks per aircraft
struct MatePeaks {
    const double *pk;
    const int *owner;
    const int *n;
};

// Device state of a co-simulated batch between planner launches.
struct BatchState {
    double *pk;
    int *owner, *n;
    int *active;     // aircraft flying in the step just planned
    int *prev_n;     // its point count before that step
    int *any;        // 1 while an aircraft is flying
};

// nt: workgroup size; kPlanThreads is the one built.  prop.mode selects the
// proposal path (FASTMDP_PROPOSE_NONE: full sweep only).
hipError_t launch_planner(int nblk, int nt, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                          const int *list, const Traj &tr, int budget, int validate, int epoch, const EvalOut &ev,
                          const PropArgs &prop, const LaunchStop &stop, const MatePeaks &mates = MatePeaks{});

// batch.hip: after each planner step of a co-simulated batch (slots 0..n-1):
// separation between the aircraft that moved, goal capture and step limit,
// then the peaks of the aircraft still flying for the next step.  first:
// the launch before it only checked the origins.
hipError_t launch_batch_step(const DevCfg &c, Slot *slots, int n, const Traj &tr, const BatchState &bs, int first,
                             hipStream_t st);
bool planner_shape_supported(int n_climb, int n_speed, int zero_climb);

// Supported (climbs, speeds, zero-climb index) shapes of the planner kernels.
#define FMDP_PLANNER_SHAPES(X) \
    X(1, 1, 0) X(1, 1, -1) X(1, 2, 0) X(1, 2, -1) X(1, 3, 0) X(1, 3, -1) \
    X(2, 1, -1) X(2, 2, -1) X(2, 3, -1) \
    X(3, 1, 1) X(3, 1, -1) X(3, 2, 1) X(3, 2, -1) X(3, 3, 1) X(3, 3, -1) \
    X(5, 1, 2) X(5, 3, 2) X(5, 3, -1)

// range.hip: the range-query planner, kRangeThreads per request and
// kRangePerCU requests per compute unit, or kRangeThreadsSolo per request
// alone on a compute unit (full sweep with the range query, window W = 1,
// at most kRangeMaxHeads headings, no proposal, no co-simulated batch, no
// single-step outputs).
hipError_t launch_range_planner(int nblk, hipStream_t st, const DevCfg &c, const DevTable &t, Slot *s,
                                const int *list, const Traj &tr, int budget, int validate, int epoch,
                                const LaunchStop &stop);
// The full-sweep launches of this configuration go to the range-query
// planner.
inline bool uses_range_planner(const DevCfg &c, int prop_mode) {
    return c.range_query && c.lookahead <= 1 && prop_mode == FASTMDP_PROPOSE_NONE && c.n_head <= kRangeMaxHeads &&
           c.planner_threads != kPlanThreads;
}
// Its workgroup size for a launch of nblk requests: as configured, else
// one request per CU on kRangeThreadsSolo threads when the launch holds no
// more requests than CUs, two to four per CU on kRangeThreads otherwise.
inline int range_planner_threads(const DevCfg &c, int nblk) {
    if (c.planner_threads == kRangeThreads || c.planner_threads == kRangeThreadsSolo) return c.planner_threads;
    return nblk <= c.n_cu ? kRangeThreadsSolo : kRangeThreads;
}

// features.hip: proposal features of n states (device arrays, see
// fastmdp_features).
hipError_t launch_features(const DevCfg &c, const DevTable &t, int n, const double *states, const double *goals,
                           const int *rows, const int *seqs, float *feat, hipStream_t st);

// mlp.hip: the planner's view of a network's weights.
int mlp_weights(const fastmdp_mlp *m, PropNet *w);

// table.hip
hipError_t launch_fill_int(int *p, int value, int n, hipStream_t st);
hipError_t launch_scatter_points(const DevTable &t, const float *pts, const int *rows, const int *cols, int n,
                                 int own, hipStream_t st);
// Append n plans (t0[j], len[j], points plan-major in xyz; all device
// pointers) in order, each row's entries in plan order; the caller has
// checked rows and capacity.
hipError_t launch_append_plans(const DevTable &t, const int *t0, const int *len, int n, const float *xyz,
                               hipStream_t st);
hipError_t launch_commit_check(const DevCfg &c, const DevTable &t, const double *pts, int t0, int n, int seq,
                               int *flag, hipStream_t st);
hipError_t launch_commit_append(const DevTable &t, const double *pts, int t0, int n, int own, const int *flag,
                                hipStream_t st);
// Pack listed slots' trajectories (points from off[i]) into dst: total*3
// doubles xyz, total doubles value, total ints action.
hipError_t launch_gather_traj(const Slot *slots, const int *list, int n_list, const long long *off, long long total,
                              const Traj &tr, void *dst, hipStream_t st);
// FCFS pass over the finished, not yet accepted slots in `list`:
// tentative insert, interaction check, withdrawal (see table.hip).
hipError_t launch_fcfs_pass(const DevCfg &c, const DevTable &t, Slot *slots, const int *list, int n_list,
                            const Traj &tr, const DeathLog &dl, const PassBufs &pb, int epoch, int dl_len,
                            hipStream_t st);
// Withdraw every table entry of the listed slots owned by sequence numbers
// from min_own on (an interrupted FCFS call).
hipError_t launch_fcfs_abort(const DevTable &t, Slot *slots, const int *list, int n_list, const Traj &tr, int min_own,
                             int epoch, hipStream_t st);

}  // namespace fmdp
