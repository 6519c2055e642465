// api.hip -- host side of libfastmdp: the C ABI declared in include/fastmdp.h.
//
// The context owns the device state: the time-major SoA known-plan table,
// the terrain heightmap, per-slot trajectory buffers and small scratch.  A
// host mirror of the per-row entry counts is kept for capacity checks and
// for loading plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fastmdp.h"
#include "planner.h"

using fmdp::DeathLog;
using fmdp::DevCfg;
using fmdp::DevTable;
using fmdp::EvalOut;
using fmdp::Slot;
using fmdp::Traj;

// Staging of fastmdp_load_plans_noalloc: a fixed device array, one copy on
// every GPU the library runs on, held until the process ends.  Plan starts
// and lengths take the first kNoallocPlanBytes, the FP32 points the rest.
// Host code never passes `scratch` itself (its name is a host-side stand-in,
// not a device address): it uses the address hipGetSymbolAddress returns on
// each device (noalloc_scratch).
constexpr int kNoallocMaxPlans = 65536;
constexpr int kNoallocMaxPoints = 655360;
constexpr size_t kNoallocPlanBytes = (size_t)2 * kNoallocMaxPlans * sizeof(int);
constexpr size_t kNoallocBytes = kNoallocPlanBytes + (size_t)3 * kNoallocMaxPoints * sizeof(float);   // 8 MiB
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), looked up once per
// device.  nullptr if the lookup fails.
void *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            std::fprintf(stderr, "libfastmdp: hipGetSymbolAddress(scratch) failed on device %d\n", dev);
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}
}  // namespace

struct fastmdp_ctx {
    fastmdp_config cfg{};
    DevCfg dc{};
    DevTable tb{};
    int A = 0;
    hipStream_t own = nullptr, stream = nullptr;
    std::vector<int> hRowN;
    int n_plans = 0;
    int seq = 0;                          // next request sequence number (table entry owners are below it)
    std::vector<int> snapRowN;            // table snapshot (row counts)
    int snap_plans = 0;
    float *dTerr = nullptr;
    int max_slots = 1, stride = 0;
    int n_cu = 256;                       // compute units of the device
    int dev = 0;                          // HIP device of the context
    void *dScratch = nullptr;             // this device's `scratch` (allocation-free plan loading)
    std::vector<int> hRowTmp;             // row counts being checked by fastmdp_load_plans_noalloc
    Slot *dSlots = nullptr;
    int *dList = nullptr, *dOrder = nullptr, *dNdone = nullptr;
    Traj tr{};
    double *dEv = nullptr;        // 4*A eval outputs
    int *dBest = nullptr;
    double *dPts = nullptr;       // stride*3 commit staging (FP64 trajectory)
    int *dFlag = nullptr;
    // FCFS withdrawal log
    int *dDlRow = nullptr, *dDlCol = nullptr, *dDlEp = nullptr, *dDlLen = nullptr, *dDlStart = nullptr;
    int *dDlOwn = nullptr;
    float *dDlX = nullptr, *dDlY = nullptr;
    // acceptance-pass work buffers (fmdp::PassBufs)
    int *dRowNPre = nullptr, *dInsList = nullptr, *dInsN = nullptr;
    float4 *dBox = nullptr;
    int dl_cap = 0, dl_start_cap = 0;
    // pinned host mirrors and the trajectory gather buffers of the FCFS engine
    Slot *hSlots = nullptr;
    int *dList2 = nullptr;
    long long *dOff = nullptr;
    void *dGather = nullptr, *hGather = nullptr;
    size_t gather_cap = 0;                // bytes
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t eGather = nullptr;         // after the last trajectory gather's copy to the host
    hipStream_t gstream = nullptr;        // the gathers' stream: their copies leave the planning stream free
    // pinned staging of the engine's small per-round transfers (the copies
    // read or write it when the stream reaches them, so each region is
    // rewritten only after the round's synchronisation): gather offsets, the
    // launch list, the pass list, the gather list, and the withdrawal log's
    // epoch start and length
    void *hRound = nullptr;
    long long *hOff = nullptr;
    int *hList = nullptr, *hPass = nullptr, *hList2 = nullptr, *hDl = nullptr;
    // learned action proposal
    fmdp::PropArgs prop{};
    float *dEvF = nullptr;        // proposal eval outputs: features, logits
    int *dEvI = nullptr;          // top-k, certified, proposal's action
    int *dStop = nullptr;         // finished-workgroup counter of a planner launch
    int *dPass = nullptr;         // slots of an acceptance pass
    fmdp::BatchState bs{};        // co-simulated batch: peaks and step bookkeeping
    std::mutex mu;
    // counters of the last call
    long long st_pairs = 0, st_steps = 0, st_resumes = 0, st_launches = 0, st_entries = 0;
    long long st_hit = 0, st_miss = 0;
    double st_ms = 0.0;
};

namespace {

#define HIP_TRY(x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) {                                                                     \
            std::fprintf(stderr, "libfastmdp: %s failed: %s\n", #x, hipGetErrorString(e_));         \
            return FASTMDP_E_DEVICE;                                                                \
        }                                                                                           \
    } while (0)

template <class T>
int dev_alloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) return 0;
    if (hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return FASTMDP_E_NOMEM;
    }
    return 0;
}

void free_all(fastmdp_ctx *c) {
    hipFree(c->tb.X); hipFree(c->tb.Y); hipFree(c->tb.Z); hipFree(c->tb.rowN);
    hipFree(c->tb.vis); hipFree(c->tb.own); hipFree(c->tb.dead);
    hipFree(c->dDlRow); hipFree(c->dDlCol); hipFree(c->dDlEp); hipFree(c->dDlLen); hipFree(c->dDlStart);
    hipFree(c->dDlOwn); hipFree(c->dDlX); hipFree(c->dDlY);
    hipFree(c->dRowNPre); hipFree(c->dInsList); hipFree(c->dInsN); hipFree(c->dBox);
    hipFree(c->dTerr);
    hipFree(c->dSlots); hipFree(c->dList); hipFree(c->dOrder); hipFree(c->dNdone);
    hipFree(c->tr.xyz); hipFree(c->tr.act); hipFree(c->tr.val); hipFree(c->tr.seen); hipFree(c->tr.top);
    hipFree(c->tr.ep); hipFree(c->tr.col); hipFree(c->tr.nd); hipFree(c->tr.seenw);
    hipFree(c->dEv); hipFree(c->dBest); hipFree(c->dPts); hipFree(c->dFlag);
    if (c->hSlots) hipHostFree(c->hSlots);
    if (c->hGather) hipHostFree(c->hGather);
    hipFree(c->dGather); hipFree(c->dList2); hipFree(c->dOff);
    hipFree(c->dEvF); hipFree(c->dEvI); hipFree(c->dStop); hipFree(c->dPass);
    hipFree(c->bs.pk); hipFree(c->bs.owner); hipFree(c->bs.n); hipFree(c->bs.active); hipFree(c->bs.prev_n);
    hipFree(c->bs.any);
    if (c->e0) hipEventDestroy(c->e0);
    if (c->e1) hipEventDestroy(c->e1);
    if (c->eGather) hipEventDestroy(c->eGather);
    if (c->hRound) hipHostFree(c->hRound);
    if (c->own) hipStreamDestroy(c->own);
    if (c->gstream) hipStreamDestroy(c->gstream);
}

int check_cfg(const fastmdp_config *c) {
    if (!c) return FASTMDP_E_INVAL;
    if (c->n_head < 1 || c->n_head > fmdp::kMaxHeads) return FASTMDP_E_INVAL;
    if (c->n_climb < 1 || c->n_climb > FASTMDP_MAX_ACT_DIM) return FASTMDP_E_INVAL;
    if (c->n_speed < 1 || c->n_speed > FASTMDP_MAX_ACT_DIM) return FASTMDP_E_INVAL;
    if ((long)c->n_head * c->n_climb * c->n_speed > fmdp::kMaxActions) return FASTMDP_E_INVAL;
    if (!(c->dt > 0.0) || !(c->gamma > 0.0 && c->gamma < 1.0)) return FASTMDP_E_INVAL;
    if (!(c->gamma_intr > 0.0 && c->gamma_intr < 1.0) || !(c->gamma_terr > 0.0 && c->gamma_terr < 1.0))
        return FASTMDP_E_INVAL;
    for (int v = 0; v < c->n_speed; ++v)
        if (!(c->speed[v] > 0.0)) return FASTMDP_E_INVAL;
    if (c->max_steps < 1 || c->max_steps + 1 > fmdp::kMaxPoints || c->max_rows < 2) return FASTMDP_E_INVAL;
    // rows are read four entries (16 bytes) per lane
    if (c->plan_capacity < 4 || c->plan_capacity % 4 != 0)
        return FASTMDP_E_INVAL;
    if (!(c->tie_rel >= 0.0)) return FASTMDP_E_INVAL;
    if (c->lookahead < 0 || c->lookahead > fmdp::kMaxLookahead) return FASTMDP_E_INVAL;
    if (c->range_query != 0 && c->range_query != 1) return FASTMDP_E_INVAL;
    if (c->planner_threads != 0 && c->planner_threads != fmdp::kPlanThreads &&
        !((c->planner_threads == fmdp::kRangeThreads || c->planner_threads == fmdp::kRangeThreadsSolo) &&
          c->range_query == 1 && c->lookahead <= 1 && c->n_head <= fmdp::kRangeMaxHeads))
        return FASTMDP_E_INVAL;
    if (!(c->peak_growth >= 0.0)) return FASTMDP_E_INVAL;
    return 0;
}

void make_devcfg(const fastmdp_config &c, DevCfg &d) {
    std::memset(&d, 0, sizeof(d));
    for (int k = 0; k < 3; ++k) { d.box_lo[k] = c.box_min[k]; d.box_hi[k] = c.box_max[k]; }
    double vmax = 0.0;
    for (int v = 0; v < c.n_speed; ++v) vmax = std::max(vmax, c.speed[v]);
    d.dt = c.dt;
    d.ell = vmax * c.dt;
    d.gamma = c.gamma; d.r_goal = c.r_goal;
    d.r_intr = c.r_intr; d.R_intr = c.R_intr; d.gamma_intr = c.gamma_intr;
    d.R_sep = c.R_sep;
    d.r_terr = c.r_terr; d.R_terr = c.R_terr; d.gamma_terr = c.gamma_terr;
    d.log_gamma = std::log(c.gamma);
    d.log_gamma_intr = std::log(c.gamma_intr);
    d.log_gamma_terr = std::log(c.gamma_terr);
    d.abs_r_goal = std::fabs(c.r_goal);
    d.abs_r_intr = std::fabs(c.r_intr);
    d.abs_r_terr = std::fabs(c.r_terr);
    d.log2_gamma_f = (float)std::log2(c.gamma);
    d.inv_ell_f = (float)(1.0 / d.ell);
    d.abs_r_goal_f = (float)d.abs_r_goal;
    for (int k = 0; k < FASTMDP_MAX_ACT_DIM; ++k) {
        d.climb[k] = c.climb[k];
        d.speed[k] = c.speed[k];
        d.climb_f[k] = (float)c.climb[k];
        d.kv[k] = (float)(-2.0 * c.speed[k] * c.dt);
    }
    d.zeta_scale = (float)(-2.0 * c.dt);
    d.tie_rel = c.tie_rel;
    d.reach = std::max(c.R_intr, c.R_sep) + 1.0;
    d.band_lo2 = std::max(c.R_intr - fmdp::kBand, 0.0) * std::max(c.R_intr - fmdp::kBand, 0.0);
    d.band_hi2 = (c.R_intr + fmdp::kBand) * (c.R_intr + fmdp::kBand);
    double cmax = 0.0;
    for (int k = 0; k < c.n_climb; ++k) cmax = std::max(cmax, std::fabs(c.climb[k]));
    d.reach_state = d.reach + std::sqrt(vmax * vmax + cmax * cmax) * c.dt;
    d.n_head = c.n_head; d.n_climb = c.n_climb; d.n_speed = c.n_speed;
    d.n_actions = c.n_head * c.n_climb * c.n_speed;
    const int mid = c.n_climb / 2;
    d.zero_climb = (c.climb[mid] == 0.0) ? mid : -1;
    d.max_steps = c.max_steps;
    d.lookahead = c.lookahead > 1 ? c.lookahead : 1;
    d.max_step = std::sqrt(vmax * vmax + cmax * cmax) * c.dt;
    d.range_query = c.range_query ? 1 : 0;
    d.peak_growth = c.peak_growth;
    // every point scored in a step lies within lookahead * max_step of the
    // state; a plan farther than reach from all of them changes nothing
    const double rc = d.reach + d.lookahead * d.max_step + 1.0;
    d.cull_r2 = (float)(rc * rc);
    // Box test of the range-query planner: an entry the exact test keeps has
    // |q_x|, |q_y| < sqrt(cull_r2) (1 + 2^-23), and the FP32 offset of the
    // box test differs from q_x by under |state| 2^-24 plus 2 |q_x| 2^-24.
    double max_abs = 0.0;
    for (int k = 0; k < 3; ++k) max_abs = std::max({max_abs, std::fabs(c.box_min[k]), std::fabs(c.box_max[k])});
    d.cull_box = (float)(std::sqrt((double)d.cull_r2) * 1.001 + 1.0 + max_abs * 1e-6);
    d.planner_threads = c.planner_threads;
    d.n_cu = 256;                          // the device's count is set once the context knows it
}

// Adds the last planner launch's duration (its events have completed).
int planner_time(fastmdp_ctx *c) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, c->e0, c->e1));
    c->st_ms += ms;
    c->st_launches += 1;
    return 0;
}

int timed_planner(fastmdp_ctx *c, int nblk, const int *list, int budget, int validate, int epoch,
                  const EvalOut &ev, int stop_target = 0, bool sync = true,
                  const fmdp::MatePeaks &mates = fmdp::MatePeaks{}) {
    const int nt = fmdp::kPlanThreads;
    HIP_TRY(hipEventRecord(c->e0, c->stream));
    const fmdp::LaunchStop stop{c->dStop, stop_target};
    if (stop_target > 0) HIP_TRY(fmdp::launch_fill_int(c->dStop, 0, 1, c->stream));
    hipError_t e = fmdp::launch_planner(nblk, nt, c->stream, c->dc, c->tb, c->dSlots, list, c->tr, budget, validate,
                                        epoch, ev, c->prop, stop, mates);
    if (e != hipSuccess) {
        std::fprintf(stderr, "libfastmdp: planner launch failed: %s\n", hipGetErrorString(e));
        return FASTMDP_E_DEVICE;
    }
    HIP_TRY(hipEventRecord(c->e1, c->stream));
    if (!sync) return 0;                     // the caller synchronises, then calls planner_time
    HIP_TRY(hipEventSynchronize(c->e1));
    return planner_time(c);
}

void reset_stats(fastmdp_ctx *c) {
    c->st_pairs = c->st_steps = c->st_resumes = c->st_launches = c->st_entries = 0;
    c->st_hit = c->st_miss = 0;
    c->st_ms = 0.0;
}

Slot fresh_slot(const fastmdp_request &r, int req_index, int seq) {
    Slot s;
    std::memset(&s, 0, sizeof(s));
    s.seq = seq;
    s.origin[0] = r.origin.x; s.origin[1] = r.origin.y; s.origin[2] = r.origin.z;
    s.goal[0] = r.goal.x; s.goal[1] = r.goal.y; s.goal[2] = r.goal.z;
    s.t0 = r.t0;
    s.n_points = 0;
    s.status = fmdp::kRunning;
    s.req = req_index;
    s.resume_at = -1;
    s.clean_ep = -1;
    return s;
}

int copy_plan_out(fastmdp_ctx *c, int slot, const Slot &s, fastmdp_plan *out) {
    const int n = s.n_points;
    if (out->capacity < n || !out->xyz || !out->action || !out->value) return FASTMDP_E_CAPACITY;
    const size_t base = (size_t)slot * c->stride;
    HIP_TRY(hipMemcpyAsync(out->xyz, c->tr.xyz + base * 3, (size_t)n * 3 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(out->action, c->tr.act + base, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(out->value, c->tr.val + base, (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    out->status = s.status;
    out->t0 = s.t0;
    out->n_points = n;
    return 0;
}

// Copy the trajectories of accepted slots to the callers' plans: one gather
// kernel into a device staging buffer, one copy into pinned host memory.
// Accepted trajectories on their way to the caller's plans: the device
// packs them into one buffer and copies it to pinned host memory; the host
// unpacks after a later synchronisation.
struct PendingPlans {
    std::vector<int> slots, reqs, n, status, t0;
    std::vector<long long> off;
    long long total = 0;
    bool empty() const { return reqs.empty(); }
};

int gather_enqueue(fastmdp_ctx *c, const std::vector<int> &slots, const std::vector<int> &reqs, const Slot *hs,
                   const fastmdp_plan *plans, PendingPlans &pp) {
    const int m = (int)slots.size();
    pp = PendingPlans();
    pp.slots = slots;
    pp.reqs = reqs;
    pp.off.resize(m);
    for (int i = 0; i < m; ++i) {
        const Slot &s = hs[slots[i]];
        if (plans[reqs[i]].capacity < s.n_points) return FASTMDP_E_CAPACITY;
        pp.off[i] = pp.total;
        pp.total += s.n_points;
        pp.n.push_back(s.n_points);
        pp.status.push_back(s.status);
        pp.t0.push_back(s.t0);
    }
    const size_t bytes = (size_t)pp.total * (3 * sizeof(double) + sizeof(double) + sizeof(int));
    if (bytes > c->gather_cap) {            // no copy is in flight here: the last one was unpacked
        const size_t cap = std::max(bytes, 2 * c->gather_cap);
        hipFree(c->dGather);
        if (c->hGather) hipHostFree(c->hGather);
        c->dGather = c->hGather = nullptr;
        c->gather_cap = 0;
        if (hipMalloc(&c->dGather, cap) != hipSuccess || hipHostMalloc(&c->hGather, cap) != hipSuccess)
            return FASTMDP_E_NOMEM;
        c->gather_cap = cap;
    }
    if (m > c->max_slots) return FASTMDP_E_CAPACITY;
    std::memcpy(c->hList2, pp.slots.data(), m * sizeof(int));
    std::memcpy(c->hOff, pp.off.data(), m * sizeof(long long));
    // on the gathers' own stream, so that the planning stream's next launch
    // does not wait for the copy; the caller has synchronised the planning
    // stream, and nothing it runs before these slots are reused writes them
    HIP_TRY(hipMemcpyAsync(c->dList2, c->hList2, m * sizeof(int), hipMemcpyHostToDevice, c->gstream));
    HIP_TRY(hipMemcpyAsync(c->dOff, c->hOff, m * sizeof(long long), hipMemcpyHostToDevice, c->gstream));
    HIP_TRY(fmdp::launch_gather_traj(c->dSlots, c->dList2, m, c->dOff, pp.total, c->tr, c->dGather, c->gstream));
    HIP_TRY(hipMemcpyAsync(c->hGather, c->dGather, bytes, hipMemcpyDeviceToHost, c->gstream));
    HIP_TRY(hipEventRecord(c->eGather, c->gstream));
    return 0;
}

// After a synchronisation that follows gather_enqueue.
void gather_unpack(fastmdp_ctx *c, PendingPlans &pp, fastmdp_plan *plans) {
    const double *xyz = static_cast<const double *>(c->hGather);
    const double *val = xyz + 3 * pp.total;
    const int *act = reinterpret_cast<const int *>(val + pp.total);
    for (size_t i = 0; i < pp.reqs.size(); ++i) {
        fastmdp_plan &p = plans[pp.reqs[i]];
        const int n = pp.n[i];
        std::memcpy(p.xyz, xyz + 3 * pp.off[i], (size_t)n * 3 * sizeof(double));
        std::memcpy(p.action, act + pp.off[i], (size_t)n * sizeof(int));
        std::memcpy(p.value, val + pp.off[i], (size_t)n * sizeof(double));
        p.status = pp.status[i];
        p.t0 = pp.t0[i];
        p.n_points = n;
    }
    pp = PendingPlans();
}

}  // namespace

extern "C" {

int fastmdp_create(const fastmdp_config *cfg, fastmdp_ctx **out) {
    if (!out) return FASTMDP_E_INVAL;
    int rc = check_cfg(cfg);
    if (rc) return rc;
    fastmdp_ctx *c = new (std::nothrow) fastmdp_ctx();
    if (!c) return FASTMDP_E_NOMEM;
    c->cfg = *cfg;
    make_devcfg(*cfg, c->dc);
    if (!fmdp::planner_shape_supported(cfg->n_climb, cfg->n_speed, c->dc.zero_climb)) {
        delete c;
        return FASTMDP_E_INVAL;
    }
    c->A = c->dc.n_actions;
    c->max_slots = std::max(1, cfg->max_slots);
    c->stride = cfg->max_steps + 1;
    c->tb.cap = cfg->plan_capacity;
    c->tb.rows = cfg->max_rows;
    const size_t tsz = (size_t)cfg->max_rows * cfg->plan_capacity;
    const size_t ssz = (size_t)c->max_slots * c->stride;
    rc = 0;
    rc = rc ? rc : dev_alloc(&c->tb.X, tsz);
    rc = rc ? rc : dev_alloc(&c->tb.Y, tsz);
    rc = rc ? rc : dev_alloc(&c->tb.Z, tsz);
    rc = rc ? rc : dev_alloc(&c->tb.vis, tsz);
    rc = rc ? rc : dev_alloc(&c->tb.own, tsz);
    rc = rc ? rc : dev_alloc(&c->tb.dead, tsz);
    rc = rc ? rc : dev_alloc(&c->tb.rowN, (size_t)cfg->max_rows);
    rc = rc ? rc : dev_alloc(&c->dSlots, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->dList, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->dOrder, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->dNdone, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->tr.xyz, ssz * 3);
    rc = rc ? rc : dev_alloc(&c->tr.act, ssz);
    rc = rc ? rc : dev_alloc(&c->tr.val, ssz);
    rc = rc ? rc : dev_alloc(&c->tr.seen, ssz);
    rc = rc ? rc : dev_alloc(&c->tr.top, ssz);
    rc = rc ? rc : dev_alloc(&c->tr.ep, ssz);
    rc = rc ? rc : dev_alloc(&c->tr.col, ssz);
    rc = rc ? rc : dev_alloc(&c->tr.nd, ssz);
    if (c->dc.lookahead > 1) rc = rc ? rc : dev_alloc(&c->tr.seenw, ssz * c->dc.lookahead);
    c->dl_cap = 1 << 22;
    c->dl_start_cap = 1 << 20;             // one epoch per acceptance round
    rc = rc ? rc : dev_alloc(&c->dDlRow, (size_t)c->dl_cap);
    rc = rc ? rc : dev_alloc(&c->dDlCol, (size_t)c->dl_cap);
    rc = rc ? rc : dev_alloc(&c->dDlEp, (size_t)c->dl_cap);
    rc = rc ? rc : dev_alloc(&c->dDlOwn, (size_t)c->dl_cap);
    rc = rc ? rc : dev_alloc(&c->dDlX, (size_t)c->dl_cap);
    rc = rc ? rc : dev_alloc(&c->dDlY, (size_t)c->dl_cap);
    rc = rc ? rc : dev_alloc(&c->dRowNPre, (size_t)cfg->max_rows);
    rc = rc ? rc : dev_alloc(&c->dInsList, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->dInsN, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->dBox, (size_t)c->max_slots * fmdp::kRowBlocks);
    rc = rc ? rc : dev_alloc(&c->dDlLen, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->dDlStart, (size_t)c->dl_start_cap);
    rc = rc ? rc : dev_alloc(&c->dEv, (size_t)4 * c->A);
    rc = rc ? rc : dev_alloc(&c->dBest, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->dPts, (size_t)c->stride * 3);
    rc = rc ? rc : dev_alloc(&c->dFlag, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->dList2, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->dOff, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->dEvF, (size_t)FASTMDP_N_FEAT + fmdp::kMaxActions);
    rc = rc ? rc : dev_alloc(&c->dEvI, (size_t)FASTMDP_MAX_TOPK + 2);
    rc = rc ? rc : dev_alloc(&c->dStop, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->dPass, (size_t)c->max_slots);
    rc = rc ? rc : dev_alloc(&c->bs.pk, (size_t)fmdp::kMaxBatch * fmdp::kMatePeaks * 4);
    rc = rc ? rc : dev_alloc(&c->bs.owner, (size_t)fmdp::kMaxBatch * fmdp::kMatePeaks);
    rc = rc ? rc : dev_alloc(&c->bs.n, (size_t)1);
    rc = rc ? rc : dev_alloc(&c->bs.active, (size_t)fmdp::kMaxBatch);
    rc = rc ? rc : dev_alloc(&c->bs.prev_n, (size_t)fmdp::kMaxBatch);
    rc = rc ? rc : dev_alloc(&c->bs.any, (size_t)1);
    if (!rc && hipHostMalloc(reinterpret_cast<void **>(&c->hSlots), (size_t)c->max_slots * sizeof(Slot)) != hipSuccess)
        rc = FASTMDP_E_NOMEM;
    if (!rc && hipStreamCreate(&c->own) != hipSuccess) rc = FASTMDP_E_DEVICE;
    if (!rc && hipStreamCreate(&c->gstream) != hipSuccess) rc = FASTMDP_E_DEVICE;
    if (!rc && hipEventCreate(&c->e0) != hipSuccess) rc = FASTMDP_E_DEVICE;
    if (!rc && hipEventCreate(&c->e1) != hipSuccess) rc = FASTMDP_E_DEVICE;
    if (!rc && hipEventCreateWithFlags(&c->eGather, hipEventDisableTiming) != hipSuccess) rc = FASTMDP_E_DEVICE;
    if (!rc) {
        const size_t ms = (size_t)c->max_slots;
        if (hipHostMalloc(&c->hRound, ms * sizeof(long long) + (4 * ms + 2) * sizeof(int)) != hipSuccess) {
            rc = FASTMDP_E_NOMEM;
        } else {
            c->hOff = static_cast<long long *>(c->hRound);
            c->hList = reinterpret_cast<int *>(c->hOff + ms);
            c->hPass = c->hList + ms;
            c->hList2 = c->hPass + ms;
            c->hDl = c->hList2 + ms;
        }
    }
    if (rc) {
        free_all(c);
        delete c;
        return rc;
    }
    c->stream = c->own;
    c->tr.stride = c->stride;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            c->dev = dev;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
                c->n_cu = cus;
        }
    }
    c->dc.n_cu = c->n_cu;
    c->dScratch = noalloc_scratch(c->dev);
    if (!c->dScratch) {
        free_all(c);
        delete c;
        return FASTMDP_E_DEVICE;
    }
    c->hRowN.assign(cfg->max_rows, 0);
    c->hRowTmp.assign(cfg->max_rows, 0);
    if (fmdp::launch_fill_int(c->tb.rowN, 0, cfg->max_rows, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        free_all(c);
        delete c;
        return FASTMDP_E_DEVICE;
    }
    *out = c;
    return 0;
}

void fastmdp_destroy(fastmdp_ctx *ctx) {
    if (!ctx) return;
    hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
}

int fastmdp_set_stream(fastmdp_ctx *ctx, void *hip_stream) {
    if (!ctx) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->own;
    return 0;
}

int fastmdp_load_plans(fastmdp_ctx *ctx, int32_t n, const int32_t *t0, const int32_t *len, const float *xyz) {
    if (!ctx || n < 0 || (n > 0 && (!t0 || !len || !xyz))) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    size_t total = 0;
    for (int j = 0; j < n; ++j) {
        if (t0[j] < 0 || len[j] < 1) return FASTMDP_E_INVAL;
        if ((long)t0[j] + len[j] > ctx->tb.rows) return FASTMDP_E_CAPACITY;
        total += (size_t)len[j];
    }
    std::vector<int> rowN = ctx->hRowN;
    std::vector<int> rows(total), cols(total);
    size_t p = 0;
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < len[j]; ++k, ++p) {
            const int r = t0[j] + k;
            if (rowN[r] >= ctx->tb.cap) return FASTMDP_E_CAPACITY;
            rows[p] = r;
            cols[p] = rowN[r]++;
        }
    if (total) {
        float *dP = nullptr;
        int *dR = nullptr, *dC = nullptr;
        int rc = dev_alloc(&dP, total * 3);
        rc = rc ? rc : dev_alloc(&dR, total);
        rc = rc ? rc : dev_alloc(&dC, total);
        if (rc) { hipFree(dP); hipFree(dR); hipFree(dC); return rc; }
        hipError_t e = hipMemcpyAsync(dP, xyz, total * 3 * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dR, rows.data(), total * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dC, cols.data(), total * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = fmdp::launch_scatter_points(ctx->tb, dP, dR, dC, (int)total, -1, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->tb.rowN, rowN.data(), rowN.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        hipFree(dP); hipFree(dR); hipFree(dC);
        if (e != hipSuccess) {
            std::fprintf(stderr, "libfastmdp: load_plans: %s\n", hipGetErrorString(e));
            return FASTMDP_E_DEVICE;
        }
    }
    ctx->hRowN.swap(rowN);
    ctx->n_plans += n;
    return 0;
}

int fastmdp_load_plans_noalloc(fastmdp_ctx *ctx, int32_t n, const int32_t *t0, const int32_t *len,
                               const float *xyz) {
    if (!ctx || n < 0 || (n > 0 && (!t0 || !len || !xyz))) return FASTMDP_E_INVAL;
    if (n > kNoallocMaxPlans) return FASTMDP_E_CAPACITY;
    std::lock_guard<std::mutex> lk(ctx->mu);
    long long total = 0;
    for (int j = 0; j < n; ++j) {
        if (t0[j] < 0 || len[j] < 1) return FASTMDP_E_INVAL;
        if ((long)t0[j] + len[j] > ctx->tb.rows) return FASTMDP_E_CAPACITY;
        total += len[j];
    }
    if (total > kNoallocMaxPoints) return FASTMDP_E_CAPACITY;
    if (n == 0) return 0;
    // row counts after the load, in the context's own host buffer
    std::vector<int> &rowN = ctx->hRowTmp;
    std::copy(ctx->hRowN.begin(), ctx->hRowN.end(), rowN.begin());
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < len[j]; ++k)
            if (++rowN[t0[j] + k] > ctx->tb.cap) return FASTMDP_E_CAPACITY;
    unsigned char *base = static_cast<unsigned char *>(ctx->dScratch);
    int *dT0 = reinterpret_cast<int *>(base);
    int *dLen = dT0 + kNoallocMaxPlans;
    float *dXyz = reinterpret_cast<float *>(base + kNoallocPlanBytes);
    hipError_t e = hipMemcpyAsync(dT0, t0, (size_t)n * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dLen, len, (size_t)n * sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dXyz, xyz, (size_t)total * 3 * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = fmdp::launch_append_plans(ctx->tb, dT0, dLen, n, dXyz, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        std::fprintf(stderr, "libfastmdp: load_plans_noalloc: %s\n", hipGetErrorString(e));
        return FASTMDP_E_DEVICE;
    }
    ctx->hRowN.swap(rowN);
    ctx->n_plans += n;
    return 0;
}

int fastmdp_set_terrain(fastmdp_ctx *ctx, int32_t nx, int32_t ny, const float *h, double x0, double y0, double cell) {
    if (!ctx || nx < 2 || ny < 2 || !h || !(cell > 0.0)) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    float *d = nullptr;
    int rc = dev_alloc(&d, (size_t)nx * ny);
    if (rc) return rc;
    if (hipMemcpy(d, h, (size_t)nx * ny * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(d);
        return FASTMDP_E_DEVICE;
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    hipFree(ctx->dTerr);
    ctx->dTerr = d;
    ctx->tb.terr = d;
    ctx->tb.tnx = nx; ctx->tb.tny = ny;
    ctx->tb.tx0 = x0; ctx->tb.ty0 = y0; ctx->tb.tcell = cell;
    return 0;
}

int fastmdp_eval_step(fastmdp_ctx *ctx, const fastmdp_state *state, double *values, double *goal_term,
                      double *intr_term, double *terr_term, int32_t *best) {
    if (!ctx || !state || state->t < 0) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    reset_stats(ctx);
    fastmdp_request r{};
    r.origin = state->pos;
    r.goal = state->goal;
    r.t0 = state->t;
    Slot s = fresh_slot(r, 0, ctx->seq);
    HIP_TRY(hipMemcpyAsync(ctx->dSlots, &s, sizeof(Slot), hipMemcpyHostToDevice, ctx->stream));
    const int A = ctx->A;
    EvalOut ev{ctx->dEv, ctx->dEv + A, ctx->dEv + 2 * A, ctx->dEv + 3 * A, ctx->dBest};
    int rc = timed_planner(ctx, 1, nullptr, 1, 0, 0, ev);
    if (rc) return rc;
    std::vector<double> h(4 * (size_t)A);
    int b = -1;
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->dEv, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(&b, ctx->dBest, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(&s, ctx->dSlots, sizeof(Slot), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (values) std::memcpy(values, h.data(), A * sizeof(double));
    if (goal_term) std::memcpy(goal_term, h.data() + A, A * sizeof(double));
    if (intr_term) std::memcpy(intr_term, h.data() + 2 * A, A * sizeof(double));
    if (terr_term) std::memcpy(terr_term, h.data() + 3 * A, A * sizeof(double));
    if (best) *best = b;
    ctx->st_pairs = s.pairs;
    ctx->st_entries = s.entries;
    ctx->st_steps = s.steps;
    return 0;
}

int fastmdp_plan_request(fastmdp_ctx *ctx, const fastmdp_request *req, fastmdp_plan *out) {
    if (!ctx || !req || !out || req->t0 < 0) return FASTMDP_E_INVAL;
    if (out->capacity < ctx->stride || !out->xyz || !out->action || !out->value) return FASTMDP_E_CAPACITY;
    std::lock_guard<std::mutex> lk(ctx->mu);
    reset_stats(ctx);
    Slot s = fresh_slot(*req, 0, ctx->seq);
    HIP_TRY(hipMemcpyAsync(ctx->dSlots, &s, sizeof(Slot), hipMemcpyHostToDevice, ctx->stream));
    EvalOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = timed_planner(ctx, 1, nullptr, ctx->cfg.max_steps + 1, 0, 0, none);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(&s, ctx->dSlots, sizeof(Slot), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    rc = copy_plan_out(ctx, 0, s, out);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->st_pairs = s.pairs;
    ctx->st_entries = s.entries;
    ctx->st_steps = s.steps;
    ctx->st_hit = s.cert_hit;
    ctx->st_miss = s.cert_miss;
    return 0;
}

int fastmdp_plan_departures(fastmdp_ctx *ctx, const fastmdp_request *req, int32_t n, const int32_t *t0,
                            fastmdp_plan *plans, int32_t *chosen) {
    if (!ctx || !req || n < 1 || !t0 || !plans || !chosen) return FASTMDP_E_INVAL;
    if (n > ctx->max_slots) return FASTMDP_E_CAPACITY;
    for (int i = 0; i < n; ++i) {
        if (t0[i] < 0) return FASTMDP_E_INVAL;
        if (plans[i].capacity < ctx->stride || !plans[i].xyz || !plans[i].action || !plans[i].value)
            return FASTMDP_E_CAPACITY;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    reset_stats(ctx);
    Slot *hs = ctx->hSlots;
    for (int i = 0; i < n; ++i) {
        fastmdp_request r = *req;
        r.t0 = t0[i];
        hs[i] = fresh_slot(r, i, ctx->seq);            // every candidate sees the same table
    }
    HIP_TRY(hipMemcpyAsync(ctx->dSlots, hs, n * sizeof(Slot), hipMemcpyHostToDevice, ctx->stream));
    EvalOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = timed_planner(ctx, n, nullptr, ctx->cfg.max_steps + 1, 1, 0, none);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(hs, ctx->dSlots, n * sizeof(Slot), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    int best = -1;
    for (int i = 0; i < n; ++i) {
        rc = copy_plan_out(ctx, i, hs[i], &plans[i]);
        if (rc) return rc;
        ctx->st_pairs += hs[i].pairs;
        ctx->st_entries += hs[i].entries;
        ctx->st_steps += hs[i].steps;
        // the earliest departure whose plan reached the goal and would be accepted
        if (hs[i].status == FASTMDP_OK && hs[i].valid && (best < 0 || t0[i] < t0[best])) best = i;
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *chosen = best;
    return 0;
}

int fastmdp_plan_batch(fastmdp_ctx *ctx, int32_t n, const fastmdp_request *reqs, fastmdp_plan *plans) {
    if (!ctx || n < 1 || !reqs || !plans) return FASTMDP_E_INVAL;
    if (n > fmdp::kMaxBatch || n > ctx->max_slots) return FASTMDP_E_CAPACITY;
    if (ctx->dc.lookahead > 1 || ctx->prop.mode != FASTMDP_PROPOSE_NONE) return FASTMDP_E_INVAL;
    for (int i = 0; i < n; ++i) {
        if (reqs[i].t0 < 0 || reqs[i].t0 != reqs[0].t0) return FASTMDP_E_INVAL;     // lockstep from one row
        if (plans[i].capacity < ctx->stride || !plans[i].xyz || !plans[i].action || !plans[i].value)
            return FASTMDP_E_CAPACITY;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    reset_stats(ctx);
    Slot *hs = ctx->hSlots;
    for (int i = 0; i < n; ++i) hs[i] = fresh_slot(reqs[i], i, ctx->seq);
    HIP_TRY(hipMemcpyAsync(ctx->dSlots, hs, n * sizeof(Slot), hipMemcpyHostToDevice, ctx->stream));
    const fmdp::MatePeaks mates{ctx->bs.pk, ctx->bs.owner, ctx->bs.n};
    EvalOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
    const fmdp::LaunchStop nostop{ctx->dStop, 0};
    HIP_TRY(hipEventRecord(ctx->e0, ctx->stream));
    // the origin checks (no step), then each step: one planner step of every
    // aircraft still flying, then the batch's own rules and the next peaks
    auto planner = [&](int budget) -> int {
        hipError_t e = fmdp::launch_planner(n, fmdp::kPlanThreads, ctx->stream, ctx->dc, ctx->tb, ctx->dSlots, nullptr,
                                            ctx->tr, budget, 0, 0, none, ctx->prop, nostop,
                                            budget > 0 ? mates : fmdp::MatePeaks{});
        if (e != hipSuccess) {
            std::fprintf(stderr, "libfastmdp: planner launch failed: %s\n", hipGetErrorString(e));
            return FASTMDP_E_DEVICE;
        }
        ctx->st_launches += 1;
        return 0;
    };
    int rc = planner(0);
    if (rc) return rc;
    HIP_TRY(fmdp::launch_batch_step(ctx->dc, ctx->dSlots, n, ctx->tr, ctx->bs, 1, ctx->stream));
    int any = 1;
    for (int k = 0; any; ++k) {
        rc = planner(1);
        if (rc) return rc;
        HIP_TRY(fmdp::launch_batch_step(ctx->dc, ctx->dSlots, n, ctx->tr, ctx->bs, 0, ctx->stream));
        if ((k & 15) == 15 || k >= ctx->cfg.max_steps) {
            HIP_TRY(hipMemcpyAsync(&any, ctx->bs.any, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            if (k > ctx->cfg.max_steps + 1) break;                 // every aircraft has hit the step limit
        }
    }
    HIP_TRY(hipEventRecord(ctx->e1, ctx->stream));
    HIP_TRY(hipMemcpyAsync(hs, ctx->dSlots, n * sizeof(Slot), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->e0, ctx->e1));
    ctx->st_ms = ms;
    for (int i = 0; i < n; ++i) {
        rc = copy_plan_out(ctx, i, hs[i], &plans[i]);
        if (rc) return rc;
        ctx->st_pairs += hs[i].pairs;
        ctx->st_entries += hs[i].entries;
        ctx->st_steps += hs[i].steps;
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return 0;
}

int fastmdp_commit_plan(fastmdp_ctx *ctx, const fastmdp_plan *plan) {
    if (!ctx || !plan || !plan->xyz || plan->n_points < 1 || plan->t0 < 0) return FASTMDP_E_INVAL;
    if (plan->status != FASTMDP_OK) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const int n = plan->n_points, t0 = plan->t0;
    if ((long)t0 + n > ctx->tb.rows || n > ctx->stride) return FASTMDP_E_CAPACITY;
    for (int k = 0; k < n; ++k)
        if (ctx->hRowN[t0 + k] >= ctx->tb.cap) return FASTMDP_E_CAPACITY;
    HIP_TRY(hipMemcpyAsync(ctx->dPts, plan->xyz, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(fmdp::launch_fill_int(ctx->dFlag, 0, 1, ctx->stream));
    HIP_TRY(fmdp::launch_commit_check(ctx->dc, ctx->tb, ctx->dPts, t0, n, ctx->seq, ctx->dFlag, ctx->stream));
    HIP_TRY(fmdp::launch_commit_append(ctx->tb, ctx->dPts, t0, n, ctx->seq, ctx->dFlag, ctx->stream));
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, ctx->dFlag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (flag & 2) return FASTMDP_E_CAPACITY;
    if (flag) return FASTMDP_E_CONFLICT;
    for (int k = 0; k < n; ++k) ctx->hRowN[t0 + k] += 1;
    ctx->n_plans += 1;
    ctx->seq += 1;
    return 0;
}

int fastmdp_num_plans(const fastmdp_ctx *ctx) { return ctx ? ctx->n_plans : FASTMDP_E_INVAL; }

int fastmdp_plan_fcfs(fastmdp_ctx *ctx, int32_t n, const fastmdp_request *reqs, const double *arrival_s,
                      fastmdp_plan *plans, int32_t *committed, double *done_s) {
    if (!ctx || n < 0 || (n > 0 && (!reqs || !plans || !committed))) return FASTMDP_E_INVAL;
    for (int i = 0; i < n; ++i) {
        if (reqs[i].t0 < 0) return FASTMDP_E_INVAL;
        if (arrival_s && (i > 0 && arrival_s[i] < arrival_s[i - 1])) return FASTMDP_E_INVAL;
        if (plans[i].capacity < ctx->stride || !plans[i].xyz || !plans[i].action || !plans[i].value)
            return FASTMDP_E_CAPACITY;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    reset_stats(ctx);
    using clk = std::chrono::steady_clock;
    const auto t_start = clk::now();
    auto now_s = [&]() { return std::chrono::duration<double>(clk::now() - t_start).count(); };
    const int S = std::min(ctx->max_slots, std::max(n, 1));
    const int budget = ctx->cfg.steps_per_launch > 0 ? ctx->cfg.steps_per_launch : 512;
    const int seq0 = ctx->seq;
    Slot *hs = ctx->hSlots;                  // pinned mirror of the slots
    std::vector<int> slot_req(S, -1);        // request held by each slot
    std::vector<int> req_slot(n, -1);
    int next_req = 0, next_commit = 0;
    std::vector<int> list, pass;
    PendingPlans pending;                    // accepted trajectories still being copied
    bool gathered = false;                   // a gather was enqueued in this call
    // withdrawal log of this call: epoch e's withdrawals start at dl_start[e]
    int epoch = 0, dl_len = 0;
    std::vector<int> dl_start(2, 0);
    HIP_TRY(fmdp::launch_fill_int(ctx->dDlLen, 0, 1, ctx->stream));
    HIP_TRY(fmdp::launch_fill_int(ctx->dDlStart, 0, 2, ctx->stream));
    DeathLog dl{ctx->dDlRow, ctx->dDlCol, ctx->dDlEp, ctx->dDlLen, ctx->dl_cap, ctx->dDlStart,
                ctx->dDlX, ctx->dDlY, ctx->dDlOwn};
    auto finish = [&](int rc) {
        // the device row counts include tentative and withdrawn entries
        if (hipMemcpyAsync(ctx->hRowN.data(), ctx->tb.rowN, ctx->hRowN.size() * sizeof(int), hipMemcpyDeviceToHost,
                           ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            return FASTMDP_E_DEVICE;
        return rc;
    };
    auto run = [&]() -> int {
        while (next_commit < n) {
            // admit arrived requests into free slots, in request order
            bool dirty = false;
            const double t_now = arrival_s ? now_s() : 0.0;
            for (int s = 0; s < S && next_req < n; ++s)
                if (slot_req[s] < 0) {
                    if (arrival_s && arrival_s[next_req] > t_now) break;
                    hs[s] = fresh_slot(reqs[next_req], next_req, seq0 + next_req);
                    slot_req[s] = next_req;
                    req_slot[next_req] = s;
                    ++next_req;
                    dirty = true;
                }
            if (dirty) {
                // a reused slot: its accepted trajectory's gather comes first
                if (gathered) HIP_TRY(hipStreamWaitEvent(ctx->stream, ctx->eGather, 0));
                HIP_TRY(hipMemcpyAsync(ctx->dSlots, hs, S * sizeof(Slot), hipMemcpyHostToDevice, ctx->stream));
            }
            // plan the oldest running requests, one per compute unit (the
            // planner's workgroups take a CU each; the range-query planner's
            // two: it could hold four, but the oldest requests, which the later
            // ones depend on, then step more slowly; measured: 3 % shorter
            // FCFS passes with two), for up to `budget` steps: a
            // request that waits for the next launch plans against the plans its
            // predecessors finish in this one instead of re-planning after them
            list.clear();
            for (int s = 0; s < S; ++s)
                if (slot_req[s] >= 0 && hs[s].status == fmdp::kRunning) list.push_back(s);
            const int per_launch =
                ctx->n_cu * (fmdp::uses_range_planner(ctx->dc, ctx->prop.mode) ? fmdp::kRangeLaunchPerCU : 1);
            if ((int)list.size() > per_launch) {
                std::nth_element(list.begin(), list.begin() + per_launch, list.end(),
                                 [&](int a, int b) { return hs[a].req < hs[b].req; });
                list.resize(per_launch);
            }
            if (list.empty() && next_commit == next_req) {
                // idle until the next arrival
                const double wait = arrival_s[next_req] - now_s();
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.001)));
                continue;
            }
            // One synchronisation per round: the planner launch, the acceptance
            // pass over every admitted, not yet accepted request (its kernels
            // skip the ones still planning), the copy of the slots back, and the
            // trajectories accepted in the previous round on their way to the
            // caller's plans, all in stream order.
            const bool planned = !list.empty();
            if (planned) {
                std::memcpy(ctx->hList, list.data(), list.size() * sizeof(int));
                HIP_TRY(hipMemcpyAsync(ctx->dList, ctx->hList, list.size() * sizeof(int), hipMemcpyHostToDevice,
                                       ctx->stream));
                EvalOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
                // the launch ends once a quarter of its requests have finished:
                // the others resume after the acceptance pass, with new requests
                // in the freed compute units.  The range-query planner's launches
                // hold two requests per CU, and few wait for one after the first
                // launches, so the launch runs until half have finished (fewer
                // acceptance passes; measured: about 10 % shorter FCFS passes
                // than with a quarter, while the one-per-CU planners lose with
                // half)
                const int stop_div = fmdp::uses_range_planner(ctx->dc, ctx->prop.mode) ? 2 : 4;
                const int stop_target = std::max(1, (int)list.size() / stop_div);
                int rc = timed_planner(ctx, (int)list.size(), ctx->dList, budget, 1, epoch, none, stop_target, false);
                if (rc) return finish(rc);
            }
            pass.clear();
            for (int r = next_commit; r < next_req; ++r) pass.push_back(req_slot[r]);
            epoch += 1;
            if (epoch + 1 >= ctx->dl_start_cap) return finish(FASTMDP_E_CAPACITY);
            dl_start.resize(epoch + 1);
            dl_start[epoch] = dl_len;
            ctx->hDl[0] = dl_len;
            std::memcpy(ctx->hPass, pass.data(), pass.size() * sizeof(int));
            HIP_TRY(hipMemcpyAsync(ctx->dDlStart + epoch, ctx->hDl, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(ctx->dPass, ctx->hPass, pass.size() * sizeof(int), hipMemcpyHostToDevice,
                                   ctx->stream));
            const fmdp::PassBufs pbufs{ctx->dRowNPre, ctx->dInsList, ctx->dInsN, ctx->dBox};
            HIP_TRY(fmdp::launch_fcfs_pass(ctx->dc, ctx->tb, ctx->dSlots, ctx->dPass, (int)pass.size(), ctx->tr, dl,
                                           pbufs, epoch, dl_len, ctx->stream));
            HIP_TRY(hipMemcpyAsync(hs, ctx->dSlots, S * sizeof(Slot), hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipMemcpyAsync(ctx->hDl + 1, ctx->dDlLen, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            // the trajectories accepted last round were gathered ahead of this
            // round's launch: hand them to the caller while the planner runs
            if (!pending.empty()) {
                HIP_TRY(hipEventSynchronize(ctx->eGather));
                gather_unpack(ctx, pending, plans);
            }
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            dl_len = ctx->hDl[1];
            if (planned) {
                int rc = planner_time(ctx);
                if (rc) return finish(rc);
            }
            if (dl_len > ctx->dl_cap) return finish(FASTMDP_E_CAPACITY);
            for (int s : pass) {
                if (hs[s].err) return finish(FASTMDP_E_CAPACITY);
            }
            // accept in request order: a finished request whose predecessors are
            // all accepted is final; one that withdrew entries in this pass ends
            // the walk (later requests are checked against it next pass)
            const double t_done = now_s();
            std::vector<int> acc_slots, acc_reqs;
            while (next_commit < next_req) {
                const int s = req_slot[next_commit];
                if (hs[s].status == fmdp::kRunning) break;
                const int r = next_commit;
                committed[r] = (hs[s].status == FASTMDP_OK && hs[s].valid) ? 1 : 0;
                if (done_s) done_s[r] = t_done;
                ctx->n_plans += committed[r];
                ctx->st_pairs += hs[s].pairs;
                ctx->st_entries += hs[s].entries;
                ctx->st_steps += hs[s].steps;
                ctx->st_hit += hs[s].cert_hit;
                ctx->st_miss += hs[s].cert_miss;
                ctx->st_resumes += hs[s].resumes;
                acc_slots.push_back(s);
                acc_reqs.push_back(r);
                ++next_commit;
                if (hs[s].killed) break;
            }
            if (!acc_slots.empty()) {
                int rc = gather_enqueue(ctx, acc_slots, acc_reqs, hs, plans, pending);
                if (rc) return finish(rc);
                gathered = true;
                for (int s : acc_slots) slot_req[s] = -1;   // reusable: the gather precedes any new planning
            }
        }
        if (!pending.empty()) {
            HIP_TRY(hipEventSynchronize(ctx->eGather));
            gather_unpack(ctx, pending, plans);
        }
        return 0;
    };
    const int rc = run();
    if (rc == 0) {
        ctx->seq = seq0 + n;
        return finish(0);
    }
    // An interrupted call keeps exactly the accepted requests: their plans
    // stay in the table and are visible to every later request (sequence
    // numbers below ctx->seq); the entries of every admitted request not yet
    // accepted are withdrawn.  Accepted trajectories still on their way to
    // the caller are delivered; committed[] is 0 from the first unaccepted
    // request on.
    hipStreamSynchronize(ctx->stream);
    if (!pending.empty() && hipEventSynchronize(ctx->eGather) == hipSuccess) gather_unpack(ctx, pending, plans);
    int m = 0;
    for (int s = 0; s < S; ++s)
        if (slot_req[s] >= 0) ctx->hPass[m++] = s;
    if (m > 0 && hipMemcpyAsync(ctx->dPass, ctx->hPass, m * sizeof(int), hipMemcpyHostToDevice, ctx->stream) == hipSuccess)
        fmdp::launch_fcfs_abort(ctx->tb, ctx->dSlots, ctx->dPass, m, ctx->tr, seq0 + next_commit, epoch + 1,
                                ctx->stream);
    for (int r = next_commit; r < n; ++r) committed[r] = 0;
    ctx->seq = seq0 + next_commit;
    return finish(rc);
}

int fastmdp_table_snapshot(fastmdp_ctx *ctx) {
    if (!ctx) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->snapRowN = ctx->hRowN;
    ctx->snap_plans = ctx->n_plans;
    return 0;
}

int fastmdp_table_rewind(fastmdp_ctx *ctx) {
    if (!ctx) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->snapRowN.empty()) {
        ctx->snapRowN.assign(ctx->tb.rows, 0);
        ctx->snap_plans = 0;
    }
    HIP_TRY(hipMemcpyAsync(ctx->tb.rowN, ctx->snapRowN.data(), ctx->snapRowN.size() * sizeof(int),
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->hRowN = ctx->snapRowN;
    ctx->n_plans = ctx->snap_plans;
    return 0;
}

int fastmdp_last_stats(const fastmdp_ctx *ctx, int64_t *pairs, int64_t *steps, int64_t *resumes, int64_t *launches,
                       double *kernel_ms, int64_t *row_entries) {
    if (!ctx) return FASTMDP_E_INVAL;
    if (pairs) *pairs = ctx->st_pairs;
    if (row_entries) *row_entries = ctx->st_entries;
    if (steps) *steps = ctx->st_steps;
    if (resumes) *resumes = ctx->st_resumes;
    if (launches) *launches = ctx->st_launches;
    if (kernel_ms) *kernel_ms = ctx->st_ms;
    return 0;
}

int fastmdp_features(fastmdp_ctx *ctx, int32_t n, const double *states, const double *goals, const int32_t *rows,
                     const int32_t *seqs, float *feat) {
    if (!ctx || n < 0 || (n > 0 && (!states || !goals || !rows || !seqs || !feat))) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_TRY(fmdp::launch_features(ctx->dc, ctx->tb, n, states, goals, rows, seqs, feat, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return 0;
}

int fastmdp_next_seq(const fastmdp_ctx *ctx) { return ctx ? ctx->seq : FASTMDP_E_INVAL; }

int fastmdp_set_proposal(fastmdp_ctx *ctx, int32_t mode, int32_t top_k, int32_t refresh, const fastmdp_mlp *net) {
    if (!ctx || refresh < 1) return FASTMDP_E_INVAL;
    fmdp::PropArgs p{};
    p.mode = mode;
    p.k = top_k;
    p.refresh = refresh;
    if (mode == FASTMDP_PROPOSE_NONE) {
        p.k = 0;
    } else if (mode == FASTMDP_PROPOSE_MLP || mode == FASTMDP_PROPOSE_GOAL) {
        if (ctx->dc.lookahead > 1) return FASTMDP_E_INVAL;      // the window runs the full sweep
        if (top_k < 1 || top_k > FASTMDP_MAX_TOPK || top_k > ctx->A) return FASTMDP_E_INVAL;
        if (mode == FASTMDP_PROPOSE_MLP) {
            if (fmdp::mlp_weights(net, &p.net)) return FASTMDP_E_INVAL;
            if (p.net.n_in != FASTMDP_N_FEAT || p.net.n_hid != FASTMDP_MLP_HIDDEN || p.net.n_out < ctx->A)
                return FASTMDP_E_INVAL;
        }
    } else {
        return FASTMDP_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->prop = p;
    return 0;
}

int fastmdp_eval_proposal(fastmdp_ctx *ctx, const fastmdp_state *state, float *features, float *logits,
                          int32_t *topk, int32_t *certified, int32_t *best) {
    if (!ctx || !state || state->t < 0) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->prop.mode == FASTMDP_PROPOSE_NONE) return FASTMDP_E_INVAL;
    reset_stats(ctx);
    fastmdp_request r{};
    r.origin = state->pos;
    r.goal = state->goal;
    r.t0 = state->t;
    Slot s = fresh_slot(r, 0, ctx->seq);
    HIP_TRY(hipMemcpyAsync(ctx->dSlots, &s, sizeof(Slot), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->dEvF, 0, (FASTMDP_N_FEAT + fmdp::kMaxActions) * sizeof(float), ctx->stream));
    const int A = ctx->A;
    EvalOut ev{nullptr, nullptr, nullptr, nullptr, ctx->dBest, ctx->dEvF, ctx->dEvF + FASTMDP_N_FEAT,
               ctx->dEvI, ctx->dEvI + FASTMDP_MAX_TOPK, ctx->dEvI + FASTMDP_MAX_TOPK + 1};
    int rc = timed_planner(ctx, 1, nullptr, 1, 0, 0, ev);
    if (rc) return rc;
    std::vector<float> hf(FASTMDP_N_FEAT + (size_t)A);
    int hi[FASTMDP_MAX_TOPK + 2];
    HIP_TRY(hipMemcpyAsync(hf.data(), ctx->dEvF, hf.size() * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(hi, ctx->dEvI, sizeof(hi), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (features) std::memcpy(features, hf.data(), FASTMDP_N_FEAT * sizeof(float));
    if (logits) std::memcpy(logits, hf.data() + FASTMDP_N_FEAT, A * sizeof(float));
    if (topk) std::memcpy(topk, hi, ctx->prop.k * sizeof(int));
    if (certified) *certified = hi[FASTMDP_MAX_TOPK];
    if (best) *best = hi[FASTMDP_MAX_TOPK + 1];
    return 0;
}

int fastmdp_proposal_stats(const fastmdp_ctx *ctx, int64_t *certified, int64_t *fallbacks) {
    if (!ctx) return FASTMDP_E_INVAL;
    if (certified) *certified = ctx->st_hit;
    if (fallbacks) *fallbacks = ctx->st_miss;
    return 0;
}

// Checkpoint file: "FMDPTAB2", rows, cap, n_plans, live entries per row
// [rows], then for each row its live entries' x, y and z (FP32).  Withdrawn
// entries are dropped; loaded entries are owned by no request.
int fastmdp_save_table(fastmdp_ctx *ctx, const char *path) {
    if (!ctx || !path) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const int rows = ctx->tb.rows, cap = ctx->tb.cap;
    std::vector<int> dead((size_t)cap), live(rows, 0);
    std::vector<float> buf[3];
    for (auto &b : buf) b.resize((size_t)cap);
    std::vector<std::vector<float>> keep(rows);
    for (int r = 0; r < rows; ++r) {
        const int m = std::min(ctx->hRowN[r], cap);
        if (!m) continue;
        const size_t off = (size_t)r * cap;
        float *src[3] = {ctx->tb.X, ctx->tb.Y, ctx->tb.Z};
        if (hipMemcpy(dead.data(), ctx->tb.dead + off, m * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            return FASTMDP_E_DEVICE;
        for (int a = 0; a < 3; ++a)
            if (hipMemcpy(buf[a].data(), src[a] + off, m * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
                return FASTMDP_E_DEVICE;
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < m; ++j)
                if (dead[j] == fmdp::kAlive) keep[r].push_back(buf[a][j]);
        live[r] = (int)keep[r].size() / 3;
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return FASTMDP_E_IO;
    int hdr[3] = {rows, cap, ctx->n_plans};
    bool ok = std::fwrite("FMDPTAB2", 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int), 3, f) == 3 &&
              std::fwrite(live.data(), sizeof(int), rows, f) == (size_t)rows;
    for (int r = 0; ok && r < rows; ++r)
        if (!keep[r].empty()) ok = std::fwrite(keep[r].data(), sizeof(float), keep[r].size(), f) == keep[r].size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? 0 : FASTMDP_E_IO;
}

int fastmdp_load_table(fastmdp_ctx *ctx, const char *path) {
    if (!ctx || !path) return FASTMDP_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    FILE *f = std::fopen(path, "rb");
    if (!f) return FASTMDP_E_IO;
    char magic[8];
    int hdr[3];
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "FMDPTAB2", 8) != 0 ||
        std::fread(hdr, sizeof(int), 3, f) != 3) {
        std::fclose(f);
        return FASTMDP_E_IO;
    }
    const int rows = hdr[0];
    if (rows != ctx->tb.rows || hdr[2] < 0) {
        std::fclose(f);
        return FASTMDP_E_CAPACITY;
    }
    std::vector<int> rowN(rows);
    if (std::fread(rowN.data(), sizeof(int), rows, f) != (size_t)rows) {
        std::fclose(f);
        return FASTMDP_E_IO;
    }
    for (int r = 0; r < rows; ++r)
        if (rowN[r] < 0 || rowN[r] > ctx->tb.cap) {
            std::fclose(f);
            return FASTMDP_E_CAPACITY;
        }
    const int cap = ctx->tb.cap;
    std::vector<float> buf((size_t)cap * 3);
    std::vector<int> own((size_t)cap, -1), alive((size_t)cap, fmdp::kAlive);
    for (int r = 0; r < rows; ++r) {
        const int m = rowN[r];
        if (!m) continue;
        if (std::fread(buf.data(), sizeof(float), (size_t)m * 3, f) != (size_t)m * 3) {
            std::fclose(f);
            return FASTMDP_E_IO;
        }
        const size_t off = (size_t)r * cap;
        float *dst[3] = {ctx->tb.X, ctx->tb.Y, ctx->tb.Z};
        bool ok = true;
        for (int a = 0; a < 3 && ok; ++a)
            ok = hipMemcpy(dst[a] + off, buf.data() + (size_t)a * m, m * sizeof(float), hipMemcpyHostToDevice) ==
                 hipSuccess;
        ok = ok && hipMemcpy(ctx->tb.vis + off, own.data(), m * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(ctx->tb.own + off, own.data(), m * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(ctx->tb.dead + off, alive.data(), m * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        if (!ok) {
            std::fclose(f);
            return FASTMDP_E_DEVICE;
        }
    }
    std::fclose(f);
    if (hipMemcpy(ctx->tb.rowN, rowN.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return FASTMDP_E_DEVICE;
    ctx->hRowN.swap(rowN);
    ctx->n_plans = hdr[2];
    return 0;
}

const char *fastmdp_strerror(int code) {
    switch (code) {
        case 0: return "ok";
        case FASTMDP_E_INVAL: return "invalid argument or unsupported configuration";
        case FASTMDP_E_CAPACITY: return "table or buffer capacity exceeded";
        case FASTMDP_E_DEVICE: return "HIP runtime error";
        case FASTMDP_E_CONFLICT: return "commit refused: separation or terrain conflict";
        case FASTMDP_E_NOMEM: return "out of memory";
        case FASTMDP_E_IO: return "file input/output error";
        default: return "unknown code";
    }
}

}  // extern "C"
