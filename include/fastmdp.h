/*
 * fastmdp.h -- C ABI of the MI355X (gfx950) FastMDP first-come-first-served
 * pre-departure planner.
 *
 * Method: Bertram, Zambreno & Wei, "Scalable FastMDP for Pre-departure
 * Airspace Reservation and Strategic De-conflict".  A request (aircraft id,
 * source, destination; Sec. I) is flown in simulation one time step at a
 * time.  At each step every action's successor state is scored by the
 * closed-form FastMDP value -- the goal's positive peak discounted by the
 * time-to-go minus the largest risk-well penalty from the known plans'
 * positions at that time and from terrain (Sec. III, Alg. 1; Sec. IV
 * kernels "Process positive / negative intruder / negative terrain rewards"
 * and "Compute value") -- and the best action is taken ("Select best
 * action", "Determine terminal state").  A collision-free trajectory is
 * stored as an accepted plan and every later request must avoid it
 * (Sec. V, Experimental Setup).
 *
 * Conventions shared by every entry point
 *   - Return value: 0 on success, a negative FASTMDP_E_* code on error.
 *     Nothing throws across this boundary.  fastmdp_strerror() names codes.
 *   - All pointers in signatures are HOST pointers.  The caller owns every
 *     input and output buffer and keeps them alive for the duration of the
 *     call; the context owns all device memory (known-plan table, terrain,
 *     per-request trajectories, scratch).  Every call is synchronous with
 *     respect to its outputs.
 *   - Calls on one context are serialised by the context; the order of
 *     fastmdp_commit_plan calls is the first-come-first-served order.
 *   - Units: metres, seconds, radians.  Positions are in the airspace box
 *     frame.  Time is an integer row index: row t is time t*dt.
 *   - Actions: a = (h * n_climb + c) * n_speed + v, with heading offset
 *     2*pi*h/n_head from the bearing to the goal, climb rate climb[c] and
 *     horizontal speed speed[v], held for one step dt.
 */
#ifndef FASTMDP_H
#define FASTMDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FASTMDP_MAX_ACT_DIM 8

/* error codes (return values) */
#define FASTMDP_E_INVAL     (-1)   /* bad argument or unsupported configuration      */
#define FASTMDP_E_CAPACITY  (-2)   /* table rows / per-row capacity / buffers too small */
#define FASTMDP_E_DEVICE    (-3)   /* a HIP runtime call failed                      */
#define FASTMDP_E_CONFLICT  (-4)   /* commit refused: separation or terrain conflict  */
#define FASTMDP_E_NOMEM     (-5)   /* host or device allocation failed               */
#define FASTMDP_E_IO        (-6)   /* file could not be read or written              */

/* plan outcomes (fastmdp_plan.status) */
#define FASTMDP_OK                 0  /* goal reached within one step of travel      */
#define FASTMDP_REJECT_SEPARATION  1  /* chosen successor inside an intruder well    */
#define FASTMDP_REJECT_TERRAIN     2  /* chosen successor below the terrain surface  */
#define FASTMDP_REJECT_ORIGIN      3  /* origin outside the box, too close to a plan, or below terrain */
#define FASTMDP_TIMEOUT            4  /* max_steps taken without reaching the goal   */
#define FASTMDP_NO_VALID_ACTION    5  /* every successor leaves the airspace box      */

typedef struct fastmdp_ctx fastmdp_ctx;

typedef struct { double x, y, z; } fastmdp_vec3;

/* Problem constants; every size is fixed at fastmdp_create.
 * Peaks follow the tuple {r, gamma, position, R} of Sec. III: the goal is a
 * positive peak (r_goal, gamma, infinite radius); each known plan contributes
 * one risk well (r_intr, gamma_intr, its position at the successor's time,
 * R_intr); terrain contributes a clearance well (r_terr, gamma_terr, R_terr).
 * The discount exponent is the distance in steps of ell = max(speed)*dt. */
typedef struct {
    double box_min[3], box_max[3];   /* airspace box; successors outside it score -inf */
    double dt;                       /* step length [s]                           */
    double gamma, r_goal;            /* goal peak                                 */
    double r_intr, R_intr, gamma_intr;
    double R_sep;                    /* separation radius checked by commit [m]   */
    double r_terr, R_terr, gamma_terr;
    int32_t n_head, n_climb, n_speed;
    double climb[FASTMDP_MAX_ACT_DIM];   /* [m/s], n_climb used                   */
    double speed[FASTMDP_MAX_ACT_DIM];   /* [m/s], n_speed used, all > 0          */
    int32_t max_steps;               /* steps per request (<= max_steps+1 points) */
    int32_t plan_capacity;           /* known-plan entries per time row           */
    int32_t max_rows;                /* time rows in the table                    */
    int32_t max_slots;               /* requests planned concurrently (>= 1)      */
    int32_t steps_per_launch;        /* FCFS engine: steps per slot between
                                        acceptance passes (0: 256)                */
    int32_t planner_threads;         /* planning workgroup size: 0 or 1024 (one
                                        request per compute unit)                 */
    double tie_rel;                  /* argmax: values within tie_rel*|max| of the
                                        maximum tie; the lowest index wins        */
} fastmdp_config;

/* A plan request: aircraft identifier, source and destination (Sec. I),
 * departure row t0. */
typedef struct {
    uint64_t id;
    fastmdp_vec3 origin, goal;
    int32_t t0;
} fastmdp_request;

/* A planned trajectory.  The caller allocates xyz (3*capacity doubles,
 * point-major), action and value (capacity each).  Point 0 is the origin at
 * row t0 (action -1, value 0); point k is the state at row t0+k, reached by
 * action[k] whose value was value[k].  The outcome is in status. */
typedef struct {
    int32_t status;
    int32_t t0;
    int32_t n_points;
    int32_t capacity;
    double *xyz;
    int32_t *action;
    double *value;
} fastmdp_plan;

/* The state scored by fastmdp_eval_step: position at row t, and the goal. */
typedef struct {
    fastmdp_vec3 pos, goal;
    int32_t t;
} fastmdp_state;

/* Create a context on the current HIP device: allocates the time-major
 * structure-of-arrays plan table (max_rows x plan_capacity FP32 x, y, z) and
 * per-slot trajectory buffers.  Errors: E_INVAL (unsupported action-set
 * shape or bad constant), E_NOMEM, E_DEVICE.  *out is set only on success. */
int fastmdp_create(const fastmdp_config *cfg, fastmdp_ctx **out);

/* Release every device buffer and the context.  NULL is a no-op. */
void fastmdp_destroy(fastmdp_ctx *ctx);

/* Run the context's work on the given hipStream_t (NULL restores the
 * context's own stream).  The stream must outlive its use. */
int fastmdp_set_stream(fastmdp_ctx *ctx, void *hip_stream);

/* Load known plans (the accepted-plan database of Sec. V) without
 * validation, appended in the given order.  Plan j has len[j] points
 * starting at row t0[j]; xyz holds all points plan-major, 3 FP32 each.
 * Errors: E_INVAL, E_CAPACITY (a row would exceed plan_capacity or a plan
 * run past max_rows; the table is then unchanged), E_DEVICE. */
int fastmdp_load_plans(fastmdp_ctx *ctx, int32_t n, const int32_t *t0, const int32_t *len,
                       const float *xyz);

/* Terrain heightmap (the static terrain peaks of Sec. IV, "Build peaks"):
 * h[j*nx + i] is the height at (x0 + i*cell, y0 + j*cell); heights between
 * vertices are bilinear, positions outside the grid are clamped to its edge.
 * Replaces any previous terrain.  Errors: E_INVAL, E_NOMEM, E_DEVICE. */
int fastmdp_set_terrain(fastmdp_ctx *ctx, int32_t nx, int32_t ny, const float *h,
                        double x0, double y0, double cell);

/* One step of the method from state->pos at row state->t against the plans
 * active at row t+1 (Alg. 1 body; kernels "Forward project" through "Select
 * best action").  Writes, per action (n_head*n_climb*n_speed entries each,
 * any of the four arrays may be NULL): values (-inf outside the box),
 * goal_term r_goal*gamma^(d/ell), intr_term the largest intruder well,
 * terr_term the terrain well.  *best is the chosen action, -1 if all values
 * are -inf.  Errors: E_INVAL, E_DEVICE. */
int fastmdp_eval_step(fastmdp_ctx *ctx, const fastmdp_state *state, double *values,
                      double *goal_term, double *intr_term, double *terr_term, int32_t *best);

/* Plan one request against the current table (Fig. "myflowchart" loop until
 * the goal, a collision or max_steps; Sec. V).  Does NOT commit.  out->xyz,
 * out->action, out->value must hold out->capacity >= max_steps+1 points.
 * Errors: E_INVAL, E_CAPACITY, E_DEVICE. */
int fastmdp_plan_request(fastmdp_ctx *ctx, const fastmdp_request *req, fastmdp_plan *out);

/* Accept a plan into the table (Sec. V: the accepted-plan database grows by
 * one trajectory).  The points are rounded to FP32 and re-validated against
 * every plan in the table (3-D distance >= R_sep at every shared row) and
 * the terrain (clearance >= 0).  Returns 0 and appends, or E_CONFLICT with
 * the table unchanged; E_CAPACITY if a row is full or the plan runs past
 * max_rows; E_INVAL if plan->status is not FASTMDP_OK. */
int fastmdp_commit_plan(fastmdp_ctx *ctx, const fastmdp_plan *plan);

/* Number of plans in the table (loaded plus committed). */
int fastmdp_num_plans(const fastmdp_ctx *ctx);

/* First-come-first-served planning of a request stream (Sec. V; the
 * paper's "independent parallel instances" generalised to overlapping
 * requests).  Requests are admitted in order into up to max_slots slots --
 * request i not before arrival_s[i] seconds after the call starts (NULL: all
 * at once) -- and planned concurrently against the table as it stands.  Then,
 * strictly in request order, each finished trajectory is checked against
 * the plans committed after it scored their rows: if no committed point lies
 * within reach of a scored successor, the trajectory is the one a
 * sequential plan-then-commit would produce and it is accepted (appended
 * when its status is OK, after the commit validation); otherwise planning
 * resumes from the first affected step.  plans[i] receives request i's
 * trajectory (caller buffers as for fastmdp_plan_request); committed[i] is 1
 * if it entered the table; done_s[i] (may be NULL) is the time, in seconds
 * since the call started, at which request i was accepted or rejected.
 * Errors: E_INVAL, E_CAPACITY, E_DEVICE. */
int fastmdp_plan_fcfs(fastmdp_ctx *ctx, int32_t n, const fastmdp_request *reqs, const double *arrival_s,
                      fastmdp_plan *plans, int32_t *committed, double *done_s);

/* Remember the table's current extent / drop every plan appended since the
 * last snapshot (row counts return to the snapshot; nothing is copied).
 * Rewinding without a snapshot empties the table.  For re-running a batch
 * against the same accepted plans, or discarding tentative commits. */
int fastmdp_table_snapshot(fastmdp_ctx *ctx);
int fastmdp_table_rewind(fastmdp_ctx *ctx);

/* Counters of the last fastmdp_plan_request / fastmdp_plan_fcfs /
 * fastmdp_eval_step call: pair evaluations (action x active plan per step),
 * steps taken, resumes, planner launches, and summed planner-kernel time
 * in milliseconds measured with HIP events on the context's stream.  Any
 * pointer may be NULL. */
int fastmdp_last_stats(const fastmdp_ctx *ctx, int64_t *pairs, int64_t *steps, int64_t *resumes,
                       int64_t *launches, double *kernel_ms);

/* Checkpoint (the accepted-plan file of Sec. V): write / read the whole
 * table (row counts and FP32 points) to / from a binary file.  Loading
 * replaces the table; the configuration's sizes must match.
 * Errors: E_IO, E_CAPACITY, E_DEVICE. */
int fastmdp_save_table(fastmdp_ctx *ctx, const char *path);
int fastmdp_load_table(fastmdp_ctx *ctx, const char *path);

/* Static description of an error code or plan status (never NULL). */
const char *fastmdp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* FASTMDP_H */
