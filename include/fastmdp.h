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
 *   - Pointers in signatures are HOST pointers, except the training and
 *     feature arrays of the learned action proposal, whose comments say
 *     DEVICE (memory of the context's or the network's HIP device).  The
 *     caller owns every input and output buffer and keeps them alive for
 *     the duration of the call; the context owns all other device memory
 *     (known-plan table, terrain, per-request trajectories, scratch), the
 *     network its weights, optimiser state and activations.  Every call is
 *     synchronous with respect to its outputs.
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
    int32_t max_steps;               /* steps per request (<= max_steps+1 points),
                                        at most 16383                             */
    int32_t plan_capacity;           /* known-plan entries per time row, a
                                        multiple of 4                            */
    int32_t max_rows;                /* time rows in the table                    */
    int32_t max_slots;               /* requests planned concurrently (>= 1)      */
    int32_t steps_per_launch;        /* FCFS engine: most steps per slot between
                                        acceptance passes (0: 512); a launch also
                                        ends once a quarter of its requests have
                                        finished                                  */
    int32_t planner_threads;         /* full-sweep planning workgroup: 0 (auto),
                                        1024 (one request per compute unit) or,
                                        with range_query = 1, lookahead <= 1 and
                                        n_head <= 64, 256 (four requests per
                                        compute unit) or 512 (one request per
                                        compute unit).  0 takes, where allowed,
                                        512 for a launch of at most one request
                                        per compute unit and 256 for a larger
                                        one, else 1024; the proposal path keeps
                                        its own workgroup and single-step
                                        outputs and co-simulated batches the
                                        1024-thread one.  Every choice gives
                                        the same plans bit for bit               */
    double tie_rel;                  /* argmax: values within tie_rel*|max| of the
                                        maximum tie; the lowest index wins        */
    int32_t lookahead;               /* scoring window W, 1..16 (0 reads as 1):
                                        action a held for w = 1..W steps reaches
                                        s + w*Delta_a at row t+w, and its value is
                                        the largest value along the window (Alg. 1
                                        forward projections; "Forward project" and
                                        "Compute value" kernels); -inf if the
                                        successor (w = 1) leaves the box, window
                                        points outside the box are left out.  The
                                        state still advances one step, and a
                                        successor inside an intruder well still
                                        rejects.  W > 1 runs the full sweep at
                                        every step (no proposal). */
    int32_t range_query;             /* 1: without a proposal, each step sweeps
                                        only the plans within reach of the state
                                        (max(R_intr, R_sep) + 1 m + the longest
                                        action step; W > 1 adds (W-1) steps), a
                                        range query over the row (Sec. VII: range
                                        queries restrict the trajectories
                                        considered to the relevant volume).  A
                                        plan outside that ball cannot reach any
                                        scored point's well or the commit
                                        check's reach, so values and plans are
                                        those of the full sweep; pair counts
                                        then count the plans swept.  0: off. */
    double peak_growth;              /* co-simulated batches (fastmdp_plan_batch):
                                        the radius of the peak at time offset tau
                                        along another aircraft's track is R_intr +
                                        peak_growth * tau [m/s], >= 0 */
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

/* fastmdp_load_plans for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same arguments, result and table layout, but the plans travel through a
 * fixed 8 MiB device staging array that the library holds on each GPU until
 * the process ends, so the call makes no device or host allocation.  At most
 * 65536 plans and 655360 points per call; larger loads return E_CAPACITY
 * (split them over several calls).  Every context on one GPU shares that
 * GPU's staging array: calls that overlap in time on one GPU (from several
 * threads, on different contexts) race and must be serialised by the
 * caller.  Errors: E_INVAL, E_CAPACITY (also: a row would exceed
 * plan_capacity or a plan run past max_rows; the table is then unchanged),
 * E_DEVICE. */
int fastmdp_load_plans_noalloc(fastmdp_ctx *ctx, int32_t n, const int32_t *t0, const int32_t *len,
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

/* Candidate departure times of one request (ground delay): the paper plans
 * to generate candidate flight plans with different departure times and let
 * the operator choose among the viable ones (Sec. V, scheduling at different
 * departure times; "Expected Outcome").  The request is planned from each
 * departure row t0[i], i < n, against the current table, all candidates at
 * once (one workgroup each, all seeing the same table); nothing is
 * committed.  plans[i] receives candidate i (buffers as for
 * fastmdp_plan_request); *chosen is the index of the earliest departure whose
 * plan reached the goal and passes the commit validation (the lowest index
 * among equal rows), -1 if none.  1 <= n <= max_slots.
 * Errors: E_INVAL, E_CAPACITY, E_DEVICE. */
int fastmdp_plan_departures(fastmdp_ctx *ctx, const fastmdp_request *req, int32_t n, const int32_t *t0,
                            fastmdp_plan *plans, int32_t *chosen);

/* Co-simulated batch (Sec. V: several aircraft planned together, each aware
 * of the others and of every accepted plan).  The n requests (all with the
 * same departure row) fly in lockstep.  At each step every aircraft still
 * flying scores its actions against the known plans, the terrain and five
 * risk wells per other flying aircraft, placed along that aircraft's
 * extrapolated track at p + v*tau for tau in {-5, 0, 5, 10, 15} s with
 * radius R_intr + peak_growth*tau, magnitude r_intr and discount gamma_intr
 * (the peak table; "Build peaks"; "Process negative rewards"), p its
 * position and v its last step over dt (0 before its first step); the value
 * is the goal term less the largest of the intruder, batch and terrain
 * wells ("Compute value").  Then all apply their choices; an aircraft is
 * rejected (REJECT_SEPARATION) when a known plan's well contains its new
 * point or another aircraft that moved in the same step is closer than
 * R_sep, and an aircraft within one step of its goal or at max_steps is
 * done at the start of the next step.  One planner launch per step, one
 * workgroup per aircraft.  plans[i] receives aircraft i (buffers as for
 * fastmdp_plan_request); nothing is committed.  1 <= n <= 32 and n <=
 * max_slots; needs lookahead 1 and no proposal.
 * Errors: E_INVAL, E_CAPACITY, E_DEVICE. */
int fastmdp_plan_batch(fastmdp_ctx *ctx, int32_t n, const fastmdp_request *reqs, fastmdp_plan *plans);

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
 * at once) -- and planned concurrently against the table as it stands, each
 * planner launch taking the oldest unfinished requests, at most one per
 * compute unit, and the finished ones entering the table tentatively.  Then,
 * strictly in request order, each finished trajectory is checked against
 * the plans committed after it scored their rows: if no committed point lies
 * within reach of a scored successor, the trajectory is the one a
 * sequential plan-then-commit would produce and it is accepted (appended
 * when its status is OK, after the commit validation); otherwise planning
 * resumes from the first affected step.  plans[i] receives request i's
 * trajectory (caller buffers as for fastmdp_plan_request); committed[i] is 1
 * if it entered the table; done_s[i] (may be NULL) is the time, in seconds
 * since the call started, at which request i was accepted or rejected.
 * Errors: E_INVAL, E_CAPACITY (a row full, a trajectory past max_rows, the
 * withdrawal log full), E_DEVICE.  A call that fails after admitting
 * requests keeps the ones accepted so far: their plans stay in the table,
 * visible to every later call, with plans[i] and committed[i] filled in;
 * every entry of the other admitted requests is withdrawn and their
 * committed[i] is 0, and the next call's requests follow the last accepted
 * one in sequence. */
int fastmdp_plan_fcfs(fastmdp_ctx *ctx, int32_t n, const fastmdp_request *reqs, const double *arrival_s,
                      fastmdp_plan *plans, int32_t *committed, double *done_s);

/* Remember the table's current extent / drop every plan appended since the
 * last snapshot (row counts return to the snapshot; nothing is copied).
 * Rewinding without a snapshot empties the table.  For re-running a batch
 * against the same accepted plans, or discarding tentative commits. */
int fastmdp_table_snapshot(fastmdp_ctx *ctx);
int fastmdp_table_rewind(fastmdp_ctx *ctx);

/* Counters of the last planning call (fastmdp_plan_request, _plan_fcfs,
 * _plan_departures, _plan_batch, _eval_step): pair evaluations (action x
 * plan swept per step), steps taken, resumes, planner launches, summed
 * planner-kernel time in milliseconds measured with HIP events on the
 * context's stream, and table row entries read (each step reads the
 * successor's row, 16 bytes per entry: x, y, z, visibility; every window
 * row with a window).  Any pointer may be NULL. */
int fastmdp_last_stats(const fastmdp_ctx *ctx, int64_t *pairs, int64_t *steps, int64_t *resumes,
                       int64_t *launches, double *kernel_ms, int64_t *row_entries);

/* Checkpoint (the accepted-plan file of Sec. V): write / read the whole
 * table (row counts and FP32 points) to / from a binary file.  Loading
 * replaces the table; the configuration's sizes must match.
 * Errors: E_IO, E_CAPACITY, E_DEVICE. */
int fastmdp_save_table(fastmdp_ctx *ctx, const char *path);
int fastmdp_load_table(fastmdp_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------
 * Learned action proposal (an addition to the method, not in the paper).
 *
 * At each step a small network ranks the actions from features of the
 * state; only the top_k are scored exactly (the same closed-form value as
 * the full sweep), and the step is taken from them only when a certificate
 * proves that no other action can reach the chosen value: every other
 * action's value is at most its goal term (the penalties are
 * non-negative), so if the best exact value among the k, less the argmax
 * tie band, exceeds every other action's goal term, the full sweep would
 * choose the same action.  Otherwise the step runs the full sweep.  Plans
 * are therefore identical, bit for bit, to the plain method's.
 *
 * Features (FASTMDP_N_FEAT FP32 per state s at row t, goal g; plans are the
 * entries of row t+1 the request sees, q = p - s):
 *   [0,32)  per (sector k, half u): 1 - d/600 of the nearest plan with
 *           d = |q| < 600 m, in sector k = floor((phi+pi)*16/(2 pi)) of the
 *           bearing phi of q measured from the horizontal direction to the
 *           goal (positive to the left), u = 0 if q_z >= 0 else 1;
 *           index 2k+u; 0 if none;
 *   [32,64) the count of such plans, clipped to 4, divided by 4;
 *   64 horizontal distance to the goal / 10 km; 65 (g_z - s_z) / 500 m;
 *   66 |g - s| / ell / 1000; 67 log(1 + |g - s|/ell) / 8; 68 s_z / 1000 m;
 *   69-71 s_z, s_x, s_y scaled to [0,1] over the box; 72-73 the horizontal
 *   unit vector to the goal; 74 min(n/16, 1) with n the plans within 600 m;
 *   75 the nearest such distance / 600 (1 if none); 76-95 zero.
 * Network: FASTMDP_N_FEAT -> n_hidden -> n_hidden -> n_out, ReLU, logits;
 * BF16 weights and activations with FP32 accumulation; FP32 master weights
 * trained with softmax cross-entropy on the chosen action and Adam.
 * Parameters, packed FP32 in this order: W1 [n_hidden][n_in], b1 [n_hidden],
 * W2 [n_hidden][n_hidden], b2 [n_hidden], W3 [n_out][n_hidden], b3 [n_out]
 * (row-major, output index first). */
#define FASTMDP_N_FEAT        96
#define FASTMDP_MLP_HIDDEN   256   /* hidden width the planner's inference supports */
#define FASTMDP_MAX_TOPK      16

/* proposal modes (fastmdp_set_proposal) */
#define FASTMDP_PROPOSE_NONE  0    /* full sweep at every step                       */
#define FASTMDP_PROPOSE_MLP   1    /* the network's top_k logits                      */
#define FASTMDP_PROPOSE_GOAL  2    /* the top_k goal terms (no network)               */

typedef struct fastmdp_mlp fastmdp_mlp;

/* Create a network on the current HIP device with zero parameters, for
 * batches of up to max_batch rows.  n_in and n_hidden must be multiples of
 * 32 (n_in = FASTMDP_N_FEAT for use by a planner); n_out >= 1.
 * Errors: E_INVAL, E_NOMEM, E_DEVICE. */
int fastmdp_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, fastmdp_mlp **out);

/* Release the network.  NULL is a no-op.  A context using it for proposals
 * must have its proposal reset first. */
void fastmdp_mlp_destroy(fastmdp_mlp *net);

/* Number of packed FP32 parameters (layout above). */
int64_t fastmdp_mlp_num_params(const fastmdp_mlp *net);

/* Copy all parameters in (HOST, packed FP32; resets the Adam state) or
 * out.  Errors: E_INVAL, E_DEVICE. */
int fastmdp_mlp_set_params(fastmdp_mlp *net, const float *params);
int fastmdp_mlp_get_params(fastmdp_mlp *net, float *params);

/* Logits of a batch: x DEVICE [batch][n_in] FP32, logits DEVICE
 * [batch][n_out] FP32.  1 <= batch <= max_batch.  Errors: E_INVAL, E_DEVICE. */
int fastmdp_mlp_forward(fastmdp_mlp *net, int32_t batch, const float *x, float *logits);

/* Mean softmax cross-entropy of labels y (DEVICE [batch] int32 in
 * [0, n_out)) and its gradient with respect to every parameter, written to
 * grads (HOST, packed like the parameters); *loss (HOST) may be NULL.
 * batch must be a multiple of 32.  Errors: E_INVAL, E_DEVICE. */
int fastmdp_mlp_gradient(fastmdp_mlp *net, int32_t batch, const float *x, const int32_t *y, float *grads,
                         float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * size lr) on the gradient of the batch, as fastmdp_mlp_gradient defines
 * it.  *loss (HOST, may be NULL) receives the batch loss before the step.
 * batch must be a multiple of 32.  Errors: E_INVAL, E_DEVICE. */
int fastmdp_mlp_train_step(fastmdp_mlp *net, int32_t batch, const float *x, const int32_t *y, float lr,
                           float *loss);

/* Proposal features (definition above) of n states against the table as a
 * request with sequence number seqs[i] sees it: states and goals DEVICE
 * [n][3] FP64, rows and seqs DEVICE [n] int32 (the plans are those of row
 * rows[i] + 1), feat DEVICE [n][FASTMDP_N_FEAT] FP32.  Errors: E_INVAL,
 * E_DEVICE. */
int fastmdp_features(fastmdp_ctx *ctx, int32_t n, const double *states, const double *goals, const int32_t *rows,
                     const int32_t *seqs, float *feat);

/* Sequence number of the next request (the first of the next
 * fastmdp_plan_fcfs call; request i of that call has this plus i). */
int fastmdp_next_seq(const fastmdp_ctx *ctx);

/* Select the proposal for later planning calls: mode FASTMDP_PROPOSE_*,
 * 1 <= top_k <= FASTMDP_MAX_TOPK.  The ranking and its top_k are recomputed
 * every `refresh` steps (>= 1; 1 = every step) and after every step that
 * fell back to the full sweep; in between the same actions (relative to the
 * goal bearing) are scored exactly, and the certificate is decided at every
 * step, so plans do not depend on refresh.  FASTMDP_PROPOSE_MLP needs a
 * network with n_in = FASTMDP_N_FEAT, n_hidden = FASTMDP_MLP_HIDDEN and
 * n_out >= the number of actions, on the same device; the context reads its
 * current weights at every ranking, so it must stay alive while selected.
 * Errors: E_INVAL. */
int fastmdp_set_proposal(fastmdp_ctx *ctx, int32_t mode, int32_t top_k, int32_t refresh, const fastmdp_mlp *net);

/* The proposal at one state (as fastmdp_eval_step): features (HOST
 * FASTMDP_N_FEAT) and logits (HOST, one per action), both
 * FASTMDP_PROPOSE_MLP only (zero otherwise),
 * the top_k proposed actions (HOST top_k, best first), whether the
 * certificate held, and the action the proposal path takes (-1 when it
 * falls back).  Any pointer may be NULL.  Errors: E_INVAL (no proposal
 * selected), E_DEVICE. */
int fastmdp_eval_proposal(fastmdp_ctx *ctx, const fastmdp_state *state, float *features, float *logits,
                          int32_t *topk, int32_t *certified, int32_t *best);

/* Steps of the last planning call that took the certified proposal path
 * and that fell back to the full sweep.  Either pointer may be NULL. */
int fastmdp_proposal_stats(const fastmdp_ctx *ctx, int64_t *certified, int64_t *fallbacks);

/* Device memory for the DEVICE arguments above, for callers without an
 * allocator of their own (memory of the current HIP device; copies are
 * synchronous).  fastmdp_gather_rows copies n rows of row_bytes bytes:
 * dst row i = src row idx[i], zero if idx[i] is not in [0, n_src) (dst,
 * src, idx DEVICE; row_bytes a multiple of 4).  Errors: E_INVAL, E_NOMEM,
 * E_DEVICE. */
int fastmdp_device_alloc(int64_t bytes, void **ptr);
int fastmdp_device_free(void *ptr);
int fastmdp_copy_to_device(void *dst, const void *src, int64_t bytes);
int fastmdp_copy_to_host(void *dst, const void *src, int64_t bytes);
int fastmdp_gather_rows(void *dst, const void *src, int64_t n_src, const int64_t *idx, int64_t n,
                        int32_t row_bytes);

/* Static description of an error code or plan status (never NULL). */
const char *fastmdp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* FASTMDP_H */
