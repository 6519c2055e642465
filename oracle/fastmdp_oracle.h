/*
 * FP64 CPU oracle for FastMDP first-come-first-served pre-departure planning.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the HIP
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Bertram, Zambreno & Wei, "Scalable FastMDP for
 * Pre-departure Airspace Reservation and Strategic De-conflict"):
 *   - per step, every action's successor state is scored by the closed-form
 *     FastMDP value: a positive peak at the goal, r_g * gamma^(d/ell)
 *     (Alg. 1, positive-peak loop; "Process positive rewards" kernel), minus
 *     the larger of the intruder and terrain risk-well penalties, each a
 *     maximum over peaks of [d < R] * |r| * gamma^(d/ell) (Alg. 1,
 *     negative-peak loop; "Process negative intruder/terrain rewards"
 *     kernels; "Compute value" kernel);
 *   - the action with the largest value is taken (Alg. 1 argmax; "Select
 *     best action" kernel) and the state advances ("Determine terminal
 *     state" kernel);
 *   - the loop runs until the goal is reached or a collision occurs, and only
 *     a collision-free trajectory is accepted into the known-plan table
 *     (Sec. V, Experimental Setup).
 *
 * Readings where the paper is silent (all stated in the design notes):
 *   - distance in the discount exponent is measured in steps of
 *     ell = max_speed * dt metres;
 *   - one intruder peak per known plan, at that plan's own trajectory point
 *     at the time of the scored point;
 *   - lookahead window of W steps (Alg. 1's one-step and ten-step forward
 *     projections, "Forward project" and "Compute value" kernels): action a
 *     held for w = 1..W steps reaches s + w * Delta_a at row t + w; its
 *     value is the largest of the W point values (no floor at 0), -inf if
 *     the first point leaves the box (window points outside it are left
 *     out); the state advances by one step; W = 1 scores the successor
 *     alone;
 *   - range query (Sec. VII): with range_radius > 0 only the plans within
 *     that distance of the state take part in a step (dmin then reports the
 *     nearest of those);
 *   - kinematic action model: heading offsets 2*pi*h/H from the goal bearing,
 *     climb rates and speeds from the config; action index a = (h*C + c)*S + v;
 *   - the airspace box is a hard mask (value -inf outside);
 *   - argmax ties: values within 1e-9 (relative) of the maximum are equal,
 *     and the lowest action index among them is taken;
 *   - separation radius R_sep is checked on the sampled time grid.
 *
 * Parity pins (tests/test_oracle_pins.py): the worked risk-well example of
 * Fig. "riskwell", closed-form straight flight with no intruders, brute-force
 * value iteration on a 1-D chain, a min-distance cross-formulation of the
 * per-peak maximum, permutation and mirror invariances, the separation
 * invariant, and the acceptance rule.  FastMDP-versus-value-iteration with
 * risk wells is parity unpinned (the paper only claims a close
 * approximation).
 */
#ifndef FASTMDP_ORACLE_H
#define FASTMDP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_ACT_DIM 32

enum {
    ORC_OK = 0,
    ORC_REJECT_SEPARATION = 1,
    ORC_REJECT_TERRAIN = 2,
    ORC_REJECT_ORIGIN = 3,
    ORC_TIMEOUT = 4,
    ORC_NO_VALID_ACTION = 5
};

enum { ORC_E_INVAL = -1, ORC_E_CONFLICT = -4, ORC_E_NOMEM = -5 };

typedef struct {
    double box_min[3], box_max[3];
    double dt;
    double gamma, r_goal;                 /* positive peak (goal)          */
    double r_intr, R_intr, gamma_intr;    /* intruder risk well            */
    double R_sep;                         /* separation radius             */
    double r_terr, R_terr, gamma_terr;    /* terrain risk well (clearance) */
    int32_t n_head, n_climb, n_speed;
    double climb[ORC_MAX_ACT_DIM];        /* m/s, index c                  */
    double speed[ORC_MAX_ACT_DIM];        /* m/s, index v                  */
    int32_t max_steps;
    double tie_rel;                       /* argmax tie band (relative)    */
    double amb_band;                      /* boundary-ambiguity band [m]   */
    int32_t lookahead;                    /* window W >= 1 (0 reads as 1)  */
    double range_radius;                  /* > 0: plans farther than this
                                             from the state are skipped   */
    double peak_growth;                   /* batch peaks: radius R_intr +
                                             peak_growth * tau [m/s]      */
} orc_config;

#define ORC_MATE_PEAKS 5

typedef struct orc_world orc_world;

int  orc_create(const orc_config *cfg, orc_world **out);
void orc_destroy(orc_world *w);

/* Append a plan without validation (known plans loaded from the database). */
int  orc_add_plan(orc_world *w, int32_t t0, int32_t n, const float *xyz);
int  orc_num_plans(const orc_world *w);
/* Threads the per-action loop of orc_eval_step may use (OpenMP). */
int  orc_num_threads(void);

/* Heightmap h[j*nx+i] at (x0 + i*cell, y0 + j*cell); bilinear, clamped. */
int  orc_set_terrain(orc_world *w, int32_t nx, int32_t ny, const float *h,
                     double x0, double y0, double cell);

/* Score every action from state s at time row t: its window points
 * s + w * Delta_a against the plans active at row t + w, w = 1..W.
 * Outputs (length A each, any may be NULL): V value (the window maximum),
 * G goal term, I intruder term, T terrain term (the three at the window
 * point that gives V, the first such; at the first point when V = -inf),
 * dmin nearest-plan distance of the first point (inf if none), amb 1 if a
 * plan distance or a clearance of any window point lies within amb_band of
 * its radius.  *best = chosen action or -1 if every value is -inf. */
int  orc_eval_step(const orc_world *w, const double s[3], const double g[3], int32_t t,
                   double *V, double *G, double *I, double *T, double *dmin,
                   int32_t *amb, int32_t *best);

/* Plan one request from origin at row t0 towards goal.  Writes up to cap
 * points: xyz[k*3..], act[k] (-1 for the origin), val[k] (0 for the origin).
 * Returns 0 and sets *n_pts and *status, or a negative error. */
int  orc_plan(const orc_world *w, const double origin[3], const double goal[3], int32_t t0,
              int32_t cap, double *xyz, int32_t *act, double *val,
              int32_t *n_pts, int32_t *status);

/* Co-simulated batch (Sec. V: several aircraft planned together, aware of
 * each other and of every accepted plan): n aircraft departing at row t0,
 * in lockstep.  Each step: (1) an aircraft within ell of its goal is done
 * (OK), one that has taken max_steps times out; (2) every aircraft still
 * flying scores its actions against the known plans, the terrain and five
 * risk wells per other flying aircraft, placed along that aircraft's
 * extrapolated track at p + v*tau, tau in {-5, 0, 5, 10, 15} s, radius
 * R_intr + peak_growth*tau, magnitude |r_intr|, discount gamma_intr (Table
 * "Peaks created in the environment"; "Build peaks"; "Process negative
 * rewards"), with p its position and v its last step over dt (0 before its
 * first step), and chooses as for one aircraft; (3) all apply their choices
 * ("Now that all aircraft have selected an action, apply it"); (4) an
 * aircraft is rejected (REJECT_SEPARATION) if a known plan lies inside its
 * well at the new row or another aircraft that moved in this step is
 * closer than R_sep, and (REJECT_TERRAIN) if below the terrain.  Aircraft
 * i's points go to xyz[(i*cap + k)*3 ..], act[i*cap + k], val[i*cap + k];
 * n_pts[i], status[i] as for orc_plan.  Nothing is committed. */
int  orc_plan_batch(const orc_world *w, int32_t n, const double *origins, const double *goals, int32_t t0,
                    int32_t cap, double *xyz, int32_t *act, double *val, int32_t *n_pts, int32_t *status);

/* Validate a trajectory as planned (FP64) against every plan in the table
 * as stored (FP32) and against the terrain; if clear, append it rounded to
 * FP32.  Returns 0, or ORC_E_CONFLICT with the table unchanged. */
int  orc_commit(orc_world *w, int32_t t0, int32_t n, const double *xyz);

#ifdef __cplusplus
}
#endif
#endif
