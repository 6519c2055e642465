/*
 * FP64 CPU oracle for FastMDP first-come-first-served pre-departure planning.
 * TEST INFRASTRUCTURE ONLY -- see fastmdp_oracle.h for scope and readings.
 *
 * Written to be checked against the paper by eye: every per-peak term is
 * evaluated literally (one distance, one radius test and one discount power
 * per peak, then a maximum), in the order of the paper's algorithms.  No
 * blocking, no min-distance shortcut, no reuse across actions.
 */
#include "fastmdp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t t0, n;
    float *xyz;          /* n points, FP32 (the table's storage format) */
} orc_plan_rec;

struct orc_world {
    orc_config cfg;
    double ell;          /* metres per step at the fastest speed */
    int32_t n_plans, cap_plans;
    orc_plan_rec *plans;
    int32_t tnx, tny;
    float *terr;
    double tx0, ty0, tcell;
};

static double max_speed(const orc_config *c) {
    double m = 0.0;
    for (int v = 0; v < c->n_speed; ++v)
        if (c->speed[v] > m) m = c->speed[v];
    return m;
}

int orc_create(const orc_config *cfg, orc_world **out) {
    if (!cfg || !out) return ORC_E_INVAL;
    if (cfg->n_head < 1 || cfg->n_climb < 1 || cfg->n_speed < 1 ||
        cfg->n_climb > ORC_MAX_ACT_DIM || cfg->n_speed > ORC_MAX_ACT_DIM || cfg->dt <= 0.0)
        return ORC_E_INVAL;
    orc_world *w = (orc_world *)calloc(1, sizeof(orc_world));
    if (!w) return ORC_E_NOMEM;
    w->cfg = *cfg;
    w->ell = max_speed(cfg) * cfg->dt;
    if (!(w->ell > 0.0)) { free(w); return ORC_E_INVAL; }
    *out = w;
    return 0;
}

void orc_destroy(orc_world *w) {
    if (!w) return;
    for (int j = 0; j < w->n_plans; ++j) free(w->plans[j].xyz);
    free(w->plans);
    free(w->terr);
    free(w);
}

int orc_num_plans(const orc_world *w) { return w ? w->n_plans : ORC_E_INVAL; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_add_plan(orc_world *w, int32_t t0, int32_t n, const float *xyz) {
    if (!w || n < 1 || t0 < 0 || !xyz) return ORC_E_INVAL;
    if (w->n_plans == w->cap_plans) {
        int32_t nc = w->cap_plans ? 2 * w->cap_plans : 64;
        orc_plan_rec *p = (orc_plan_rec *)realloc(w->plans, (size_t)nc * sizeof(orc_plan_rec));
        if (!p) return ORC_E_NOMEM;
        w->plans = p;
        w->cap_plans = nc;
    }
    float *copy = (float *)malloc((size_t)n * 3 * sizeof(float));
    if (!copy) return ORC_E_NOMEM;
    memcpy(copy, xyz, (size_t)n * 3 * sizeof(float));
    w->plans[w->n_plans].t0 = t0;
    w->plans[w->n_plans].n = n;
    w->plans[w->n_plans].xyz = copy;
    w->n_plans++;
    return 0;
}

int orc_set_terrain(orc_world *w, int32_t nx, int32_t ny, const float *h,
                    double x0, double y0, double cell) {
    if (!w || nx < 2 || ny < 2 || !h || !(cell > 0.0)) return ORC_E_INVAL;
    float *copy = (float *)malloc((size_t)nx * ny * sizeof(float));
    if (!copy) return ORC_E_NOMEM;
    memcpy(copy, h, (size_t)nx * ny * sizeof(float));
    free(w->terr);
    w->terr = copy;
    w->tnx = nx; w->tny = ny; w->tx0 = x0; w->ty0 = y0; w->tcell = cell;
    return 0;
}

/* Plan j's position at time row t, if it is active there. */
static int plan_point(const orc_plan_rec *p, int32_t t, double q[3]) {
    if (t < p->t0 || t >= p->t0 + p->n) return 0;
    const float *x = p->xyz + (size_t)(t - p->t0) * 3;
    q[0] = (double)x[0]; q[1] = (double)x[1]; q[2] = (double)x[2];
    return 1;
}

static double dist3(const double a[3], const double b[3]) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Terrain height: bilinear interpolation of the vertex grid, the position
 * clamped to the grid's extent. */
static double terrain_height(const orc_world *w, double x, double y) {
    double fx = (x - w->tx0) / w->tcell;
    double fy = (y - w->ty0) / w->tcell;
    if (fx < 0.0) fx = 0.0;
    if (fy < 0.0) fy = 0.0;
    if (fx > (double)(w->tnx - 1)) fx = (double)(w->tnx - 1);
    if (fy > (double)(w->tny - 1)) fy = (double)(w->tny - 1);
    int i = (int)floor(fx), j = (int)floor(fy);
    if (i > w->tnx - 2) i = w->tnx - 2;
    if (j > w->tny - 2) j = w->tny - 2;
    double ax = fx - i, ay = fy - j;
    double h00 = w->terr[(size_t)j * w->tnx + i];
    double h10 = w->terr[(size_t)j * w->tnx + i + 1];
    double h01 = w->terr[(size_t)(j + 1) * w->tnx + i];
    double h11 = w->terr[(size_t)(j + 1) * w->tnx + i + 1];
    return (1.0 - ay) * ((1.0 - ax) * h00 + ax * h10) + ay * ((1.0 - ax) * h01 + ax * h11);
}

static int outside_box(const orc_config *c, const double p[3]) {
    for (int k = 0; k < 3; ++k)
        if (p[k] < c->box_min[k] || p[k] > c->box_max[k]) return 1;
    return 0;
}

/* Forward projection of one action held for w steps: heading offset
 * 2*pi*h/H from the goal bearing beta, horizontal speed v, climb rate c,
 * for w * dt ("Forward project" kernel; w = 1 is the successor). */
static void window_point(const orc_config *c, const double s[3], double beta, int a, int w, double out[3]) {
    int v = a % c->n_speed;
    int cl = (a / c->n_speed) % c->n_climb;
    int h = a / (c->n_speed * c->n_climb);
    double th = beta + 2.0 * M_PI * (double)h / (double)c->n_head;
    double k = (double)w;
    double step = c->speed[v] * c->dt;
    out[0] = s[0] + (k * step) * cos(th);
    out[1] = s[1] + (k * step) * sin(th);
    out[2] = s[2] + k * (c->climb[cl] * c->dt);
}

static void successor(const orc_config *c, const double s[3], double beta, int a, double out[3]) {
    window_point(c, s, beta, a, 1, out);
}

static int window(const orc_config *c) { return c->lookahead > 1 ? c->lookahead : 1; }

/* Intruder risk well at point p and row t: the largest [d < R] |r| gamma^(d/ell)
 * over the plans active at row t, one peak per plan, evaluated literally.
 * Also the nearest plan distance and whether any distance lies within the
 * boundary band of the radius. */
static double intruder_term(const orc_world *w, const double p[3], int32_t t, const double *state, double *dnear,
                            int *amb) {
    const orc_config *c = &w->cfg;
    double Ineg = 0.0, dn = INFINITY;
    for (int j = 0; j < w->n_plans; ++j) {
        double q[3];
        if (!plan_point(&w->plans[j], t, q)) continue;
        /* range query: only plans within range_radius of the state */
        if (state && c->range_radius > 0.0 && dist3(state, q) >= c->range_radius) continue;
        double d = dist3(p, q);
        int in = d < c->R_intr;
        double val = in ? fabs(c->r_intr) * pow(c->gamma_intr, d / w->ell) : 0.0;
        if (val > Ineg) Ineg = val;
        if (d < dn) dn = d;
        if (fabs(d - c->R_intr) <= c->amb_band) *amb = 1;
    }
    *dnear = dn;
    return Ineg;
}

/* Terrain clearance well at point p (0 without terrain). */
static double terrain_term(const orc_world *w, const double p[3], int *amb) {
    const orc_config *c = &w->cfg;
    if (!w->terr) return 0.0;
    double clr = p[2] - terrain_height(w, p[0], p[1]);
    int in = clr < c->R_terr;
    if (fabs(clr - c->R_terr) <= c->amb_band) *amb = 1;
    return in ? fabs(c->r_terr) * pow(c->gamma_terr, (clr > 0.0 ? clr : 0.0) / w->ell) : 0.0;
}

static double goal_bearing(const double s[3], const double g[3]) {
    double dx = g[0] - s[0], dy = g[1] - s[1];
    if (dx == 0.0 && dy == 0.0) return 0.0;
    return atan2(dy, dx);
}

/* Argmax with the tie band: the lowest index among values within tie_rel
 * (relative) of the maximum.  -1 if every value is -inf. */
static int select_action(const double *V, int A, double tie_rel) {
    double vmax = -INFINITY;
    for (int a = 0; a < A; ++a)
        if (V[a] > vmax) vmax = V[a];
    if (vmax == -INFINITY) return -1;
    double thr = vmax - tie_rel * fabs(vmax);
    for (int a = 0; a < A; ++a)
        if (V[a] >= thr) return a;
    return -1;
}

/* Risk wells of the peaks built from other aircraft of a co-simulated batch
 * (peaks[4k..4k+3] = x, y, z, radius): the largest [d < R_k] |r| gamma^(d/ell),
 * one peak at a time. */
static double mate_term(const orc_world *w, const double p[3], const double *peaks, int np, int *amb) {
    const orc_config *c = &w->cfg;
    double M = 0.0;
    for (int k = 0; k < np; ++k) {
        const double *q = peaks + 4 * k;
        double d = dist3(p, q);
        int in = d < q[3];
        double val = in ? fabs(c->r_intr) * pow(c->gamma_intr, d / w->ell) : 0.0;
        if (val > M) M = val;
        if (fabs(d - q[3]) <= c->amb_band) *amb = 1;
    }
    return M;
}

static int eval_core(const orc_world *w, const double s[3], const double g[3], int32_t t, const double *peaks,
                     int np, double *V, double *G, double *I, double *T, double *dmin, int32_t *amb, int32_t *best);

int orc_eval_step(const orc_world *w, const double s[3], const double g[3], int32_t t,
                  double *V, double *G, double *I, double *T, double *dmin,
                  int32_t *amb, int32_t *best) {
    return eval_core(w, s, g, t, NULL, 0, V, G, I, T, dmin, amb, best);
}

/* Score every action; with np > 0 the peaks of the other aircraft of a
 * co-simulated batch add their wells ("Process negative rewards"), and the
 * value is the goal term less the largest of the three penalty classes
 * ("Compute value"); I then reports the larger of the intruder and batch
 * wells. */
static int eval_core(const orc_world *w, const double s[3], const double g[3], int32_t t, const double *peaks,
                     int np, double *V, double *G, double *I, double *T, double *dmin, int32_t *amb, int32_t *best) {
    if (!w || !s || !g || t < 0) return ORC_E_INVAL;
    const orc_config *c = &w->cfg;
    const int A = c->n_head * c->n_climb * c->n_speed;
    double *Vloc = (double *)malloc((size_t)A * sizeof(double));
    if (!Vloc) return ORC_E_NOMEM;
    const double beta = goal_bearing(s, g);
    const double ell = w->ell;

#pragma omp parallel for schedule(static)
    for (int a = 0; a < A; ++a) {
        double Vb = -INFINITY, Gb = 0.0, Ib = 0.0, Tb = 0.0, d1 = INFINITY;
        int ambiguous = 0, inside1 = 1;
        for (int k = 1; k <= window(c); ++k) {
            double sp[3];
            window_point(c, s, beta, a, k, sp);

            /* positive peak: the goal */
            double dg = dist3(g, sp);
            double Gp = fabs(c->r_goal) * pow(c->gamma, dg / ell);

            /* negative peaks: one risk well per plan active at this point's
             * time, and the terrain clearance well */
            double dnear;
            double Ineg = intruder_term(w, sp, t + k, s, &dnear, &ambiguous);
            if (np > 0) {
                double Mneg = mate_term(w, sp, peaks, np, &ambiguous);
                if (Mneg > Ineg) Ineg = Mneg;
            }
            double Tneg = terrain_term(w, sp, &ambiguous);

            double value = Gp - (Ineg > Tneg ? Ineg : Tneg);
            if (outside_box(c, sp)) value = -INFINITY;
            if (k == 1) {
                d1 = dnear;
                inside1 = value > -INFINITY;
                Vb = value; Gb = Gp; Ib = Ineg; Tb = Tneg;
            } else if (value > Vb) {
                Vb = value; Gb = Gp; Ib = Ineg; Tb = Tneg;
            }
        }
        /* the step itself must stay inside the box */
        double value = inside1 ? Vb : -INFINITY;

        Vloc[a] = value;
        if (V) V[a] = value;
        if (G) G[a] = Gb;
        if (I) I[a] = Ib;
        if (T) T[a] = Tb;
        if (dmin) dmin[a] = d1;
        if (amb) amb[a] = ambiguous;
    }
    if (best) *best = select_action(Vloc, A, c->tie_rel);
    free(Vloc);
    return 0;
}

/* Clearance below zero or any plan within R_sep at row t. */
static int origin_blocked(const orc_world *w, const double s[3], int32_t t) {
    const orc_config *c = &w->cfg;
    if (outside_box(c, s)) return 1;
    for (int j = 0; j < w->n_plans; ++j) {
        double q[3];
        if (plan_point(&w->plans[j], t, q) && dist3(s, q) < c->R_sep) return 1;
    }
    if (w->terr && s[2] - terrain_height(w, s[0], s[1]) < 0.0) return 1;
    return 0;
}

int orc_plan(const orc_world *w, const double origin[3], const double goal[3], int32_t t0,
             int32_t cap, double *xyz, int32_t *act, double *val,
             int32_t *n_pts, int32_t *status) {
    if (!w || !origin || !goal || t0 < 0 || cap < 1 || !xyz || !act || !val || !n_pts || !status)
        return ORC_E_INVAL;
    const orc_config *c = &w->cfg;
    const int A = c->n_head * c->n_climb * c->n_speed;
    double *V = (double *)malloc((size_t)A * sizeof(double));
    double *I = (double *)malloc((size_t)A * sizeof(double));
    double *T = (double *)malloc((size_t)A * sizeof(double));
    if (!V || !I || !T) { free(V); free(I); free(T); return ORC_E_NOMEM; }

    double s[3] = {origin[0], origin[1], origin[2]};
    int32_t n = 0, t = t0, st = ORC_TIMEOUT;
    xyz[0] = s[0]; xyz[1] = s[1]; xyz[2] = s[2];
    act[0] = -1; val[0] = 0.0;
    n = 1;
    if (origin_blocked(w, s, t0)) {
        st = ORC_REJECT_ORIGIN;
    } else {
        for (int32_t k = 0;; ++k) {
            if (dist3(goal, s) <= w->ell) { st = ORC_OK; break; }
            if (k == c->max_steps || n == cap) { st = ORC_TIMEOUT; break; }
            int best = -1;
            orc_eval_step(w, s, goal, t, V, NULL, I, T, NULL, NULL, &best);
            if (best < 0) { st = ORC_NO_VALID_ACTION; break; }
            double sp[3];
            successor(c, s, goal_bearing(s, goal), best, sp);
            s[0] = sp[0]; s[1] = sp[1]; s[2] = sp[2];
            t += 1;
            xyz[3 * n + 0] = s[0]; xyz[3 * n + 1] = s[1]; xyz[3 * n + 2] = s[2];
            act[n] = best; val[n] = V[best];
            n += 1;
            /* stop at the first collision: inside an intruder well means a
             * plan closer than the separation radius at this time (the
             * chosen successor's own well, whatever the window scored) */
            double dn;
            int amb_unused = 0;
            if (intruder_term(w, s, t, NULL, &dn, &amb_unused) > 0.0) { st = ORC_REJECT_SEPARATION; break; }
            if (w->terr && s[2] - terrain_height(w, s[0], s[1]) < 0.0) { st = ORC_REJECT_TERRAIN; break; }
        }
    }
    *n_pts = n;
    *status = st;
    free(V); free(I); free(T);
    return 0;
}

/* Time offsets [s] of the five peaks placed along another aircraft's
 * extrapolated track (Table "Peaks created in the environment"). */
static const double mate_tau[ORC_MATE_PEAKS] = {-5.0, 0.0, 5.0, 10.0, 15.0};

int orc_plan_batch(const orc_world *w, int32_t n, const double *origins, const double *goals, int32_t t0,
                   int32_t cap, double *xyz, int32_t *act, double *val, int32_t *n_pts, int32_t *status) {
    if (!w || n < 1 || !origins || !goals || t0 < 0 || cap < 1 || !xyz || !act || !val || !n_pts || !status)
        return ORC_E_INVAL;
    const orc_config *c = &w->cfg;
    const int A = c->n_head * c->n_climb * c->n_speed;
    double *V = (double *)malloc((size_t)A * sizeof(double));
    double *peaks = (double *)malloc((size_t)n * ORC_MATE_PEAKS * 4 * sizeof(double));
    int32_t *choice = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    double *vals = (double *)malloc((size_t)n * sizeof(double));
    int *moved = (int *)malloc((size_t)n * sizeof(int));
    if (!V || !peaks || !choice || !vals || !moved) {
        free(V); free(peaks); free(choice); free(vals); free(moved);
        return ORC_E_NOMEM;
    }
    /* aircraft i's point k is xyz[(i * cap + k) * 3] */
    for (int i = 0; i < n; ++i) {
        double *x = xyz + (size_t)i * cap * 3;
        x[0] = origins[3 * i]; x[1] = origins[3 * i + 1]; x[2] = origins[3 * i + 2];
        act[(size_t)i * cap] = -1;
        val[(size_t)i * cap] = 0.0;
        n_pts[i] = 1;
        status[i] = origin_blocked(w, x, t0) ? ORC_REJECT_ORIGIN : -1;   /* -1: flying */
    }
    for (int32_t k = 0;; ++k) {
        const int32_t t = t0 + k;
        /* 1. goal capture and step limit of every aircraft still flying */
        int flying = 0;
        for (int i = 0; i < n; ++i) {
            if (status[i] != -1) continue;
            const double *s = xyz + ((size_t)i * cap + n_pts[i] - 1) * 3;
            if (dist3(goals + 3 * i, s) <= w->ell) status[i] = ORC_OK;
            else if (k == c->max_steps || n_pts[i] == cap) status[i] = ORC_TIMEOUT;
            else flying += 1;
        }
        if (!flying) break;
        /* 2.-3. every flying aircraft scores its actions against the known
         * plans, the terrain and the five peaks of every other flying
         * aircraft, built from its position and velocity now (the set of
         * flying aircraft is the one at the start of the step: choices are
         * made before any of them is applied) */
        for (int i = 0; i < n; ++i) moved[i] = status[i] == -1;   /* flying in this step */
        for (int i = 0; i < n; ++i) {
            choice[i] = -1;
            if (!moved[i]) continue;
            int np = 0;
            for (int j = 0; j < n; ++j) {
                if (j == i || !moved[j]) continue;
                const double *pj = xyz + ((size_t)j * cap + n_pts[j] - 1) * 3;
                double vj[3] = {0.0, 0.0, 0.0};
                if (n_pts[j] > 1) {
                    const double *qj = pj - 3;
                    for (int a = 0; a < 3; ++a) vj[a] = (pj[a] - qj[a]) / c->dt;
                }
                for (int m = 0; m < ORC_MATE_PEAKS; ++m, ++np) {
                    double *pk = peaks + 4 * np;
                    for (int a = 0; a < 3; ++a) pk[a] = pj[a] + vj[a] * mate_tau[m];
                    pk[3] = c->R_intr + c->peak_growth * mate_tau[m];
                }
            }
            const double *s = xyz + ((size_t)i * cap + n_pts[i] - 1) * 3;
            int best = -1;
            eval_core(w, s, goals + 3 * i, t, peaks, np, V, NULL, NULL, NULL, NULL, NULL, &best);
            choice[i] = best;
            vals[i] = best >= 0 ? V[best] : 0.0;
        }
        /* 4. all apply their choices */
        for (int i = 0; i < n; ++i) {
            if (!moved[i]) continue;
            if (choice[i] < 0) {
                status[i] = ORC_NO_VALID_ACTION;
                moved[i] = 0;
                continue;
            }
            const double *s = xyz + ((size_t)i * cap + n_pts[i] - 1) * 3;
            double sp[3];
            successor(c, s, goal_bearing(s, goals + 3 * i), choice[i], sp);
            double *x = xyz + ((size_t)i * cap + n_pts[i]) * 3;
            x[0] = sp[0]; x[1] = sp[1]; x[2] = sp[2];
            act[(size_t)i * cap + n_pts[i]] = choice[i];
            val[(size_t)i * cap + n_pts[i]] = vals[i];
            n_pts[i] += 1;
        }
        /* 5. collisions at the new positions: a known plan within its well
         * (R_intr = R_sep), another aircraft of the batch that moved in this
         * step closer than R_sep, the terrain */
        for (int i = 0; i < n; ++i) {
            if (!moved[i]) continue;
            const double *x = xyz + ((size_t)i * cap + n_pts[i] - 1) * 3;
            double dn;
            int amb_unused = 0;
            int hit = intruder_term(w, x, t + 1, NULL, &dn, &amb_unused) > 0.0;
            for (int j = 0; j < n && !hit; ++j)
                if (j != i && moved[j] && dist3(x, xyz + ((size_t)j * cap + n_pts[j] - 1) * 3) < c->R_sep) hit = 1;
            if (hit) status[i] = ORC_REJECT_SEPARATION;
            else if (w->terr && x[2] - terrain_height(w, x[0], x[1]) < 0.0) status[i] = ORC_REJECT_TERRAIN;
        }
    }
    free(V); free(peaks); free(choice); free(vals); free(moved);
    return 0;
}

int orc_commit(orc_world *w, int32_t t0, int32_t n, const double *xyz) {
    if (!w || t0 < 0 || n < 1 || !xyz) return ORC_E_INVAL;
    const orc_config *c = &w->cfg;
    float *f = (float *)malloc((size_t)n * 3 * sizeof(float));
    if (!f) return ORC_E_NOMEM;
    for (int32_t k = 0; k < 3 * n; ++k) f[k] = (float)xyz[k];
    /* the trajectory as planned is checked against the plans as stored */
    for (int32_t k = 0; k < n; ++k) {
        const double *x = xyz + 3 * k;
        for (int j = 0; j < w->n_plans; ++j) {
            double q[3];
            if (plan_point(&w->plans[j], t0 + k, q) && dist3(x, q) < c->R_sep) {
                free(f);
                return ORC_E_CONFLICT;
            }
        }
        if (w->terr && x[2] - terrain_height(w, x[0], x[1]) < 0.0) {
            free(f);
            return ORC_E_CONFLICT;
        }
    }
    int rc = orc_add_plan(w, t0, n, f);
    free(f);
    return rc;
}
