/*
 * Drives the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers.py with gcc -fsanitize=address,undefined).
 *
 * Input file (native endianness, written by the test from the seeded
 * scenario): int32 n_head, n_climb, n_speed, max_steps, n_plans, n_req,
 * nx, ny (nx = ny = 0 without terrain); float64 box_min[3], box_max[3], dt,
 * gamma, r_goal, r_intr, R_intr, gamma_intr, R_sep, r_terr, R_terr,
 * gamma_terr, tie_rel, amb_band, climb[n_climb], speed[n_speed], and with
 * terrain x0, y0, cell; int32 t0[n_plans], len[n_plans]; float32 plan
 * points [sum(len)][3]; float64 origins [n_req][3], goals [n_req][3];
 * int32 request rows [n_req]; float32 heights [ny][nx].
 *
 * Output (stdout): per request "q status n_points committed x y z" of the
 * last point, then one line per scored step of request 0's first state:
 * "eval best" and the values.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/fastmdp_oracle.h"

static int rd(FILE *f, void *p, size_t sz, size_t n) { return fread(p, sz, n, f) == n ? 0 : -1; }

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[8];
    if (rd(f, hdr, sizeof(int32_t), 8)) return 3;
    const int n_plans = hdr[4], n_req = hdr[5], nx = hdr[6], ny = hdr[7];
    orc_config c;
    memset(&c, 0, sizeof(c));
    c.n_head = hdr[0]; c.n_climb = hdr[1]; c.n_speed = hdr[2]; c.max_steps = hdr[3];
    if (c.n_climb > ORC_MAX_ACT_DIM || c.n_speed > ORC_MAX_ACT_DIM) return 3;
    double d[18];
    if (rd(f, d, sizeof(double), 18)) return 3;
    memcpy(c.box_min, d, 3 * sizeof(double));
    memcpy(c.box_max, d + 3, 3 * sizeof(double));
    c.dt = d[6]; c.gamma = d[7]; c.r_goal = d[8]; c.r_intr = d[9]; c.R_intr = d[10];
    c.gamma_intr = d[11]; c.R_sep = d[12]; c.r_terr = d[13]; c.R_terr = d[14]; c.gamma_terr = d[15];
    c.tie_rel = d[16]; c.amb_band = d[17];
    if (rd(f, c.climb, sizeof(double), c.n_climb) || rd(f, c.speed, sizeof(double), c.n_speed)) return 3;
    double tg[3] = {0, 0, 0};
    if (nx > 0 && rd(f, tg, sizeof(double), 3)) return 3;
    int32_t *t0 = malloc(sizeof(int32_t) * (n_plans ? n_plans : 1));
    int32_t *len = malloc(sizeof(int32_t) * (n_plans ? n_plans : 1));
    if (rd(f, t0, sizeof(int32_t), n_plans) || rd(f, len, sizeof(int32_t), n_plans)) return 3;
    size_t total = 0;
    for (int j = 0; j < n_plans; ++j) total += (size_t)len[j];
    float *pts = malloc(sizeof(float) * 3 * (total ? total : 1));
    double *org = malloc(sizeof(double) * 3 * n_req), *goal = malloc(sizeof(double) * 3 * n_req);
    int32_t *rows = malloc(sizeof(int32_t) * n_req);
    if (rd(f, pts, sizeof(float), 3 * total) || rd(f, org, sizeof(double), 3 * n_req) ||
        rd(f, goal, sizeof(double), 3 * n_req) || rd(f, rows, sizeof(int32_t), n_req))
        return 3;
    float *h = NULL;
    if (nx > 0) {
        h = malloc(sizeof(float) * (size_t)nx * ny);
        if (rd(f, h, sizeof(float), (size_t)nx * ny)) return 3;
    }
    fclose(f);

    orc_world *w = NULL;
    if (orc_create(&c, &w)) return 4;
    size_t o = 0;
    for (int j = 0; j < n_plans; ++j) {
        if (orc_add_plan(w, t0[j], len[j], pts + 3 * o)) return 4;
        o += (size_t)len[j];
    }
    if (h && orc_set_terrain(w, nx, ny, h, tg[0], tg[1], tg[2])) return 4;
    const int cap = c.max_steps + 1;
    double *xyz = malloc(sizeof(double) * 3 * cap), *val = malloc(sizeof(double) * cap);
    int32_t *act = malloc(sizeof(int32_t) * cap);
    for (int q = 0; q < n_req; ++q) {
        int32_t n = 0, st = 0;
        if (orc_plan(w, org + 3 * q, goal + 3 * q, rows[q], cap, xyz, act, val, &n, &st)) return 5;
        int committed = st == ORC_OK ? orc_commit(w, rows[q], n, xyz) == 0 : 0;
        printf("%d %d %d %d %.17g %.17g %.17g\n", q, st, n, committed, xyz[3 * (n - 1)], xyz[3 * (n - 1) + 1],
               xyz[3 * (n - 1) + 2]);
    }
    const int A = c.n_head * c.n_climb * c.n_speed;
    double *V = malloc(sizeof(double) * A), *G = malloc(sizeof(double) * A), *I = malloc(sizeof(double) * A);
    double *T = malloc(sizeof(double) * A), *D = malloc(sizeof(double) * A);
    int32_t *amb = malloc(sizeof(int32_t) * A), best = -2;
    if (orc_eval_step(w, org, goal, rows[0], V, G, I, T, D, amb, &best)) return 6;
    printf("eval %d", best);
    for (int a = 0; a < A; ++a) printf(" %.17g", V[a]);
    printf("\n");
    orc_destroy(w);
    free(t0); free(len); free(pts); free(org); free(goal); free(rows); free(h);
    free(xyz); free(val); free(act); free(V); free(G); free(I); free(T); free(D); free(amb);
    return 0;
}
