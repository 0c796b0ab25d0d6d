/*
 * Plain FP64 CPU oracle for the squared Mallows distance and the
 * nearest-centroid labelling of D2-clustering.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: it exists so that the HIP path can be checked against an
 * independent, slow, obviously correct computation.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes (paper, Sec. 1.1, Eq. (1) with the centroid z fixed):
 * for P = {(x_a, p_a)}_{a<t} and Q = {(y_b, q_b)}_{b<s} in R^d,
 *
 *     D^2(P,Q) = min_{w >= 0} sum_a sum_b w_ab |x_a - y_b|^2
 *                subject to sum_b w_ab = p_a,  sum_a w_ab = q_b,
 *
 * with p and q probability vectors (the equal-mass constraints of Eq. (1)).
 * The label of object i is argmin_j D(v_i, z_j) (Alg. 2, Step 2).
 *
 * The paper does not say how it solves the per-pair linear program (it only
 * notes that linear programs are polynomial).  The oracle uses the classical
 * transportation simplex (Dantzig's u-v method), kept deliberately plain:
 *
 *   1. weights are divided by their FP64 sum (summed in index order);
 *      non-finite, negative or zero-sum weight vectors are rejected;
 *   2. C_ab = sum_k (x_ak - y_bk)^2, k = 0..d-1 in order (direct form);
 *   3. a starting basis of exactly t+s-1 cells forming a spanning tree of
 *      rows and columns, by the north-west-corner rule or by Vogel's
 *      approximation; where a row and a column run out together a zero
 *      ("degenerate") cell is kept so the basis stays a tree;
 *   4. every pivot recomputes the potentials from scratch: u_0 = 0 and
 *      u_a + v_b = C_ab on every basic cell, propagated over the tree;
 *   5. reduced costs r_ab = C_ab - u_a - v_b; stop when min r >= -delta with
 *      delta = 1e-14 * max C (the basis is then optimal for costs perturbed
 *      by at most delta, so the objective is within delta of the optimum);
 *   6. the entering cell is the most negative r (Dantzig), ties to the lowest
 *      row-major index; after 2(t+s) degenerate pivots in a row (or a
 *      caller-given streak length, `bland_after` > 0) the rule switches to
 *      Bland's (first negative cell in row-major order) until a pivot moves
 *      flow again;
 *   7. the cycle is the entering cell plus the tree path from its row to its
 *      column; signs alternate starting with + on the entering cell; theta
 *      is the least flow on a - cell and the leaving cell is the lowest
 *      row-major index among the - cells that reach theta;
 *   8. a pivot count above max(50 t s, 100) is reported as failure;
 *   9. the objective is sum over basic cells of w_ab C_ab in row-major order.
 *
 * Each solve also reports its pivot count and how many of those pivots were
 * taken under Bland's rule (step 6), so tests can show that a family of
 * inputs does reach the anti-cycling branch.
 *
 * oracle_emd_cost takes the ground cost as given instead of step 2 (any
 * finite values; non-finite ones give status 4), which serves the MM
 * distance of Eq. (10) and any other cost.
 *
 * Batches run over host threads, each pair independent (the labelling step
 * parallelises per point, Sec. 1.2).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "emd_oracle.h"

#define ORACLE_OK 0
#define ORACLE_BAD_WEIGHTS 1
#define ORACLE_TOO_LARGE 2
#define ORACLE_PIVOT_CAP 3
#define ORACLE_BAD_COST 4

/* ---------------------------------------------------------------- scratch */

typedef struct {
    int cap_t, cap_s;
    double *p, *q, *C, *u, *v, *rs, *rd;
    int *bi, *bj;       /* basic cells: row, column                    */
    double *bw;         /* flow on each basic cell                      */
    int *basic_at;      /* [t*s] index into the basis, or -1            */
    int *known_u, *known_v;
    int *queue, *pred_node, *pred_cell, *seen;
    int *path_cell;
    int *row_on, *col_on;
} scratch_t;

static void scratch_free(scratch_t *sc) {
    free(sc->p); free(sc->q); free(sc->C); free(sc->u); free(sc->v);
    free(sc->rs); free(sc->rd); free(sc->bi); free(sc->bj); free(sc->bw);
    free(sc->basic_at); free(sc->known_u); free(sc->known_v); free(sc->queue);
    free(sc->pred_node); free(sc->pred_cell); free(sc->seen); free(sc->path_cell);
    free(sc->row_on); free(sc->col_on);
    memset(sc, 0, sizeof(*sc));
}

static int scratch_init(scratch_t *sc, int t, int s) {
    int V = t + s;
    memset(sc, 0, sizeof(*sc));
    sc->cap_t = t; sc->cap_s = s;
    sc->p = malloc(sizeof(double) * t);
    sc->q = malloc(sizeof(double) * s);
    sc->C = malloc(sizeof(double) * (size_t)t * s);
    sc->u = malloc(sizeof(double) * t);
    sc->v = malloc(sizeof(double) * s);
    sc->rs = malloc(sizeof(double) * t);
    sc->rd = malloc(sizeof(double) * s);
    sc->bi = malloc(sizeof(int) * V);
    sc->bj = malloc(sizeof(int) * V);
    sc->bw = malloc(sizeof(double) * V);
    sc->basic_at = malloc(sizeof(int) * (size_t)t * s);
    sc->known_u = malloc(sizeof(int) * t);
    sc->known_v = malloc(sizeof(int) * s);
    sc->queue = malloc(sizeof(int) * V);
    sc->pred_node = malloc(sizeof(int) * V);
    sc->pred_cell = malloc(sizeof(int) * V);
    sc->seen = malloc(sizeof(int) * V);
    sc->path_cell = malloc(sizeof(int) * V);
    sc->row_on = malloc(sizeof(int) * t);
    sc->col_on = malloc(sizeof(int) * s);
    if (!sc->p || !sc->q || !sc->C || !sc->u || !sc->v || !sc->rs || !sc->rd || !sc->bi ||
        !sc->bj || !sc->bw || !sc->basic_at || !sc->known_u || !sc->known_v || !sc->queue ||
        !sc->pred_node || !sc->pred_cell || !sc->seen || !sc->path_cell || !sc->row_on ||
        !sc->col_on) {
        scratch_free(sc);
        return -1;
    }
    return 0;
}

/* ------------------------------------------------------------ steps 1, 2 */

/* Probability vector: divide by the FP64 sum (Eq. (1) needs unit mass). */
static int normalise(int n, const double *w, double *out) {
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!isfinite(w[i]) || w[i] < 0.0) return ORACLE_BAD_WEIGHTS;
        sum += w[i];
    }
    if (!(sum > 0.0) || !isfinite(sum)) return ORACLE_BAD_WEIGHTS;
    for (int i = 0; i < n; ++i) out[i] = w[i] / sum;
    return ORACLE_OK;
}

/* Squared-L2 ground cost, direct difference form. */
static void ground_cost(int t, int s, int d, const double *x, const double *y, double *C) {
    for (int a = 0; a < t; ++a)
        for (int b = 0; b < s; ++b) {
            double acc = 0.0;
            for (int k = 0; k < d; ++k) {
                double diff = x[(size_t)a * d + k] - y[(size_t)b * d + k];
                acc += diff * diff;
            }
            C[(size_t)a * s + b] = acc;
        }
}

/* ---------------------------------------------------------------- step 3 */

static void add_basic(scratch_t *sc, int *nb, int s, int a, int b, double w) {
    sc->bi[*nb] = a; sc->bj[*nb] = b; sc->bw[*nb] = w;
    sc->basic_at[(size_t)a * s + b] = *nb;
    (*nb)++;
}

/* North-west corner.  The last row takes each remaining column's demand and
 * the last column takes each remaining row's supply, so rounding leftovers
 * land on one line.  On a tie the rule moves down, keeping a zero cell. */
static int start_nwc(scratch_t *sc, int t, int s) {
    int nb = 0, a = 0, b = 0;
    memcpy(sc->rs, sc->p, sizeof(double) * t);
    memcpy(sc->rd, sc->q, sizeof(double) * s);
    for (;;) {
        double x;
        if (a == t - 1) x = sc->rd[b];
        else if (b == s - 1) x = sc->rs[a];
        else x = sc->rs[a] < sc->rd[b] ? sc->rs[a] : sc->rd[b];
        add_basic(sc, &nb, s, a, b, x);
        sc->rs[a] -= x;
        sc->rd[b] -= x;
        if (a == t - 1 && b == s - 1) break;
        if (a == t - 1) b++;
        else if (b == s - 1) a++;
        else if (sc->rs[a] <= sc->rd[b]) a++;
        else b++;
    }
    return nb;
}

/* Vogel's approximation: repeatedly take the line (row or column) whose two
 * cheapest open cells differ most, fill its cheapest open cell as far as the
 * remaining supply/demand allows, and close one exhausted line.  Ties: larger
 * penalty, then rows before columns, then lower index; within a line the
 * cheapest cell, ties to the lower index.  Once a single row (column) is open
 * it takes every open column's remaining demand (row's remaining supply). */
static int start_vogel(scratch_t *sc, int t, int s) {
    int nb = 0, nr = t, nc = s;
    const double *C = sc->C;
    memcpy(sc->rs, sc->p, sizeof(double) * t);
    memcpy(sc->rd, sc->q, sizeof(double) * s);
    for (int a = 0; a < t; ++a) sc->row_on[a] = 1;
    for (int b = 0; b < s; ++b) sc->col_on[b] = 1;
    for (;;) {
        if (nr == 1) {
            int a = 0;
            while (!sc->row_on[a]) a++;
            for (int b = 0; b < s; ++b)
                if (sc->col_on[b]) add_basic(sc, &nb, s, a, b, sc->rd[b]);
            return nb;
        }
        if (nc == 1) {
            int b = 0;
            while (!sc->col_on[b]) b++;
            for (int a = 0; a < t; ++a)
                if (sc->row_on[a]) add_basic(sc, &nb, s, a, b, sc->rs[a]);
            return nb;
        }
        double best_pen = -1.0;
        int best_is_row = 1, best_line = -1;
        for (int a = 0; a < t; ++a) {
            if (!sc->row_on[a]) continue;
            double c1 = INFINITY, c2 = INFINITY;
            for (int b = 0; b < s; ++b) {
                if (!sc->col_on[b]) continue;
                double c = C[(size_t)a * s + b];
                if (c < c1) { c2 = c1; c1 = c; }
                else if (c < c2) c2 = c;
            }
            double pen = c2 - c1;
            if (pen > best_pen) { best_pen = pen; best_is_row = 1; best_line = a; }
        }
        for (int b = 0; b < s; ++b) {
            if (!sc->col_on[b]) continue;
            double c1 = INFINITY, c2 = INFINITY;
            for (int a = 0; a < t; ++a) {
                if (!sc->row_on[a]) continue;
                double c = C[(size_t)a * s + b];
                if (c < c1) { c2 = c1; c1 = c; }
                else if (c < c2) c2 = c;
            }
            double pen = c2 - c1;
            if (pen > best_pen) { best_pen = pen; best_is_row = 0; best_line = b; }
        }
        int a, b;
        if (best_is_row) {
            a = best_line; b = -1;
            for (int j = 0; j < s; ++j)
                if (sc->col_on[j] && (b < 0 || C[(size_t)a * s + j] < C[(size_t)a * s + b])) b = j;
        } else {
            b = best_line; a = -1;
            for (int i = 0; i < t; ++i)
                if (sc->row_on[i] && (a < 0 || C[(size_t)i * s + b] < C[(size_t)a * s + b])) a = i;
        }
        double x = sc->rs[a] < sc->rd[b] ? sc->rs[a] : sc->rd[b];
        add_basic(sc, &nb, s, a, b, x);
        sc->rs[a] -= x;
        sc->rd[b] -= x;
        if (sc->rs[a] <= sc->rd[b]) { sc->row_on[a] = 0; nr--; }
        else { sc->col_on[b] = 0; nc--; }
    }
}

/* ---------------------------------------------------------------- step 4 */

/* u_0 = 0, then u_a + v_b = C_ab on basic cells, repeated sweeps over the
 * basis until every potential is fixed (the basis is a spanning tree). */
static void potentials(scratch_t *sc, int t, int s, int nb) {
    for (int a = 0; a < t; ++a) sc->known_u[a] = 0;
    for (int b = 0; b < s; ++b) sc->known_v[b] = 0;
    sc->u[0] = 0.0;
    sc->known_u[0] = 1;
    int fixed = 1, changed = 1;
    while (changed && fixed < t + s) {
        changed = 0;
        for (int e = 0; e < nb; ++e) {
            int a = sc->bi[e], b = sc->bj[e];
            double c = sc->C[(size_t)a * s + b];
            if (sc->known_u[a] && !sc->known_v[b]) {
                sc->v[b] = c - sc->u[a]; sc->known_v[b] = 1; fixed++; changed = 1;
            } else if (sc->known_v[b] && !sc->known_u[a]) {
                sc->u[a] = c - sc->v[b]; sc->known_u[a] = 1; fixed++; changed = 1;
            }
        }
    }
}

/* ---------------------------------------------------------------- step 7 */

/* Tree path from row node ra to column node cb (nodes: rows 0..t-1, columns
 * t..t+s-1), by breadth-first search over the basic cells.  Returns the
 * number of cells on the path; path_cell[0] touches column cb and the last
 * entry touches row ra. */
static int tree_path(scratch_t *sc, int t, int s, int nb, int ra, int cb) {
    int V = t + s, head = 0, tail = 0;
    for (int i = 0; i < V; ++i) sc->seen[i] = 0;
    sc->queue[tail++] = ra;
    sc->seen[ra] = 1;
    int target = t + cb;
    while (head < tail && !sc->seen[target]) {
        int node = sc->queue[head++];
        for (int e = 0; e < nb; ++e) {
            int other;
            if (node < t && sc->bi[e] == node) other = t + sc->bj[e];
            else if (node >= t && sc->bj[e] == node - t) other = sc->bi[e];
            else continue;
            if (sc->seen[other]) continue;
            sc->seen[other] = 1;
            sc->pred_node[other] = node;
            sc->pred_cell[other] = e;
            sc->queue[tail++] = other;
        }
    }
    int len = 0;
    for (int node = target; node != ra; node = sc->pred_node[node])
        sc->path_cell[len++] = sc->pred_cell[node];
    return len;
}

/* ----------------------------------------------------------- one LP solve */

/* `cost`, when given, is the t x s ground cost (row-major) to use instead of
 * step 2; it may hold any finite values (the transport LP with a general
 * cost, as in the MM distance of Eq. (10)).  The stopping tolerance is taken
 * against max |C|, which for the squared distances of step 2 is max C. */
static int solve_pair(scratch_t *sc, int t, int s, int d, const double *x, const double *pw,
                      const double *y, const double *qw, const double *cost, int init_rule,
                      int bland_after, double *d2_out, double *plan_out, double *u_out, double *v_out,
                      long long *pivots_out, long long *bland_out) {
    *d2_out = NAN;
    if (pivots_out) *pivots_out = 0;
    if (bland_out) *bland_out = 0;
    if (t < 1 || s < 1) return ORACLE_TOO_LARGE;
    if (normalise(t, pw, sc->p) != ORACLE_OK) return ORACLE_BAD_WEIGHTS;
    if (normalise(s, qw, sc->q) != ORACLE_OK) return ORACLE_BAD_WEIGHTS;
    if (cost) {
        for (size_t c = 0; c < (size_t)t * s; ++c) {
            if (!isfinite(cost[c])) return ORACLE_BAD_COST;
            sc->C[c] = cost[c];
        }
    } else {
        ground_cost(t, s, d, x, y, sc->C);
    }

    double cmax = 0.0;
    for (size_t c = 0; c < (size_t)t * s; ++c) {
        if (fabs(sc->C[c]) > cmax) cmax = fabs(sc->C[c]);
        sc->basic_at[c] = -1;
    }
    const double delta = 1e-14 * cmax;

    int nb = init_rule == ORACLE_INIT_VOGEL ? start_vogel(sc, t, s) : start_nwc(sc, t, s);

    long long cap = 50LL * t * s;
    if (cap < 100) cap = 100;
    long long pivots = 0, bland_pivots = 0;
    int degenerate_run = 0, bland = 0;
    for (;;) {
        potentials(sc, t, s, nb);
        /* pricing */
        int enter = -1;
        double rmin = -delta;
        for (int a = 0; a < t && !(bland && enter >= 0); ++a)
            for (int b = 0; b < s; ++b) {
                size_t c = (size_t)a * s + b;
                if (sc->basic_at[c] >= 0) continue;
                double r = sc->C[c] - sc->u[a] - sc->v[b];
                if (r < rmin) {
                    rmin = r;
                    enter = (int)c;
                    if (bland) break;
                }
            }
        if (enter < 0) break;
        if (pivots >= cap) {
            if (pivots_out) *pivots_out = pivots;
            if (bland_out) *bland_out = bland_pivots;
            return ORACLE_PIVOT_CAP;
        }
        int ea = enter / s, eb = enter % s;
        int len = tree_path(sc, t, s, nb, ea, eb);
        /* path_cell[0] touches column eb: sign -, then +, -, ... */
        double theta = INFINITY;
        int leave = -1;
        for (int k = 0; k < len; k += 2) {
            int e = sc->path_cell[k];
            size_t idx = (size_t)sc->bi[e] * s + sc->bj[e];
            size_t lidx = leave < 0 ? 0 : (size_t)sc->bi[leave] * s + sc->bj[leave];
            if (sc->bw[e] < theta || (sc->bw[e] == theta && idx < lidx)) {
                theta = sc->bw[e];
                leave = e;
            }
        }
        for (int k = 0; k < len; ++k) {
            int e = sc->path_cell[k];
            if (k % 2 == 0) sc->bw[e] -= theta;
            else sc->bw[e] += theta;
        }
        sc->basic_at[(size_t)sc->bi[leave] * s + sc->bj[leave]] = -1;
        sc->bi[leave] = ea;
        sc->bj[leave] = eb;
        sc->bw[leave] = theta;
        sc->basic_at[enter] = leave;
        pivots++;
        if (bland) bland_pivots++;
        if (theta == 0.0) {
            degenerate_run++;
            if (degenerate_run >= (bland_after > 0 ? bland_after : 2 * (t + s))) bland = 1;
        } else {
            degenerate_run = 0;
            bland = 0;
        }
    }

    double obj = 0.0;
    for (int a = 0; a < t; ++a)
        for (int b = 0; b < s; ++b) {
            int e = sc->basic_at[(size_t)a * s + b];
            if (e >= 0) obj += sc->bw[e] * sc->C[(size_t)a * s + b];
        }
    *d2_out = obj;
    if (plan_out) {
        for (size_t c = 0; c < (size_t)t * s; ++c) {
            int e = sc->basic_at[c];
            plan_out[c] = e >= 0 ? sc->bw[e] : 0.0;
        }
    }
    if (u_out) memcpy(u_out, sc->u, sizeof(double) * t);
    if (v_out) memcpy(v_out, sc->v, sizeof(double) * s);
    if (pivots_out) *pivots_out = pivots;
    if (bland_out) *bland_out = bland_pivots;
    return ORACLE_OK;
}

int oracle_emd_pair(int t, int s, int d, const double *x, const double *p, const double *y,
                    const double *q, int init_rule, int bland_after, double *d2_out, double *plan_out,
                    double *u_out, double *v_out, long long *pivots_out, long long *bland_out) {
    scratch_t sc;
    if (t < 1 || s < 1 || d < 1) return ORACLE_TOO_LARGE;
    if (scratch_init(&sc, t, s) != 0) return -1;
    int st = solve_pair(&sc, t, s, d, x, p, y, q, NULL, init_rule, bland_after, d2_out, plan_out,
                        u_out, v_out, pivots_out, bland_out);
    scratch_free(&sc);
    return st;
}

int oracle_emd_cost(int t, int s, const double *cost, const double *p, const double *q,
                    int init_rule, int bland_after, double *d2_out, double *plan_out, double *u_out, double *v_out,
                    long long *pivots_out, long long *bland_out) {
    scratch_t sc;
    if (t < 1 || s < 1 || !cost) return ORACLE_TOO_LARGE;
    if (scratch_init(&sc, t, s) != 0) return -1;
    int st = solve_pair(&sc, t, s, 1, NULL, p, NULL, q, cost, init_rule, bland_after, d2_out,
                        plan_out, u_out, v_out, pivots_out, bland_out);
    scratch_free(&sc);
    return st;
}

/* ---------------------------------------------------------------- batches */

typedef struct {
    int d;
    const int64_t *offA; const double *xA; const double *wA;
    const int64_t *offB; const double *xB; const double *wB;
    int64_t nA, nB;
    int init, bland_after;
    /* mode 0: explicit pairs; 1: all (i,j) of A x B with argmin; 2: i<j of A */
    int mode;
    const int64_t *pairs;
    int64_t npairs;
    double *dist; int32_t *status; long long *pivots, *bland;
    int32_t *labels; double *best;
    int max_t, max_s;
    int64_t begin, end;   /* chunk: pairs (modes 0, 2) or rows (mode 1) */
    int failed_alloc;
} job_t;

static int solve_ij(scratch_t *sc, const job_t *J, int64_t i, int64_t j, double *out,
                    long long *piv, long long *bl) {
    int64_t a0 = J->offA[i], a1 = J->offA[i + 1];
    int64_t b0 = J->offB[j], b1 = J->offB[j + 1];
    int t = (int)(a1 - a0), s = (int)(b1 - b0);
    if (t < 1 || s < 1 || t > J->max_t || s > J->max_s) { *out = NAN; return ORACLE_TOO_LARGE; }
    return solve_pair(sc, t, s, J->d, J->xA + a0 * J->d, J->wA + a0, J->xB + b0 * J->d,
                      J->wB + b0, NULL, J->init, J->bland_after, out, NULL, NULL, NULL, piv, bl);
}

/* Pair k of the strict upper triangle, row-major: row i holds n-1-i pairs. */
static void condensed_to_ij(int64_t n, int64_t k, int64_t *i, int64_t *j) {
    int64_t row = 0, start = 0;
    while (start + (n - 1 - row) <= k) { start += n - 1 - row; row++; }
    *i = row;
    *j = row + 1 + (k - start);
}

static void *worker(void *arg) {
    job_t *J = (job_t *)arg;
    scratch_t sc;
    if (scratch_init(&sc, J->max_t, J->max_s) != 0) { J->failed_alloc = 1; return NULL; }
    if (J->mode == 0) {
        for (int64_t k = J->begin; k < J->end; ++k) {
            long long piv = 0, bl = 0;
            int st = solve_ij(&sc, J, J->pairs[2 * k], J->pairs[2 * k + 1], &J->dist[k], &piv, &bl);
            if (J->status) J->status[k] = st;
            if (J->pivots) J->pivots[k] = piv;
            if (J->bland) J->bland[k] = bl;
        }
    } else if (J->mode == 1) {
        for (int64_t i = J->begin; i < J->end; ++i) {
            int label = -1, worst = ORACLE_OK;
            double bestv = INFINITY;
            for (int64_t j = 0; j < J->nB; ++j) {
                double dv;
                long long piv = 0, bl = 0;
                int st = solve_ij(&sc, J, i, j, &dv, &piv, &bl);
                if (J->dist) J->dist[i * J->nB + j] = dv;
                if (J->pivots) J->pivots[i * J->nB + j] = piv;
                if (J->bland) J->bland[i * J->nB + j] = bl;
                if (st != ORACLE_OK) { if (st > worst) worst = st; continue; }
                if (dv < bestv) { bestv = dv; label = (int)j; }   /* ties: lowest j */
            }
            if (worst != ORACLE_OK) { label = -1; bestv = NAN; }
            J->labels[i] = label;
            J->best[i] = bestv;
            if (J->status) J->status[i] = worst;
        }
    } else {
        int64_t i, j;
        if (J->begin < J->end) condensed_to_ij(J->nA, J->begin, &i, &j);
        for (int64_t k = J->begin; k < J->end; ++k) {
            long long piv = 0, bl = 0;
            int st = solve_ij(&sc, J, i, j, &J->dist[k], &piv, &bl);
            if (J->status) J->status[k] = st;
            if (J->pivots) J->pivots[k] = piv;
            if (J->bland) J->bland[k] = bl;
            if (++j == J->nA) { i++; j = i + 1; }
        }
    }
    scratch_free(&sc);
    return NULL;
}

static int max_support(const int64_t *off, int64_t n) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] - off[i] > m) m = off[i + 1] - off[i];
    return (int)m;
}

static int run_jobs(job_t *proto, int64_t total, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (total < nthreads) nthreads = total > 0 ? (int)total : 1;
    job_t *jobs = calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -1; }
    int64_t chunk = (total + nthreads - 1) / nthreads;
    int rc = 0;
    for (int k = 0; k < nthreads; ++k) {
        jobs[k] = *proto;
        jobs[k].begin = (int64_t)k * chunk < total ? (int64_t)k * chunk : total;
        jobs[k].end = jobs[k].begin + chunk < total ? jobs[k].begin + chunk : total;
        if (pthread_create(&th[k], NULL, worker, &jobs[k]) != 0) { rc = -1; nthreads = k; break; }
    }
    for (int k = 0; k < nthreads; ++k) {
        pthread_join(th[k], NULL);
        if (jobs[k].failed_alloc) rc = -1;
    }
    free(jobs);
    free(th);
    return rc;
}

int oracle_emd_batch(int d, const int64_t *offA, const double *xA, const double *wA, int64_t nA,
                     const int64_t *offB, const double *xB, const double *wB, int64_t nB,
                     const int64_t *pairs, int64_t npairs, int init_rule, int bland_after,
                     int nthreads, double *dist, int32_t *status, long long *pivots,
                     long long *bland) {
    job_t J;
    memset(&J, 0, sizeof(J));
    J.d = d; J.offA = offA; J.xA = xA; J.wA = wA; J.nA = nA;
    J.offB = offB; J.xB = xB; J.wB = wB; J.nB = nB;
    J.init = init_rule; J.bland_after = bland_after; J.mode = 0; J.pairs = pairs;
    J.npairs = npairs;
    J.dist = dist; J.status = status; J.pivots = pivots; J.bland = bland;
    J.max_t = max_support(offA, nA); J.max_s = max_support(offB, nB);
    for (int64_t k = 0; k < npairs; ++k)
        if (pairs[2 * k] < 0 || pairs[2 * k] >= nA || pairs[2 * k + 1] < 0 ||
            pairs[2 * k + 1] >= nB)
            return -2;
    if (J.max_t < 1) J.max_t = 1;
    if (J.max_s < 1) J.max_s = 1;
    return run_jobs(&J, npairs, nthreads);
}

int oracle_assign(int d, const int64_t *offX, const double *xX, const double *wX, int64_t nX,
                  const int64_t *offZ, const double *xZ, const double *wZ, int64_t nZ,
                  int init_rule, int nthreads, int32_t *labels, double *best, double *all,
                  int32_t *status, long long *pivots, long long *bland) {
    job_t J;
    memset(&J, 0, sizeof(J));
    J.d = d; J.offA = offX; J.xA = xX; J.wA = wX; J.nA = nX;
    J.offB = offZ; J.xB = xZ; J.wB = wZ; J.nB = nZ;
    J.init = init_rule; J.mode = 1;
    J.dist = all; J.status = status; J.pivots = pivots; J.bland = bland; J.labels = labels;
    J.best = best;
    J.max_t = max_support(offX, nX); J.max_s = max_support(offZ, nZ);
    if (J.max_t < 1) J.max_t = 1;
    if (J.max_s < 1) J.max_s = 1;
    return run_jobs(&J, nX, nthreads);
}

int oracle_pairwise(int d, const int64_t *offX, const double *xX, const double *wX, int64_t nX,
                    int init_rule, int nthreads, double *condensed, int32_t *status,
                    long long *pivots, long long *bland) {
    job_t J;
    memset(&J, 0, sizeof(J));
    J.d = d; J.offA = offX; J.xA = xX; J.wA = wX; J.nA = nX;
    J.offB = offX; J.xB = xX; J.wB = wX; J.nB = nX;
    J.init = init_rule; J.mode = 2;
    J.dist = condensed; J.status = status; J.pivots = pivots; J.bland = bland;
    J.max_t = max_support(offX, nX); J.max_s = J.max_t;
    if (J.max_t < 1) { J.max_t = 1; J.max_s = 1; }
    return run_jobs(&J, nX * (nX - 1) / 2, nthreads);
}
