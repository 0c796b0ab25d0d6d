/*
 * Plain FP64 CPU oracle for the squared Mallows distance (paper Sec. 1.1,
 * Eq. (1) with the centroid fixed) and the nearest-centroid label (Alg. 2,
 * Step 2).  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and
 * the CPU baseline of the benchmark; never by the product path.
 *
 * Ragged sets: offsets[n+1] (int64), points[offsets[n]][d] row-major FP64,
 * weights[offsets[n]] FP64 (any non-negative finite vector with positive sum;
 * it is divided by its sum).  Status per pair: 0 optimal, 1 bad weights,
 * 2 empty or oversize support, 3 pivot cap reached (value NaN), 4 a
 * non-finite given cost.  Every solve reports its pivot count and, in
 * `bland` (nullable), the number of those pivots taken under Bland's
 * anti-cycling rule.  `bland_after` is the run of degenerate pivots that
 * switches to Bland's rule (0 = the default 2(t+s)).
 */
#ifndef EMD_ORACLE_H
#define EMD_ORACLE_H
#include <stdint.h>

#define ORACLE_INIT_NWC 0
#define ORACLE_INIT_VOGEL 1

int oracle_emd_pair(int t, int s, int d, const double *x, const double *p, const double *y,
                    const double *q, int init_rule, int bland_after, double *d2_out,
                    double *plan_out, double *u_out, double *v_out, long long *pivots_out,
                    long long *bland_out);

/* The transport LP with a caller-given t x s cost (row-major, finite). */
int oracle_emd_cost(int t, int s, const double *cost, const double *p, const double *q,
                    int init_rule, int bland_after, double *d2_out, double *plan_out,
                    double *u_out, double *v_out, long long *pivots_out, long long *bland_out);

int oracle_emd_batch(int d, const int64_t *offA, const double *xA, const double *wA, int64_t nA,
                     const int64_t *offB, const double *xB, const double *wB, int64_t nB,
                     const int64_t *pairs, int64_t npairs, int init_rule, int bland_after,
                     int nthreads, double *dist, int32_t *status, long long *pivots,
                     long long *bland);

int oracle_assign(int d, const int64_t *offX, const double *xX, const double *wX, int64_t nX,
                  const int64_t *offZ, const double *xZ, const double *wZ, int64_t nZ,
                  int init_rule, int nthreads, int32_t *labels, double *best, double *all,
                  int32_t *status, long long *pivots, long long *bland);

int oracle_pairwise(int d, const int64_t *offX, const double *xX, const double *wX, int64_t nX,
                    int init_rule, int nthreads, double *condensed, int32_t *status,
                    long long *pivots, long long *bland);
#endif
