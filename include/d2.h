/*
 * libd2 -- batched exact squared Mallows distances on one MI355X (gfx950).
 *
 * The paper (Zhang, Wang & Li, "Parallel D2-Clustering: Large-Scale
 * Clustering of Discrete Distributions") works with discrete distributions,
 * "bags of weighted vectors" v = {(v^(a), p^(a)) : a = 1..t} (Sec. 1.1 and
 * Sec. 2.2), the squared Mallows distance between two of them -- the value of
 * the transportation linear program of Eq. (1) once the centroid is fixed --
 * and the labelling step C(i) = argmin_j D(v_i, z_j) (Alg. 2, Step 2), which
 * it notes parallelises per point (Sec. 1.2).  This library computes those
 * quantities exactly (FP64 optimum of the LP) for many pairs at once.
 *
 * For P = {(x_a, p_a)}_{a<t}, Q = {(y_b, q_b)}_{b<s} in R^d:
 *
 *     D^2(P,Q) = min_{w>=0} sum_ab w_ab |x_a - y_b|^2
 *                s.t. sum_b w_ab = p_a, sum_a w_ab = q_b,
 *
 * where p and q are the caller's weights divided by their FP64 sums.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every pointer inside a d2_set and every output pointer is DEVICE memory
 *    on the handle's device, owned by the caller.  The library never frees
 *    caller memory and keeps no pointer past the completion of the stream
 *    work a call enqueues.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls enqueue kernels on it and return without synchronising.
 *  - A handle is not thread-safe; use one handle per host thread.
 *  - Host-detectable problems are returned synchronously as a d2_status and
 *    nothing is enqueued.  Problems found per pair on the device are written
 *    to the per-pair (or per-row) status arrays (D2_PAIR_* codes); the
 *    distance of a failed pair is NaN.
 *  - The primary output is D^2 (the LP objective); opts->want_sqrt = 1
 *    returns D = sqrt(D^2) instead.  Labels are 0-based; ties go to the lowest
 *    centroid index; a row with any failed pair gets label -1.
 *  - Supports of more than D2_MAX_SUPPORT atoms are not handled
 *    (D2_EUNSUPPORTED when declared, D2_PAIR_TOO_LARGE when found on device),
 *    except by d2_emd_batch, d2_assign and d2_pairwise, which take up to
 *    D2_MAX_SUPPORT_LARGE on a workgroup simplex (FP64 cost only).
 */
#ifndef D2_H
#define D2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define D2_MAX_SUPPORT 64
/* d2_emd_batch, d2_assign and d2_pairwise also take supports up to this,
 * through a workgroup simplex (slower per pair; see d2_emd_batch). */
#define D2_MAX_SUPPORT_LARGE 1024

typedef enum {
    D2_OK = 0,
    D2_EINVAL = 1,       /* null pointer, negative count, bad dtype/mode/size   */
    D2_EWORKSPACE = 2,   /* ws_bytes below d2_workspace_bytes() for the call     */
    D2_EUNSUPPORTED = 3, /* declared max_support above D2_MAX_SUPPORT, etc.      */
    D2_EHIP = 4,         /* a HIP runtime call or launch failed                  */
    D2_ENOMEM = 5,       /* host allocation failed (handle creation only)        */
    D2_ESCRATCH = 6      /* d2_assign_noalloc: the call needs more workspace     *
                          * than D2_NOALLOC_SCRATCH_BYTES                        */
} d2_status;

/* Bytes of device scratch each GPU holds for d2_assign_noalloc (32 MiB),
 * from the first d2_create on it until the process ends. */
#define D2_NOALLOC_SCRATCH_BYTES (32u << 20)

/* element type of d2_set.points and d2_set.weights (always both the same) */
enum { D2_F64 = 0, D2_F32 = 1 };

/* ground-cost arithmetic */
enum {
    D2_COST_F64_DIRECT = 0, /* C_ab = sum_k (x_ak - y_bk)^2 in FP64, k ascending   */
    D2_COST_BF16_MFMA = 1   /* C_ab = max(0, |x|^2 + |y|^2 - 2 x.y): x.y by BF16   *
                             * MFMA with FP32 accumulation, norms in FP32 from the *
                             * same BF16-rounded values, result widened to FP64.  *
                             * Approximate: not held to the FP64 tolerance.  Each  *
                             * coordinate is rounded FP64->FP32->BF16 (nearest,    *
                             * ties to even).  Supports up to 32 only (else        *
                             * D2_EUNSUPPORTED); accepted by d2_cost_tiles and     *
                             * d2_assign (d2_emd_batch and d2_pairwise: EUNSUPP.). */
};

/* starting basis of the transportation simplex (every rule reaches the same
 * optimum; they differ in how many pivots remain):
 *   D2_INIT_NWC   north-west corner;
 *   D2_INIT_VOGEL Vogel's approximation (largest gap between a line's two
 *                 cheapest open cells first);
 *   D2_INIT_LCM   least cost (cheapest open cell first);
 *   D2_INIT_AUTO  the library's default (D2_INIT_LCM). */
enum { D2_INIT_AUTO = 0, D2_INIT_NWC = 1, D2_INIT_VOGEL = 2, D2_INIT_LCM = 3 };

/* per-pair status codes written by the device */
enum {
    D2_PAIR_OK = 0,
    D2_PAIR_BAD_WEIGHTS = 1, /* a weight is NaN/inf/negative, or the sum is <= 0 */
    D2_PAIR_TOO_LARGE = 2,   /* empty support, or more atoms than the call takes  */
    D2_PAIR_PIVOT_CAP = 3,   /* pivot cap reached; the value is NaN               */
    D2_PAIR_BAD_POINTS = 4,  /* a ground cost is not finite (NaN/inf coordinates) */
    D2_PAIR_UNLABELLED = 5,  /* d2_centroid_update: label outside [0, K); the     *
                              * object is left out                                 */
    D2_PAIR_INTERNAL = 6     /* a solver invariant failed (a starting basis that   *
                              * did not close within its round bound, a basis tree *
                              * that did not resolve); the value is NaN.  Never    *
                              * expected; reported apart from the pivot cap so a   *
                              * defect cannot pass for an ordinary cap.            */
};

/* A ragged set of n discrete distributions in R^d (device memory). */
typedef struct {
    int64_t n;               /* number of distributions (>= 0)                    */
    int32_t d;               /* dimension (>= 1)                                  */
    int32_t dtype;           /* D2_F64 or D2_F32                                  */
    const int64_t *offsets;  /* [n+1]; atoms of object i: offsets[i]..offsets[i+1] */
    const void *points;      /* [offsets[n]][d] row-major, dtype                  */
    const void *weights;     /* [offsets[n]], dtype, any non-negative scale       */
    int32_t max_support;     /* host-known upper bound on offsets[i+1]-offsets[i] */
    int32_t reserved;        /* set to 0                                          */
} d2_set;

/* work schedule (results are identical under every schedule) */
enum {
    D2_SCHED_AUTO = 0,  /* pairs grouped by support class, each class in the       *
                         * narrowest group shape; persistent queue for pairwise    */
    D2_SCHED_PLAIN = 1  /* one wavefront per pair, pairs in input order            */
};

typedef struct {
    int32_t cost_mode;  /* D2_COST_*                                               */
    int32_t init;       /* D2_INIT_*                                               */
    int32_t max_pivots; /* 0 = default cap max(50 t s, 100) per pair               */
    int32_t want_sqrt;  /* 0 -> D^2, 1 -> D                                        */
    double opt_tol;     /* 0 = default 1e-14; the simplex stops when every reduced *
                         * cost is >= -opt_tol * max_ab C_ab                       */
    int32_t schedule;   /* D2_SCHED_*                                              */
    int32_t flags;      /* D2_FLAG_* bits, 0 by default                            */
    int32_t bland_after; /* run of consecutive degenerate pivots after which the   *
                          * entering cell follows Bland's rule (lowest cell with a *
                          * negative reduced cost) until a pivot moves flow again; *
                          * 0 = the default 2 (t + s).  The paper leaves cycling   *
                          * open (its LP solver is unnamed); every value reaches   *
                          * the same optimum value.                                */
} d2_opts;

/* D2_FLAG_EAGER: enqueue the kernels directly instead of recording the call
 * once as a hipGraph and replaying it for later calls with the same
 * arguments (the default for d2_assign and d2_pairwise). */
#define D2_FLAG_EAGER 1

typedef struct d2_handle d2_handle;

/* Create a handle bound to HIP device `device`.  It holds host memory, one
 * private stream used only to record graphs, and the graph and schedule
 * caches; it never allocates device memory. */
d2_status d2_create(d2_handle **h, int device);
d2_status d2_destroy(d2_handle *h);
const char *d2_status_string(int code);
/* D2_MAX_SUPPORT and the library version, for binding self-checks. */
int d2_max_support(void);
const char *d2_version(void);

/* Bytes of device workspace the call with these arguments needs (may be 0).
 * `which` is 0 = d2_cost_tiles, 1 = d2_emd_batch, 2 = d2_assign,
 * 3 = d2_pairwise, 4 = d2_centroid_update (A = X, B = Z), 5 =
 * d2_assign_multi (A, B = the arrays of per-type sets, npairs = the number of
 * types), 6 = d2_centroid_update_free (A = X, B = Z, npairs = max_members),
 * 7 = d2_merge_level (A = Z, B unused, npairs = n);
 * `npairs` is the pair count for 0 and 1, ignored for 2-4; B may be NULL for
 * d2_pairwise. */
size_t d2_workspace_bytes(d2_handle *h, int which, const d2_set *A, const d2_set *B,
                          int64_t npairs, const d2_opts *opts);

/* Ground-cost tiles (the t_i x s_j matrices |x_a - y_b|^2 inside Eq. (1)).
 * pairs[npairs][2] (device int64): (i in A, j in B).  Tile k is written
 * row-major (a over A's atoms, b over B's atoms) at tiles + tile_offsets[k];
 * tile_offsets[npairs+1] (device int64) is supplied by the caller and must
 * leave t_i*s_j doubles for pair k.  For testing and the precision study. */
d2_status d2_cost_tiles(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                        int64_t npairs, int32_t cost_mode, double *tiles,
                        const int64_t *tile_offsets, void *ws, size_t ws_bytes, void *stream);

/* D^2 for an explicit pair list: the value of the transport LP of Eq. (1)
 * with the centroid fixed (Sec. 1.1: for a fixed z the LP is the squared
 * Mallows distance), dist[k] = D^2(A_i, B_j) for pairs[k] = (i,j) (device
 * int64 [npairs][2]; an index outside its set gives D2_PAIR_TOO_LARGE).
 * When the declared max_support of A or B exceeds D2_MAX_SUPPORT (up to
 * D2_MAX_SUPPORT_LARGE, else D2_EUNSUPPORTED), every pair runs on a
 * workgroup simplex instead of a lane group; it then needs a workspace of
 * d2_workspace_bytes(h, 1, A, B, npairs, opts) bytes (cost matrices of
 * max_support(A) x max_support(B) doubles per workgroup, at most 1 GiB in
 * all).  The workgroup path starts from the north-west corner under
 * D2_INIT_NWC and from the least-cost start under every other choice
 * (D2_INIT_VOGEL included), and prices in blocks of cells; results satisfy
 * the same tolerance.
 * plan_offsets, plan (nullable, both or neither): the optimal transport plan
 * of pair k is written densely row-major (t_i x s_j doubles) at
 * plan + plan_offsets[k].  duals (nullable): u[t_i] then v[s_j] at
 * duals + dual_offsets[k] (dual_offsets[npairs+1], nullable with duals),
 * satisfying u_a + v_b = C_ab on the plan's support and u_a + v_b <= C_ab +
 * tol elsewhere.  pair_status[npairs] may be NULL.
 * pivots (nullable, device int32 [npairs][2]): the number of simplex pivots
 * of pair k, then how many of them were taken under Bland's rule (see
 * d2_opts.bland_after); 0, 0 for a pair that failed before its first pivot. */
d2_status d2_emd_batch(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                       int64_t npairs, const d2_opts *opts, double *dist,
                       const int64_t *plan_offsets, double *plan, const int64_t *dual_offsets,
                       double *duals, int32_t *pair_status, int32_t *pivots, void *ws,
                       size_t ws_bytes, void *stream);

/* D^2 for an explicit pair list, with each pair's optimal basis: for fixed
 * centroid atoms the LP of Eq. (1) is a transportation problem (Sec. 1.1),
 * whose bases are spanning trees of the bipartite graph of the two atom
 * sets, t_i + s_j - 1 cells.  pairs, dist, opts and pair_status (nullable)
 * as for d2_emd_batch.  Pair k's cells go to basis_ij + 2 basis_offsets[k]
 * (int32 (A atom, B atom) per cell, atoms numbered within their objects)
 * and basis_w + basis_offsets[k] (FP64 flow, in the units of the
 * normalised weights), sorted by A atom, then B atom, zero-flow
 * (degenerate) basic cells included; basis_offsets[npairs] (device int64)
 * is supplied by the caller and must leave t_i + s_j - 1 cells for pair k.
 * Nothing is written for a pair that failed.  Supports up to
 * D2_MAX_SUPPORT (else D2_EUNSUPPORTED); FP64 direct cost only; no
 * workspace. */
d2_status d2_emd_batch_basis(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                             int64_t npairs, const d2_opts *opts, double *dist, const int64_t *basis_offsets,
                             int32_t *basis_ij, double *basis_w, int32_t *pair_status, void *stream);

/* The transport LP of Eq. (1) over caller-given ground costs, for the MM
 * distance of Eq. (10) (whose ground cost is the matrix of squared Mallows
 * distances between two centroid sets) or any other cost.  Problem k:
 *   rows     t_k = row_offsets[k+1] - row_offsets[k] weights at
 *            row_weights + row_offsets[k] (device FP64);
 *   columns  s_k likewise from col_offsets / col_weights;
 *   cost     t_k x s_k FP64, row-major, at costs + cost_offsets[k] (device;
 *            problems may share a matrix); any finite values, including
 *            negative ones.
 * Weights are normalised by their sums as everywhere (status 1 when a
 * vector is invalid); a non-finite cost gives D2_PAIR_BAD_POINTS.
 * max_rows, max_cols: host-known bounds on t_k and s_k, at most
 * D2_MAX_SUPPORT (else D2_EUNSUPPORTED); a problem beyond them gets
 * D2_PAIR_TOO_LARGE.  dist[k] is the LP value (opts->want_sqrt and
 * opts->cost_mode do not apply; D2_COST_BF16_MFMA gives D2_EUNSUPPORTED).
 * The simplex stops when every reduced cost is >= -opt_tol * max |C|.
 * plan_offsets, plan (nullable, both or neither): the optimal plan, dense
 * row-major t_k x s_k in the caller's frame.  status[nprob] may be NULL.
 * No workspace (ws may be NULL). */
d2_status d2_emd_cost_batch(d2_handle *h, int64_t nprob, const int64_t *row_offsets,
                            const double *row_weights, const int64_t *col_offsets,
                            const double *col_weights, const double *costs,
                            const int64_t *cost_offsets, int32_t max_rows, int32_t max_cols,
                            const d2_opts *opts, double *dist, const int64_t *plan_offsets,
                            double *plan, int32_t *status, void *ws, size_t ws_bytes,
                            void *stream);

/* Nearest-centroid labelling (Alg. 2, Step 2) over the full cross product:
 * for every object i of X, D^2 to every centroid j of Z, then
 * labels[i] = argmin_j (ties: lowest j), best[i] = the minimum.  all[n][K]
 * (nullable) receives every D^2; row_status[n] (nullable) the worst pair
 * status of the row.  With D2_COST_BF16_MFMA each wavefront computes the
 * cost tiles of the two pairs it solves with MFMA and keeps them in
 * registers: no tile is written to memory and none enters the workspace.
 * When a
 * declared max_support exceeds D2_MAX_SUPPORT (up to D2_MAX_SUPPORT_LARGE),
 * every pair runs on the workgroup simplex of d2_emd_batch and the
 * workspace also holds the n x K distance matrix and its statuses; such a
 * call is enqueued directly (no graph).  FP64 cost only. */
d2_status d2_assign(d2_handle *h, const d2_set *X, const d2_set *Z, const d2_opts *opts,
                    int32_t *labels, double *best, double *all, int32_t *row_status, void *ws,
                    size_t ws_bytes, void *stream);

/* d2_assign without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as d2_assign with opts->flags treated as
 * D2_FLAG_EAGER (always enqueued directly, never recorded as a graph).  The
 * workspace d2_assign would take (d2_workspace_bytes(h, 2, X, Z, 0, opts))
 * lives in a fixed device array of D2_NOALLOC_SCRATCH_BYTES per GPU instead;
 * a call needing more returns D2_ESCRATCH and enqueues nothing (C2-like
 * labelling of 100,000 objects needs under 1 MiB; supports above
 * D2_MAX_SUPPORT are beyond it).  The call performs no
 * hipMalloc/hipFree and no allocating library call.  Every call on one GPU
 * shares that GPU's array: calls whose stream work overlaps on one GPU
 * race (serialise them, e.g. on one stream).  Kernels clear what must start
 * at zero; nothing carries over between calls. */
d2_status d2_assign_noalloc(d2_handle *h, const d2_set *X, const d2_set *Z, const d2_opts *opts,
                            int32_t *labels, double *best, double *all, int32_t *row_status,
                            void *stream);

/* Centroid update of constrained D2-clustering (Alg. 2 Step 3*: the update
 * of Alg. 1 with every centroid's weights held fixed), one pass over all
 * clusters.  With the weights fixed, the LP of Alg. 1 Step 1 separates into
 * one transport problem per member (Sec. 2.2), so the pass is:
 *   Step 1  for each object i with 0 <= labels[i] < K: the optimal plan
 *           w^(i) between X_i and Z_{labels[i]} (Eq. (1), centroid fixed);
 *   Step 2  every atom r of centroid j moves to the mean of its members'
 *           atoms weighted by their flows to r (Eq. (2));
 *   Step 3  the objective of Eq. (1) with the moved atoms and the Step 1
 *           plans.
 * The centroid weights are not changed: uniform 1/s_j is the paper's case;
 * any fixed non-negative weights are accepted (normalised by their sum).
 *   labels[n]      device int32, e.g. from d2_assign.  Objects whose label is
 *                  outside [0, K) are left out (status D2_PAIR_UNLABELLED).
 *   obj_weights[n] device FP64, nullable (all 1): the object weights of
 *                  weighted D2-clustering (Eq. (3)); each member's flows
 *                  count with its weight in both sums of Eq. (4), and its
 *                  D^2 terms in both objectives.  A negative or non-finite
 *                  weight gives status D2_PAIR_BAD_WEIGHTS (left out).
 *   z_new          device FP64 [Z.offsets[K]][d]: the moved atoms, in the
 *                  layout of Z.points, which it must not overlap.  An atom
 *                  that receives no flow (empty cluster, zero weight) keeps
 *                  its coordinates.
 *   eps_step1[K]   device FP64, nullable: sum of the members' D^2 to the old
 *                  atoms, each times its weight (the Step 1 objective).
 *   eps_step3[K]   device FP64, nullable: the Step 3 objective.
 *   counts[K]      device int32, nullable: members that entered Step 2.
 *   obj_status[n]  device int32, nullable: D2_PAIR_* of each object; an
 *                  object whose transport problem fails is left out of
 *                  Steps 2 and 3.  Supports above the declared max_support of
 *                  X or Z give D2_PAIR_TOO_LARGE.
 * Workspace: d2_workspace_bytes(h, 4, X, Z, 0, opts) bytes (required).
 * Sums run in a fixed order, so repeated calls give identical bits.  FP64
 * direct cost only (D2_COST_BF16_MFMA: D2_EUNSUPPORTED); opts->want_sqrt is
 * ignored.  Always enqueued directly (no graph is recorded). */
d2_status d2_centroid_update(d2_handle *h, const d2_set *X, const d2_set *Z, const int32_t *labels,
                             const double *obj_weights, const d2_opts *opts, double *z_new,
                             double *eps_step1, double *eps_step3, int32_t *counts,
                             int32_t *obj_status, void *ws, size_t ws_bytes, void *stream);

/* One pass of the centroid update of Alg. 1 with the centroid weights free
 * (Sec. 1.1, Steps 1-3), for every cluster j = 0..K-1 at once.
 *   Step 1  with cluster j's atoms fixed, the linear program of Eq. (1)
 *           (weighted as in Eq. (3)) over the centroid weights p_z and every
 *           member's transport plan: minimise sum_i omega_i sum w |z - v|^2
 *           subject to each member's plan having the member's weights as row
 *           sums and p_z as column sums, sum p_z = 1.  The members share p_z,
 *           so the cluster is one program, solved exactly by a revised
 *           simplex (one workgroup per cluster);
 *   Step 2  every atom moves to the omega-and-flow-weighted mean of the
 *           member atoms matched to it (Eq. (4));
 *   Step 3  the objective with the moved atoms and the same plans.
 * Unlike d2_centroid_update (Alg. 2, weights fixed), this changes the weights.
 *   labels[n], obj_weights[n]  as for d2_centroid_update; a member of weight
 *                  0 takes no part (it costs and moves nothing).
 *   max_members    host bound on the members of one cluster that enter the
 *                  program (>= 1).  A cluster with more labelled members
 *                  is left unchanged with status D2_PAIR_TOO_LARGE for it and
 *                  its members.  The workspace grows with
 *                  (max_members (max_support(X) + max_support(Z) - 1) + 1)^2.
 *   z_new          device FP64 [Z.offsets[K]][d], not overlapping Z.points:
 *                  the moved atoms; an atom that receives no mass keeps its
 *                  coordinates (its new weight is 0).
 *   w_new          device FP64 [Z.offsets[K]], not overlapping Z.weights:
 *                  the new weights p_z (summing to 1 per solved cluster).  A
 *                  cluster without members, or whose program was not solved,
 *                  keeps its atoms and weights in z_new, w_new.
 *   eps_step1[K], eps_step3[K]  device FP64, nullable: the Step 1 optimum and
 *                  the Step 3 objective; 0 for a cluster without members, NaN
 *                  for one whose program was not solved.
 *   counts[K]      device int32, nullable: members that entered the program.
 *   obj_status[n]  device int32, nullable: D2_PAIR_OK, D2_PAIR_BAD_WEIGHTS
 *                  (the object's or its omega's weights invalid: left out),
 *                  D2_PAIR_UNLABELLED, or its cluster's status when that is
 *                  not D2_PAIR_OK.
 *   cluster_status[K]  device int32, nullable: D2_PAIR_OK, D2_PAIR_TOO_LARGE,
 *                  D2_PAIR_PIVOT_CAP (opts->max_pivots, 0 = max(50 m, 100)
 *                  pivots for a program of m rows) or D2_PAIR_INTERNAL (the
 *                  basis matrix lost rank numerically).
 *   cluster_pivots[K]  device int32, nullable: simplex pivots of each
 *                  cluster's program (0 where none was solved).
 *   basis_io       device int32 [K][basis_stride], nullable: starting bases
 *                  kept between calls.  Row j holds m, the row count of a
 *                  basis of cluster j's program, then its m basic variables
 *                  (w(k, a, r) numbered s (T_k + a) + r with members k in
 *                  increasing object index and T_k their first atom, then
 *                  p_z(r) as s sum(t) + r), or -1.  On entry a row whose m
 *                  equals this call's, whose variables are distinct and in
 *                  range, whose basis matrix has full rank and whose
 *                  solution is feasible starts that cluster's simplex (a
 *                  later pass over the same members: only the costs have
 *                  changed); any other row is ignored.  On return every
 *                  solved cluster's row holds its optimal basis (when
 *                  m + 1 <= basis_stride), the others -1.  Fill with -1
 *                  before the first call.  A warm start only changes the
 *                  pivot path: with several optimal solutions it may end at
 *                  another one than a cold start.
 * Workspace: d2_workspace_bytes(h, 6, X, Z, max_members, opts) bytes
 * (required).  opts->bland_after applies to degenerate pivots as in the
 * transport solver (0 = 2 m); opts->opt_tol and want_sqrt are ignored: a
 * reduced cost counts as negative below -1e-13 max C.  Sums run in a fixed
 * order, so repeated calls give identical bits.  FP64 direct cost only.
 * D2_EUNSUPPORTED when one cluster's slab would exceed 8 GiB. */
d2_status d2_centroid_update_free(d2_handle *h, const d2_set *X, const d2_set *Z, const int32_t *labels,
                                  const double *obj_weights, int32_t max_members, const d2_opts *opts,
                                  double *z_new, double *w_new, double *eps_step1, double *eps_step3,
                                  int32_t *counts, int32_t *obj_status, int32_t *cluster_status,
                                  int32_t *cluster_pivots, int32_t *basis_io, int64_t basis_stride, void *ws,
                                  size_t ws_bytes, void *stream);

/* One level's merge (Alg. 3 Step 3, Sec. 2.4).  Z holds the level's
 * centroids, the segments' centroid ranges concatenated in segment order, so
 * that labels already carry the offset of Eq. (5).  A centroid with at least
 * one member is kept; the kept ones are renumbered 0 .. kept-1 in index order
 * and become the next level's objects:
 *   labels[n]       device int32, the centroid of each level object; a label
 *                   outside [0, Z->n) makes the object nobody's member;
 *   omega[n]        device FP64 object weights, or NULL for all 1;
 *   C[n0]           device int32, in/out: on entry the level object of each
 *                   original object, on exit its inherited label (Eq. (6)),
 *                   the new index of that object's centroid, or -1 when the
 *                   entry is outside [0, n) or that object has no centroid;
 *   kept            device int64 (one value), the number of kept centroids;
 *   new_offsets     device int64 [Z->n + 1]: the first kept+1 entries are the
 *                   atom offsets of the kept centroids in their new order;
 *   new_points,     device, Z's dtype, room for Z's atoms (Z->offsets[Z->n]
 *   new_weights     rows of d values, resp. that many weights): the kept
 *                   centroids' atoms and atom weights, copied unchanged;
 *   new_omega       device FP64 [Z->n]: the first kept entries are the kept
 *                   centroids' weights, each the sum of its members' omega
 *                   (Eq. (3)), added in increasing member index.
 * No output may overlap an input.  Workspace: d2_workspace_bytes(h, 7, Z,
 * NULL, n, NULL) bytes.  Members are grouped by a counting sort with no
 * atomics, so repeated calls give identical bits. */
d2_status d2_merge_level(d2_handle *h, const d2_set *Z, int64_t n, const int32_t *labels, const double *omega,
                         int64_t n0, int32_t *C, int64_t *kept, int64_t *new_offsets, void *new_points,
                         void *new_weights, double *new_omega, void *ws, size_t ws_bytes, void *stream);

/* Nearest-centroid labelling within segments (Alg. 3 Step 2, where each
 * segment of the data is clustered on its own): object i is compared only
 * with the centroids zseg_offsets[seg[i]] .. zseg_offsets[seg[i]+1] of Z.
 *   seg[n]             device int32, the segment of each object;
 *   zseg_offsets[nseg+1]  device int64, each segment's centroid range.
 * labels[i] is the global index in Z of the nearest of them (ties: lowest),
 * best[i] its D^2; an object whose segment is outside [0, nseg) or has no
 * centroids gets label -1 and status D2_PAIR_UNLABELLED; any failed pair
 * gives label -1 and the worst status.  row_status[n] may be NULL.  No
 * workspace.  FP64 direct cost only. */
d2_status d2_assign_segmented(d2_handle *h, const d2_set *X, const d2_set *Z, const int32_t *seg,
                              int64_t nseg, const int64_t *zseg_offsets, const d2_opts *opts,
                              int32_t *labels, double *best, int32_t *row_status, void *stream);

/* Nearest-centroid labelling under the combined distance of Eq. (9), for
 * objects described by several distributions (one per feature type, such as
 * an image's colour bag and texture bag):
 *     D^2(I_i, C_j) = sum over types m of D^2(X[m]_i, Z[m]_j).
 * X[0..ntypes), Z[0..ntypes): host arrays of sets, type m of every object and
 * of every centroid; all X[m] share n and all Z[m] share K (dimensions and
 * supports may differ between types).  1 <= ntypes <= 16.  labels, best,
 * all (the summed matrix, nullable), row_status (the worst status over the
 * types, nullable) as for d2_assign; a row with any failed pair gets
 * label -1.  Workspace: d2_workspace_bytes(h, 5, X, Z, ntypes, opts)
 * (required; it holds two n x K matrices). */
d2_status d2_assign_multi(d2_handle *h, int32_t ntypes, const d2_set *X, const d2_set *Z,
                          const d2_opts *opts, int32_t *labels, double *best, double *all,
                          int32_t *row_status, void *ws, size_t ws_bytes, void *stream);

/* All unordered pairs i<j of one set: the pairwise D^2 matrix of one data
 * segment, the distances the segment-local clustering of Alg. 3 Step 2 works
 * on (each segment holds at most tau objects and is clustered on its own,
 * Sec. 2.1 and Sec. 2.4); D^2 is the LP value of Eq. (1) with one object
 * as the fixed side (Sec. 1.1).
 * condensed[k] for k = i*n - i*(i+1)/2 + (j-i-1), the order of
 * scipy.spatial.distance.squareform.  pair_status (nullable) has the same
 * shape.  Supports beyond D2_MAX_SUPPORT (up to D2_MAX_SUPPORT_LARGE) run
 * every pair on the workgroup simplex of d2_emd_batch, with its workspace
 * of cost slabs, enqueued directly (no graph).  FP64 cost only. */
d2_status d2_pairwise(d2_handle *h, const d2_set *X, const d2_opts *opts, double *condensed,
                      int32_t *pair_status, void *ws, size_t ws_bytes, void *stream);

/* Schedule autotuner for d2_pairwise (synchronous: waits for the stream).
 * Tunes each support class on its own launch, one setting at a time from
 * the defaults: persistent workgroups per CU (2, 4, 8), pairs per
 * work-queue grab (1, 4, 16) and tile width of the class's walk (128, 512,
 * 2048 objects); then the support bin edges of classes 0 and 1 ({16, 12, 8}
 * x {32, 24}) on whole calls.  Keeps the fastest schedule for this workload
 * shape (n, d, dtype, max_support, start rule) in the handle and writes the
 * time of a whole call with it to *best_ms.  Later d2_pairwise calls of the
 * same shape use it.  Outputs are written as by d2_pairwise and do not
 * depend on the schedule. */
d2_status d2_tune_pairwise(d2_handle *h, const d2_set *X, const d2_opts *opts, double *condensed,
                           int32_t *pair_status, void *ws, size_t ws_bytes, void *stream,
                           double *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* D2_H */
