// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "d2.h"

namespace d2 {

// Starting-basis rules as compiled into the kernels.
enum { kStartNWC = 0, kStartVogel = 1, kStartLCM = 2 };

// Options as the kernels see them (validated and defaulted on the host).
struct KOpts {
    int init;        // kStart* (D2_INIT_AUTO resolved on the host)
    int max_pivots;  // 0 = max(50 t s, 100)
    int want_sqrt;
    int cost_mode;
    int bland_after; // degenerate-pivot run that switches to Bland's rule (0 = 2 (t + s))
    double tol;      // relative optimality tolerance
};

// Device view of a ragged set.
struct KSet {
    const int64_t *off;
    const void *pts;
    const void *w;
    int64_t n;
    int d;
    int dtype;
};

struct LaunchCtx {
    hipStream_t stream;
    int cu_count;
};

// Persistent-kernel schedule per support class (chosen by the autotuner).
struct Schedule {
    int blocks_per_cu[4];   // persistent workgroups per CU, per support class
    int chunk[4];           // pairs taken per work-queue grab
    int tile[4];            // a positions per tile of the class's walk (default 512)
    int edge[2];            // support bin edges of classes 0 and 1 (<= 16, <= 32)
};

// Support class of a pair with these (declared) maximum supports.
int class_for(int maxsup_a, int maxsup_b);

// d2_assign: rows, optionally sorted by support into classes, each
// (row, centroid chunk) item handled by one workgroup; partial minima go to
// the workspace when the centroids are split into chunks.
struct AssignPlan {
    bool plain, binned, bf16;
    int single_class;
    int zmax;
    int64_t chunks, per_chunk;
    size_t part_bytes, sort_bytes, frag_bytes, ws_bytes;
};
AssignPlan plan_assign(const KSet &X, const KSet &Z, int xmax, int zmax, int cu_count, int schedule,
                       int cost_mode);
hipError_t launch_assign(const LaunchCtx &c, const AssignPlan &p, const KSet &X, const KSet &Z,
                         const KOpts &o, int32_t *labels, double *best, double *all,
                         int32_t *row_status, void *ws);

// Pairs with their optimal bases as sorted (A atom, B atom, flow) cells.
hipError_t launch_emd_basis(const LaunchCtx &c, int cls, const KSet &A, const KSet &B, const int64_t *pairs,
                            int64_t npairs, const KOpts &o, double *dist, const int64_t *basis_off,
                            int32_t *basis_ij, double *basis_w, int32_t *status);
hipError_t launch_emd_pairs(const LaunchCtx &c, int cls, const KSet &A, const KSet &B,
                            const int64_t *pairs, int64_t npairs, const KOpts &o, double *dist,
                            const int64_t *plan_off, double *plan, const int64_t *dual_off,
                            double *duals, int32_t *status, int32_t *pivots);

struct PairwisePlan {
    bool plain, binned;
    int plain_class;
    size_t ws_bytes;
};
PairwisePlan plan_pairwise(const KSet &X, int xmax, int schedule);
hipError_t launch_pairwise(const LaunchCtx &c, const PairwisePlan &p, const KSet &X, const KOpts &o,
                           double *condensed, int32_t *status, void *ws, const Schedule &sch,
                           int only_class = -1);

hipError_t launch_cost_tiles(const LaunchCtx &c, const KSet &A, const KSet &B,
                             const int64_t *pairs, int64_t npairs, int cost_mode, double *tiles,
                             const int64_t *tile_off);

// Workgroup simplex for pairs with more than 64 atoms on a side.
int wg_max_support();
void wg_plan(int64_t npairs, int tmax, int smax, int cu_count, int64_t *grid, int64_t *slab_elems);
hipError_t launch_emd_wg(const LaunchCtx &c, const KSet &A, const KSet &B, const int64_t *pairs, int64_t npairs,
                         const KOpts &o, int tmax, int smax, double *dist, const int64_t *plan_off, double *plan,
                         const int64_t *dual_off, double *duals, int32_t *status, int32_t *pivots, void *ws);
size_t wg_assign_bytes(int64_t n, int64_t K, int tmax, int smax, int cu_count);
hipError_t launch_assign_wg(const LaunchCtx &c, const KSet &X, const KSet &Z, const KOpts &o, int tmax, int smax,
                            int32_t *labels, double *best, double *all, int32_t *row_status, void *ws);
size_t wg_pairwise_bytes(int64_t n, int tmax, int cu_count);
hipError_t launch_pairwise_wg(const LaunchCtx &c, const KSet &X, const KOpts &o, int tmax, double *condensed,
                              int32_t *status, void *ws);

// Labelling under the multi-type distance of Eq. (9).
size_t multi_ws_bytes(int64_t n, int64_t K, size_t assign_bytes);
hipError_t launch_assign_multi(const LaunchCtx &c, int ntypes, const AssignPlan *plans, const KSet *X,
                               const KSet *Z, const KOpts &o, int32_t *labels, double *best, double *all,
                               int32_t *row_status, void *ws, size_t assign_bytes);

// The transport LP over caller-given FP64 cost matrices.
hipError_t launch_emd_cost(const LaunchCtx &c, int cls, int64_t nprob, const int64_t *roff, const double *rw,
                           const int64_t *coff, const double *cw, const double *cost, const int64_t *moff,
                           int max_rows, int max_cols, const KOpts &o, double *dist, const int64_t *plan_off,
                           double *plan, int32_t *status);

// Centroid update with fixed centroid weights (Alg. 2 Step 3*): workspace
// size and the enqueue of the whole pass.
size_t update_ws_bytes(int64_t n, int64_t K, int d, int xmax, int zmax);
void update_mean_shape(int d, int zmax, int *kb, int *P);
hipError_t launch_update(const LaunchCtx &c, int cls, const KSet &X, const KSet &Z, int xmax, int zmax,
                         const KOpts &o, const int32_t *labels, const double *obj_weights, double *z_new,
                         double *eps1, double *eps3, int32_t *counts, int32_t *obj_status, void *ws);

// Centroid update with free centroid weights (Alg. 1 Steps 1-3): the bytes
// of one cluster's slab, the whole workspace (grid returned), and the enqueue.
size_t update_free_slab_bytes(int max_members, int xmax, int zmax, int d);
size_t update_free_ws_bytes(int64_t n, int64_t K, int d, int xmax, int zmax, int max_members, int cu_count,
                            int64_t *grid_out);
hipError_t launch_update_free(const LaunchCtx &c, const KSet &X, const KSet &Z, int xmax, int zmax,
                              int max_members, const KOpts &o, const int32_t *labels, const double *obj_weights,
                              double *z_new, double *w_new, double *eps1, double *eps3, int32_t *counts,
                              int32_t *obj_status, int32_t *cluster_status, int32_t *cluster_pivots,
                              int32_t *basis_io, int64_t basis_stride, void *ws);

// Alg. 3 Step 3 for one level: kept centroids, their weights and atoms,
// inherited labels.
size_t merge_ws_bytes(int64_t n, int64_t K);
hipError_t launch_merge_level(const LaunchCtx &c, const KSet &Z, int64_t n, const int32_t *labels,
                              const double *omega, int64_t n0, int32_t *C, int64_t *kept, int64_t *new_off,
                              void *new_points, void *new_weights, double *new_omega, void *ws);

// Labelling within segments: object i against the centroids
// zoff[seg[i]] .. zoff[seg[i]+1] of Z only.
hipError_t launch_assign_seg(const LaunchCtx &c, int cls, const KSet &X, const KSet &Z, const KOpts &o,
                             const int32_t *seg, int64_t nseg, const int64_t *zoff, int32_t *labels,
                             double *best, int32_t *row_status);

}  // namespace d2
