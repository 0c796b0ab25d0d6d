// Nearest-centroid labelling within segments (Alg. 3 Step 2): the data are
// cut into segments, each clustered on its own, so object i is compared only
// with the centroids of its own segment, a contiguous range of Z.  One lane
// group per object walks that range (a handful of centroids: tau / e of
// them, or two during the binary splits of the segmentation) and keeps the
// running minimum, ties to the lowest index.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"
#include "d2_shapes.h"
#include "d2_solver.h"

namespace d2 {

namespace {

constexpr int kNoCentroids = 5;   // D2_PAIR_UNLABELLED

template <int CLS, typename TIn, int START>
__global__ __launch_bounds__(ShapeCfg<CLS>::threads, ShapeCfg<CLS>::occ) void k_assign_seg(
    KSet X, KSet Z, KOpts o, const int32_t *seg, int64_t nseg, const int64_t *zoff, int32_t *labels,
    double *best, int32_t *row_status) {
    constexpr int G = ShapeCfg<CLS>::G, GS = ShapeCfg<CLS>::GS, NG = ShapeCfg<CLS>::groups;
    constexpr bool LT = ShapeCfg<CLS>::LT;
    using TileT = TileOf<CLS, START>;
    __shared__ GroupMem<G, GS> mem[NG];
    __shared__ TileT tiles[NG];
    const int tid = threadIdx.x;
    const int g = tid / G, l = tid % G, gbase = (tid & 63) & ~(G - 1);
    const int64_t stride = (int64_t)gridDim.x * NG;
    for (int64_t i = (int64_t)blockIdx.x * NG + g; i < X.n; i += stride) {
        const int64_t sg = seg[i];
        int64_t j0 = 0, j1 = 0;
        if (sg >= 0 && sg < nseg) {
            j0 = zoff[sg];
            j1 = zoff[sg + 1];
            if (j0 < 0) j0 = 0;
            if (j1 > Z.n) j1 = Z.n;
        }
        double bv = INFINITY;
        int bj = -1, worst = j1 > j0 ? kOk : kNoCentroids;
        for (int64_t j = j0; j < j1; ++j) {   // uniform over the group
            NodeState<G, GS, LT> N;
            PairView pv = orient(X, i, Z, j, (int)sizeof(TIn));
            const SolveOut r = solve_pair<G, GS, LT, TIn, START>(mem[g], tiles[g], N, pv, X.d, o, l, gbase);
            if (r.status != kOk) {
                worst = r.status > worst ? r.status : worst;
            } else if (r.d2 < bv) {
                bv = r.d2;
                bj = (int)j;
            }
        }
        if (l == 0) {
            labels[i] = worst == kOk ? bj : -1;
            best[i] = worst == kOk ? bv : __builtin_nan("");
            if (row_status) row_status[i] = worst;
        }
    }
}

struct SegRun {
    const LaunchCtx &c;
    const KSet &X, &Z;
    const KOpts &o;
    const int32_t *seg; int64_t nseg; const int64_t *zoff;
    int32_t *labels; double *best; int32_t *row_status;
    template <int C, typename TIn, int V>
    hipError_t run() {
        const int NG = ShapeCfg<C>::groups;
        int64_t grid = (X.n + NG - 1) / NG;
        if (grid > (1LL << 30)) grid = 1LL << 30;
        hipLaunchKernelGGL((k_assign_seg<C, TIn, V>), dim3((unsigned)grid), dim3(ShapeCfg<C>::threads), 0,
                           c.stream, X, Z, o, seg, nseg, zoff, labels, best, row_status);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_assign_seg(const LaunchCtx &c, int cls, const KSet &X, const KSet &Z, const KOpts &o,
                             const int32_t *seg, int64_t nseg, const int64_t *zoff, int32_t *labels,
                             double *best, int32_t *row_status) {
    if (X.n == 0) return hipSuccess;
    SegRun r{c, X, Z, o, seg, nseg, zoff, labels, best, row_status};
    return dispatch_class(cls, X.dtype == D2_F32, o.init, r);
}

}  // namespace d2
