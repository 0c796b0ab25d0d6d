// Labelling under the combined distance of Eq. (9): an object described by
// several distributions (one per feature type, e.g. a colour bag and a
// texture bag of an image) is compared with a centroid made of the same
// types by  D^2(I_i, C_j) = sum over types m of D^2(X^m_i, Z^m_j).
//
// Each type runs the labelling path with its full distance matrix kept
// (type 0 straight into the accumulator, later types into a second matrix
// that one pass adds in), then one wave per object takes the argmin of the
// summed row (ties to the lowest centroid).  The row status is the worst
// over all types.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "d2_internal.h"

namespace d2 {

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

__global__ void k_multi_add(double *acc, const double *add, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        acc[i] += add[i];
}

__global__ void k_multi_status(int32_t *worst, const int32_t *st, int64_t n, int first) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        worst[i] = first ? st[i] : (st[i] > worst[i] ? st[i] : worst[i]);
}

// One wave per object: minimum of the summed row, lowest index on ties.
__global__ __launch_bounds__(256) void k_multi_argmin(const double *acc, int64_t n, int64_t K,
                                                      const int32_t *worst, int32_t *labels, double *best,
                                                      int32_t *row_status) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += waves) {
        double v = INFINITY;
        int64_t jj = INT64_MAX;
        for (int64_t j = lane; j < K; j += 64) {
            const double x = acc[i * K + j];
            if (x < v) { v = x; jj = j; }   // j ascending per lane: first minimum kept
        }
        for (int sh = 32; sh >= 1; sh >>= 1) {
            const double ov = __shfl_xor(v, sh, 64);
            const int64_t oj = __shfl_xor(jj, sh, 64);
            if (ov < v || (ov == v && oj < jj)) { v = ov; jj = oj; }
        }
        if (lane == 0) {
            const int st = worst[i];
            labels[i] = st == 0 ? (int32_t)jj : -1;
            best[i] = st == 0 ? v : __builtin_nan("");
            if (row_status) row_status[i] = st;
        }
    }
}

struct MultiWS {
    double *acc, *tmp, *sbest;
    int32_t *slab, *sst, *worst;
    void *assign_ws;
};

size_t multi_layout(int64_t n, int64_t K, size_t assign_bytes, void *base, MultiWS *w) {
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t b) { char *q = p ? p + off : nullptr; off += al256(b); return q; };
    const size_t nn = (size_t)(n > 0 ? n : 1), nk = nn * (size_t)(K > 0 ? K : 1);
    MultiWS s;
    s.acc = (double *)take(nk * 8);
    s.tmp = (double *)take(nk * 8);
    s.sbest = (double *)take(nn * 8);
    s.slab = (int32_t *)take(nn * 4);
    s.sst = (int32_t *)take(nn * 4);
    s.worst = (int32_t *)take(nn * 4);
    s.assign_ws = take(assign_bytes > 0 ? assign_bytes : 1);
    if (w) *w = s;
    return off;
}

}  // namespace

size_t multi_ws_bytes(int64_t n, int64_t K, size_t assign_bytes) {
    return multi_layout(n, K, assign_bytes, nullptr, nullptr);
}

hipError_t launch_assign_multi(const LaunchCtx &c, int ntypes, const AssignPlan *plans, const KSet *X,
                               const KSet *Z, const KOpts &o, int32_t *labels, double *best, double *all,
                               int32_t *row_status, void *ws, size_t assign_bytes) {
    const int64_t n = X[0].n, K = Z[0].n;
    if (n == 0) return hipSuccess;
    MultiWS w;
    multi_layout(n, K, assign_bytes, ws, &w);
    double *acc = all ? all : w.acc;
    const int64_t nk = n * K;
    const unsigned eg = (unsigned)((nk + 255) / 256 < 65536 ? (nk + 255) / 256 : 65536);
    const unsigned ng = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipError_t e = hipSuccess;
    for (int m = 0; m < ntypes && e == hipSuccess; ++m) {
        e = launch_assign(c, plans[m], X[m], Z[m], o, w.slab, w.sbest, m == 0 ? acc : w.tmp, w.sst,
                          w.assign_ws);
        if (e != hipSuccess) break;
        if (m > 0) hipLaunchKernelGGL(k_multi_add, dim3(eg), dim3(256), 0, c.stream, acc, w.tmp, nk);
        hipLaunchKernelGGL(k_multi_status, dim3(ng), dim3(256), 0, c.stream, w.worst, w.sst, n, m == 0 ? 1 : 0);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const unsigned ag = (unsigned)((n + 3) / 4 < 65536 ? (n + 3) / 4 : 65536);
    hipLaunchKernelGGL(k_multi_argmin, dim3(ag), dim3(256), 0, c.stream, acc, n, K, w.worst, labels, best,
                       row_status);
    return hipGetLastError();
}

}  // namespace d2
