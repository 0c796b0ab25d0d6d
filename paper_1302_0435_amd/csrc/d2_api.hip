// Host side of the C ABI declared in include/d2.h: argument validation,
// option defaults, work planning and kernel dispatch.  Nothing here
// allocates device memory; every device buffer belongs to the caller.
#include <hip/hip_runtime.h>
#include <math.h>
#include <new>
#include <stdint.h>
#include <string.h>

#include "d2.h"
#include "d2_internal.h"

struct d2_handle {
    int device;
    int cu_count;
};

namespace {

using d2::KOpts;
using d2::KSet;

bool set_ok(const d2_set *s) {
    if (!s) return false;
    if (s->n < 0 || s->d < 1) return false;
    if (s->dtype != D2_F64 && s->dtype != D2_F32) return false;
    if (s->n > 0 && (!s->offsets || !s->points || !s->weights)) return false;
    if (s->n > 0 && s->max_support < 1) return false;
    return true;
}

KSet kset(const d2_set *s) {
    KSet k;
    k.off = s->offsets;
    k.pts = s->points;
    k.w = s->weights;
    k.n = s->n;
    k.d = s->d;
    k.dtype = s->dtype;
    return k;
}

d2_status opts_ok(const d2_opts *o, KOpts &k) {
    d2_opts def;
    memset(&def, 0, sizeof(def));
    if (!o) o = &def;
    if (o->cost_mode != D2_COST_F64_DIRECT && o->cost_mode != D2_COST_BF16_MFMA) return D2_EINVAL;
    if (o->init != D2_INIT_AUTO && o->init != D2_INIT_NWC && o->init != D2_INIT_VOGEL) return D2_EINVAL;
    if (o->max_pivots < 0) return D2_EINVAL;
    if (o->want_sqrt != 0 && o->want_sqrt != 1) return D2_EINVAL;
    if (!(o->opt_tol >= 0.0) || !isfinite(o->opt_tol) || o->opt_tol >= 1.0) return D2_EINVAL;
    k.init = o->init == D2_INIT_VOGEL ? D2_INIT_VOGEL : D2_INIT_NWC;
    k.max_pivots = o->max_pivots;
    k.want_sqrt = o->want_sqrt;
    k.cost_mode = o->cost_mode;
    k.tol = o->opt_tol > 0.0 ? o->opt_tol : 1e-14;
    return D2_OK;
}

d2_status pair_sets_ok(const d2_set *A, const d2_set *B) {
    if (!set_ok(A) || !set_ok(B)) return D2_EINVAL;
    if (A->d != B->d || A->dtype != B->dtype) return D2_EINVAL;
    if (A->max_support > D2_MAX_SUPPORT || B->max_support > D2_MAX_SUPPORT) return D2_EUNSUPPORTED;
    return D2_OK;
}

int maxsup(const d2_set *A, const d2_set *B) {
    int m = A ? A->max_support : 1;
    if (B && B->max_support > m) m = B->max_support;
    return m < 1 ? 1 : m;
}

d2_status bind_device(d2_handle *h) {
    if (hipSetDevice(h->device) != hipSuccess) return D2_EHIP;
    return D2_OK;
}

d2::LaunchCtx ctx(d2_handle *h, void *stream) {
    d2::LaunchCtx c;
    c.stream = (hipStream_t)stream;
    c.cu_count = h->cu_count;
    return c;
}

}  // namespace

extern "C" {

const char *d2_version(void) { return "d2-mi355x 0.1"; }

int d2_max_support(void) { return D2_MAX_SUPPORT; }

const char *d2_status_string(int code) {
    switch (code) {
    case D2_OK: return "ok";
    case D2_EINVAL: return "invalid argument";
    case D2_EWORKSPACE: return "workspace too small";
    case D2_EUNSUPPORTED: return "unsupported size or mode";
    case D2_EHIP: return "HIP runtime error";
    case D2_ENOMEM: return "out of host memory";
    default: return "unknown status";
    }
}

d2_status d2_create(d2_handle **h, int device) {
    if (!h) return D2_EINVAL;
    *h = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return D2_EHIP;
    if (device < 0 || device >= count) return D2_EINVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return D2_EHIP;
    d2_handle *p = new (std::nothrow) d2_handle;
    if (!p) return D2_ENOMEM;
    p->device = device;
    p->cu_count = prop.multiProcessorCount;
    *h = p;
    return D2_OK;
}

d2_status d2_destroy(d2_handle *h) {
    delete h;
    return D2_OK;
}

size_t d2_workspace_bytes(d2_handle *h, int which, const d2_set *A, const d2_set *B,
                          int64_t npairs, const d2_opts *opts) {
    (void)npairs;
    (void)opts;
    if (!h || !A) return 0;
    if (which == 2 && B) {
        KSet X = kset(A), Z = kset(B);
        return d2::plan_assign(X, Z, maxsup(A, B), h->cu_count).ws_bytes;
    }
    return 0;
}

d2_status d2_cost_tiles(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                        int64_t npairs, int32_t cost_mode, double *tiles,
                        const int64_t *tile_offsets, void *ws, size_t ws_bytes, void *stream) {
    (void)ws;
    (void)ws_bytes;
    if (!h || npairs < 0) return D2_EINVAL;
    d2_status st = pair_sets_ok(A, B);
    if (st != D2_OK) return st;
    if (cost_mode != D2_COST_F64_DIRECT && cost_mode != D2_COST_BF16_MFMA) return D2_EINVAL;
    if (npairs > 0 && (!pairs || !tiles || !tile_offsets)) return D2_EINVAL;
    if (cost_mode == D2_COST_BF16_MFMA) return D2_EUNSUPPORTED;
    if ((st = bind_device(h)) != D2_OK) return st;
    hipError_t e = d2::launch_cost_tiles(ctx(h, stream), kset(A), kset(B), pairs, npairs, cost_mode,
                                         tiles, tile_offsets);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_emd_batch(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                       int64_t npairs, const d2_opts *opts, double *dist,
                       const int64_t *plan_offsets, double *plan, const int64_t *dual_offsets,
                       double *duals, int32_t *pair_status, void *ws, size_t ws_bytes,
                       void *stream) {
    (void)ws;
    (void)ws_bytes;
    if (!h || npairs < 0) return D2_EINVAL;
    d2_status st = pair_sets_ok(A, B);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (npairs > 0 && (!pairs || !dist)) return D2_EINVAL;
    if ((plan == nullptr) != (plan_offsets == nullptr)) return D2_EINVAL;
    if ((duals == nullptr) != (dual_offsets == nullptr)) return D2_EINVAL;
    if ((st = bind_device(h)) != D2_OK) return st;
    hipError_t e = d2::launch_emd_pairs(ctx(h, stream), d2::group_width_for(maxsup(A, B)), kset(A),
                                        kset(B), pairs, npairs, k, dist, plan_offsets, plan,
                                        dual_offsets, duals, pair_status);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_assign(d2_handle *h, const d2_set *X, const d2_set *Z, const d2_opts *opts,
                    int32_t *labels, double *best, double *all, int32_t *row_status, void *ws,
                    size_t ws_bytes, void *stream) {
    if (!h) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, Z);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (X->n > 0 && (!labels || !best)) return D2_EINVAL;
    if (X->n > 0 && Z->n < 1) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    KSet kx = kset(X), kz = kset(Z);
    d2::AssignPlan p = d2::plan_assign(kx, kz, maxsup(X, Z), h->cu_count);
    if (p.ws_bytes > 0 && (!ws || ws_bytes < p.ws_bytes)) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    hipError_t e = d2::launch_assign(ctx(h, stream), p, kx, kz, k, labels, best, all, row_status, ws);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_pairwise(d2_handle *h, const d2_set *X, const d2_opts *opts, double *condensed,
                      int32_t *pair_status, void *ws, size_t ws_bytes, void *stream) {
    (void)ws;
    (void)ws_bytes;
    if (!h) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, X);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (X->n > 1 && !condensed) return D2_EINVAL;
    if ((st = bind_device(h)) != D2_OK) return st;
    hipError_t e = d2::launch_pairwise(ctx(h, stream), d2::group_width_for(maxsup(X, X)), kset(X), k,
                                       condensed, pair_status);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

}  // extern "C"
