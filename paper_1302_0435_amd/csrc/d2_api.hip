// Host side of the C ABI declared in include/d2.h: argument validation,
// option defaults, work planning, kernel dispatch, hipGraph capture/replay
// and the schedule autotuner.  Nothing here allocates device memory; every
// device buffer belongs to the caller, except the fixed scratch array that
// d2_assign_noalloc uses in place of a workspace (a file-scope __device__
// array, one copy per GPU, held until the process ends).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "d2.h"
#include "d2_internal.h"

namespace {

using d2::KOpts;
using d2::KSet;

// One captured call: the arguments that fix its kernels and the executable.
struct GraphEntry {
    int which;
    uint64_t key[24];
    hipGraphExec_t exec;
    uint64_t last_use;
};

// Autotuned pairwise schedule for one workload shape.
struct TuneEntry {
    int64_t n;
    int d, dtype, max_support, init;
    d2::Schedule sch;
};

}  // namespace

struct d2_handle {
    int device;
    int cu_count;
    void *scratch;                  // this device's copy of `scratch` (device address)
    hipStream_t capture;            // private stream used only to record graphs
    std::vector<GraphEntry> graphs;
    std::vector<TuneEntry> tuned;
    uint64_t clock;
};

// Workspace of d2_assign_noalloc: the partial minima of split centroid
// ranges and the support-class sort live here instead of in a caller
// buffer.  In host code the name stands for a host-side shadow, not device
// memory: only the address from hipGetSymbolAddress (kept per device in
// g_scratch) may be handed to kernels.
static __device__ __align__(256) unsigned char scratch[D2_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = (size_t)D2_NOALLOC_SCRATCH_BYTES;
// Largest per-cluster slab of the free-weight update (the dense inverse of a
// basis of max_members (xmax + zmax - 1) + 1 rows): 8 GiB.
constexpr size_t kMaxFreeSlab = (size_t)8 << 30;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];

// The device address of `scratch` on `device` (current), looked up once per
// device; nullptr on failure.
void *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[device] = p;
    }
    return g_scratch[device];
}

constexpr size_t kMaxGraphs = 32;

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

d2_opts defaults() {
    d2_opts o;
    memset(&o, 0, sizeof(o));
    return o;
}

d2_status opts_ok(const d2_opts *o, KOpts &k) {
    static const d2_opts def = defaults();
    if (!o) o = &def;
    if (o->cost_mode != D2_COST_F64_DIRECT && o->cost_mode != D2_COST_BF16_MFMA) return D2_EINVAL;
    if (o->init < D2_INIT_AUTO || o->init > D2_INIT_LCM) return D2_EINVAL;
    if (o->max_pivots < 0) return D2_EINVAL;
    if (o->want_sqrt != 0 && o->want_sqrt != 1) return D2_EINVAL;
    if (!(o->opt_tol >= 0.0) || !isfinite(o->opt_tol) || o->opt_tol >= 1.0) return D2_EINVAL;
    if (o->schedule != D2_SCHED_AUTO && o->schedule != D2_SCHED_PLAIN) return D2_EINVAL;
    if (o->flags & ~D2_FLAG_EAGER) return D2_EINVAL;
    if (o->bland_after < 0) return D2_EINVAL;
    k.init = o->init == D2_INIT_NWC ? d2::kStartNWC : o->init == D2_INIT_VOGEL ? d2::kStartVogel : d2::kStartLCM;
    k.max_pivots = o->max_pivots;
    k.want_sqrt = o->want_sqrt;
    k.cost_mode = o->cost_mode;
    k.bland_after = o->bland_after;
    k.tol = o->opt_tol > 0.0 ? o->opt_tol : 1e-14;
    return D2_OK;
}

int sched_of(const d2_opts *o) { return o ? o->schedule : D2_SCHED_AUTO; }
bool eager_of(const d2_opts *o) { return o && (o->flags & D2_FLAG_EAGER); }

d2_status pair_sets_ok(const d2_set *A, const d2_set *B) {
    if (!set_ok(A) || !set_ok(B)) return D2_EINVAL;
    if (A->d != B->d || A->dtype != B->dtype) return D2_EINVAL;
    if (A->max_support > D2_MAX_SUPPORT || B->max_support > D2_MAX_SUPPORT) return D2_EUNSUPPORTED;
    return D2_OK;
}

int ms(const d2_set *s) { return s && s->max_support > 0 ? s->max_support : 1; }

// Pairs beyond the lane-group shapes go to the workgroup simplex.
bool large_pairs(const d2_set *A, const d2_set *B) {
    return A->max_support > D2_MAX_SUPPORT || B->max_support > D2_MAX_SUPPORT;
}

// Sets a workgroup-simplex call accepts (supports up to D2_MAX_SUPPORT_LARGE).
d2_status large_sets_ok(const d2_set *A, const d2_set *B) {
    if (!set_ok(A) || !set_ok(B)) return D2_EINVAL;
    if (A->d != B->d || A->dtype != B->dtype) return D2_EINVAL;
    if (A->max_support > D2_MAX_SUPPORT_LARGE || B->max_support > D2_MAX_SUPPORT_LARGE) return D2_EUNSUPPORTED;
    return D2_OK;
}

d2_status bind_device(d2_handle *h) {
    return hipSetDevice(h->device) == hipSuccess ? D2_OK : D2_EHIP;
}

d2::LaunchCtx ctx(d2_handle *h, hipStream_t s) {
    d2::LaunchCtx c;
    c.stream = s;
    c.cu_count = h->cu_count;
    return c;
}

void key_set(uint64_t *k, int &n, const d2_set *s) {
    k[n++] = (uint64_t)s->n;
    k[n++] = ((uint64_t)(uint32_t)s->d << 32) | (uint32_t)s->dtype;
    k[n++] = (uint64_t)(uintptr_t)s->offsets;
    k[n++] = (uint64_t)(uintptr_t)s->points;
    k[n++] = (uint64_t)(uintptr_t)s->weights;
    k[n++] = (uint64_t)s->max_support;
}

void key_opts(uint64_t *k, int &n, const KOpts &o) {
    k[n++] = ((uint64_t)(uint32_t)o.init << 32) | (uint32_t)o.max_pivots;
    k[n++] = ((uint64_t)(uint32_t)o.want_sqrt << 32) | (uint32_t)o.cost_mode;
    k[n++] = (uint64_t)(uint32_t)o.bland_after;
    uint64_t t;
    memcpy(&t, &o.tol, sizeof(t));
    k[n++] = t;
}

// Run `enqueue(stream)` either directly on the caller's stream or as a
// hipGraph: recorded once on the handle's private stream, then replayed on
// the caller's stream whenever a call with the same key comes again.
template <typename F>
d2_status run_graph(d2_handle *h, int which, const uint64_t *key, bool eager, hipStream_t stream,
                    F &&enqueue) {
    if (eager) return enqueue(stream) == hipSuccess ? D2_OK : D2_EHIP;
    for (auto &g : h->graphs) {
        if (g.which == which && memcmp(g.key, key, sizeof(g.key)) == 0) {
            g.last_use = ++h->clock;
            return hipGraphLaunch(g.exec, stream) == hipSuccess ? D2_OK : D2_EHIP;
        }
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return D2_EHIP;
    hipError_t e = enqueue(h->capture);
    hipError_t e2 = hipStreamEndCapture(h->capture, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return D2_EHIP;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return D2_EHIP;
    if (h->graphs.size() >= kMaxGraphs) {
        size_t victim = 0;
        for (size_t i = 1; i < h->graphs.size(); ++i)
            if (h->graphs[i].last_use < h->graphs[victim].last_use) victim = i;
        (void)hipGraphExecDestroy(h->graphs[victim].exec);
        h->graphs.erase(h->graphs.begin() + victim);
    }
    GraphEntry g;
    g.which = which;
    memcpy(g.key, key, sizeof(g.key));
    g.exec = exec;
    g.last_use = ++h->clock;
    h->graphs.push_back(g);
    return hipGraphLaunch(exec, stream) == hipSuccess ? D2_OK : D2_EHIP;
}

constexpr int kMaxTypes = 16;

// Checks the sets of a multi-type call and plans each type's labelling;
// returns the largest per-type workspace through *assign_bytes.
d2_status multi_plans(d2_handle *h, int ntypes, const d2_set *X, const d2_set *Z, int sched, int cost_mode,
                      d2::AssignPlan *plans, size_t *assign_bytes) {
    if (ntypes < 1 || ntypes > kMaxTypes || !X || !Z) return D2_EINVAL;
    size_t mx = 0;
    for (int m = 0; m < ntypes; ++m) {
        d2_status st = pair_sets_ok(&X[m], &Z[m]);
        if (st != D2_OK) return st;
        if (X[m].n != X[0].n || Z[m].n != Z[0].n) return D2_EINVAL;
        if (cost_mode == D2_COST_BF16_MFMA && (ms(&X[m]) > 32 || ms(&Z[m]) > 32)) return D2_EUNSUPPORTED;
        plans[m] = d2::plan_assign(kset(&X[m]), kset(&Z[m]), ms(&X[m]), ms(&Z[m]), h->cu_count, sched, cost_mode);
        if (plans[m].ws_bytes > mx) mx = plans[m].ws_bytes;
    }
    *assign_bytes = mx;
    return D2_OK;
}

d2::Schedule default_schedule() {
    d2::Schedule s;
    for (int c = 0; c < 4; ++c) { s.blocks_per_cu[c] = 4; s.chunk[c] = 4; s.tile[c] = 512; }
    s.blocks_per_cu[3] = 8;   // one-wave workgroups, two per SIMD
    s.edge[0] = 16;
    s.edge[1] = 32;
    return s;
}

d2::Schedule schedule_for(d2_handle *h, const d2_set *X, const KOpts &k) {
    for (auto &t : h->tuned)
        if (t.n == X->n && t.d == X->d && t.dtype == X->dtype && t.max_support == X->max_support &&
            t.init == k.init)
            return t.sch;
    return default_schedule();
}

}  // namespace

extern "C" {

const char *d2_version(void) { return "d2-mi355x 0.2"; }

int d2_max_support(void) { return D2_MAX_SUPPORT; }

const char *d2_status_string(int code) {
    switch (code) {
    case D2_OK: return "ok";
    case D2_EINVAL: return "invalid argument";
    case D2_EWORKSPACE: return "workspace too small";
    case D2_EUNSUPPORTED: return "unsupported size or mode";
    case D2_EHIP: return "HIP runtime error";
    case D2_ENOMEM: return "out of host memory";
    case D2_ESCRATCH: return "call needs more than the fixed scratch of d2_assign_noalloc";
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
    if (hipSetDevice(device) != hipSuccess) return D2_EHIP;
    void *scr = scratch_on(device);
    if (!scr) return D2_EHIP;
    d2_handle *p = new (std::nothrow) d2_handle;
    if (!p) return D2_ENOMEM;
    p->device = device;
    p->cu_count = prop.multiProcessorCount;
    p->scratch = scr;
    p->clock = 0;
    if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return D2_EHIP;
    }
    *h = p;
    return D2_OK;
}

d2_status d2_destroy(d2_handle *h) {
    if (!h) return D2_OK;
    (void)hipSetDevice(h->device);
    for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    (void)hipStreamDestroy(h->capture);
    delete h;
    return D2_OK;
}

size_t d2_workspace_bytes(d2_handle *h, int which, const d2_set *A, const d2_set *B,
                          int64_t npairs, const d2_opts *opts) {
    if (!h || !A || !set_ok(A)) return 0;
    const int sched = sched_of(opts);
    if (which == 1 && B && set_ok(B) && large_pairs(A, B)) {
        int64_t grid, elems;
        d2::wg_plan(npairs, ms(A), ms(B), h->cu_count, &grid, &elems);
        return (size_t)(grid * elems) * sizeof(double);
    }
    if (which == 2 && B && set_ok(B) && large_pairs(A, B))
        return d2::wg_assign_bytes(A->n, B->n, ms(A), ms(B), h->cu_count);
    if (which == 3 && large_pairs(A, A)) return d2::wg_pairwise_bytes(A->n, ms(A), h->cu_count);
    if (which == 2 && B && set_ok(B)) {
        KSet X = kset(A), Z = kset(B);
        return d2::plan_assign(X, Z, ms(A), ms(B), h->cu_count, sched,
                               opts ? opts->cost_mode : D2_COST_F64_DIRECT).ws_bytes;
    }
    if (which == 3) return d2::plan_pairwise(kset(A), ms(A), sched).ws_bytes;
    if (which == 4 && B && set_ok(B)) return d2::update_ws_bytes(A->n, B->n, A->d, ms(A), ms(B));
    if (which == 6 && B && set_ok(B)) {
        if (npairs < 1 || npairs > INT32_MAX ||
            d2::update_free_slab_bytes((int)npairs, ms(A), ms(B), A->d) > kMaxFreeSlab)
            return 0;
        return d2::update_free_ws_bytes(A->n, B->n, A->d, ms(A), ms(B), (int)npairs, h->cu_count, nullptr);
    }
    if (which == 7) return npairs >= 0 ? d2::merge_ws_bytes(npairs, A->n) : 0;
    if (which == 5 && B) {
        d2::AssignPlan plans[kMaxTypes];
        size_t ab = 0;
        if (multi_plans(h, (int)npairs, A, B, sched, opts ? opts->cost_mode : D2_COST_F64_DIRECT, plans, &ab) !=
            D2_OK)
            return 0;
        return d2::multi_ws_bytes(A->n, B->n, ab);
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
    if (cost_mode == D2_COST_BF16_MFMA && (A->max_support > 32 || B->max_support > 32))
        return D2_EUNSUPPORTED;
    if ((st = bind_device(h)) != D2_OK) return st;
    hipError_t e = d2::launch_cost_tiles(ctx(h, (hipStream_t)stream), kset(A), kset(B), pairs, npairs,
                                         cost_mode, tiles, tile_offsets);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_emd_batch(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                       int64_t npairs, const d2_opts *opts, double *dist,
                       const int64_t *plan_offsets, double *plan, const int64_t *dual_offsets,
                       double *duals, int32_t *pair_status, int32_t *pivots, void *ws,
                       size_t ws_bytes, void *stream) {
    if (!h || npairs < 0) return D2_EINVAL;
    if (!set_ok(A) || !set_ok(B)) return D2_EINVAL;
    if (A->d != B->d || A->dtype != B->dtype) return D2_EINVAL;
    if (A->max_support > D2_MAX_SUPPORT_LARGE || B->max_support > D2_MAX_SUPPORT_LARGE) return D2_EUNSUPPORTED;
    KOpts k;
    d2_status st = opts_ok(opts, k);
    if (st != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (npairs > 0 && (!pairs || !dist)) return D2_EINVAL;
    if ((plan == nullptr) != (plan_offsets == nullptr)) return D2_EINVAL;
    if ((duals == nullptr) != (dual_offsets == nullptr)) return D2_EINVAL;
    if (large_pairs(A, B)) {
        int64_t grid, elems;
        d2::wg_plan(npairs, ms(A), ms(B), h->cu_count, &grid, &elems);
        if (npairs > 0 && (!ws || ws_bytes < (size_t)(grid * elems) * sizeof(double))) return D2_EWORKSPACE;
        if ((st = bind_device(h)) != D2_OK) return st;
        hipError_t e = d2::launch_emd_wg(ctx(h, (hipStream_t)stream), kset(A), kset(B), pairs, npairs, k, ms(A),
                                         ms(B), dist, plan_offsets, plan, dual_offsets, duals, pair_status, pivots,
                                         ws);
        return e == hipSuccess ? D2_OK : D2_EHIP;
    }
    if ((st = bind_device(h)) != D2_OK) return st;
    const int cls = sched_of(opts) == D2_SCHED_PLAIN ? 3 : d2::class_for(ms(A), ms(B));
    hipError_t e = d2::launch_emd_pairs(ctx(h, (hipStream_t)stream), cls, kset(A), kset(B), pairs,
                                        npairs, k, dist, plan_offsets, plan, dual_offsets, duals,
                                        pair_status, pivots);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_emd_batch_basis(d2_handle *h, const d2_set *A, const d2_set *B, const int64_t *pairs,
                             int64_t npairs, const d2_opts *opts, double *dist, const int64_t *basis_offsets,
                             int32_t *basis_ij, double *basis_w, int32_t *pair_status, void *stream) {
    if (!h || npairs < 0) return D2_EINVAL;
    d2_status st = pair_sets_ok(A, B);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (npairs > 0 && (!pairs || !dist || !basis_offsets || !basis_ij || !basis_w)) return D2_EINVAL;
    if ((st = bind_device(h)) != D2_OK) return st;
    const int cls = sched_of(opts) == D2_SCHED_PLAIN ? 3 : d2::class_for(ms(A), ms(B));
    hipError_t e = d2::launch_emd_basis(ctx(h, (hipStream_t)stream), cls, kset(A), kset(B), pairs, npairs, k, dist,
                                        basis_offsets, basis_ij, basis_w, pair_status);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_assign(d2_handle *h, const d2_set *X, const d2_set *Z, const d2_opts *opts,
                    int32_t *labels, double *best, double *all, int32_t *row_status, void *ws,
                    size_t ws_bytes, void *stream) {
    if (!h) return D2_EINVAL;
    if (X && Z && set_ok(X) && set_ok(Z) && large_pairs(X, Z)) {
        // supports beyond the lane-group shapes: the workgroup simplex
        d2_status st = large_sets_ok(X, Z);
        if (st != D2_OK) return st;
        KOpts k;
        if ((st = opts_ok(opts, k)) != D2_OK) return st;
        if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
        if (X->n > 0 && (!labels || !best)) return D2_EINVAL;
        if (X->n > 0 && Z->n < 1) return D2_EINVAL;
        if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
        const size_t need = d2::wg_assign_bytes(X->n, Z->n, ms(X), ms(Z), h->cu_count);
        if (X->n > 0 && (!ws || ws_bytes < need)) return D2_EWORKSPACE;
        if ((st = bind_device(h)) != D2_OK) return st;
        hipError_t e = d2::launch_assign_wg(ctx(h, (hipStream_t)stream), kset(X), kset(Z), k, ms(X), ms(Z), labels,
                                            best, all, row_status, ws);
        return e == hipSuccess ? D2_OK : D2_EHIP;
    }
    d2_status st = pair_sets_ok(X, Z);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode == D2_COST_BF16_MFMA && (ms(X) > 32 || ms(Z) > 32)) return D2_EUNSUPPORTED;
    if (X->n > 0 && (!labels || !best)) return D2_EINVAL;
    if (X->n > 0 && Z->n < 1) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    KSet kx = kset(X), kz = kset(Z);
    d2::AssignPlan p = d2::plan_assign(kx, kz, ms(X), ms(Z), h->cu_count, sched_of(opts), k.cost_mode);
    if (p.ws_bytes > 0 && (!ws || ws_bytes < p.ws_bytes)) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    if (X->n == 0) return D2_OK;
    uint64_t key[24];
    memset(key, 0, sizeof(key));
    int n = 0;
    key_set(key, n, X);
    key_set(key, n, Z);
    key_opts(key, n, k);
    key[n++] = (uint64_t)(uintptr_t)labels;
    key[n++] = (uint64_t)(uintptr_t)best;
    key[n++] = (uint64_t)(uintptr_t)all;
    key[n++] = (uint64_t)(uintptr_t)row_status;
    key[n++] = (uint64_t)(uintptr_t)ws;
    key[n++] = (uint64_t)sched_of(opts);
    return run_graph(h, 2, key, eager_of(opts), (hipStream_t)stream, [&](hipStream_t s) {
        return d2::launch_assign(ctx(h, s), p, kx, kz, k, labels, best, all, row_status, ws);
    });
}

d2_status d2_assign_noalloc(d2_handle *h, const d2_set *X, const d2_set *Z, const d2_opts *opts,
                            int32_t *labels, double *best, double *all, int32_t *row_status, void *stream) {
    if (!h) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, Z);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode == D2_COST_BF16_MFMA && (ms(X) > 32 || ms(Z) > 32)) return D2_EUNSUPPORTED;
    if (X->n > 0 && (!labels || !best)) return D2_EINVAL;
    if (X->n > 0 && Z->n < 1) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    KSet kx = kset(X), kz = kset(Z);
    d2::AssignPlan p = d2::plan_assign(kx, kz, ms(X), ms(Z), h->cu_count, sched_of(opts), k.cost_mode);
    if (p.ws_bytes > kScratchBytes) return D2_ESCRATCH;
    if ((st = bind_device(h)) != D2_OK) return st;
    if (X->n == 0) return D2_OK;
    // enqueued directly: recording a graph could allocate
    return d2::launch_assign(ctx(h, (hipStream_t)stream), p, kx, kz, k, labels, best, all, row_status,
                             h->scratch) == hipSuccess
               ? D2_OK
               : D2_EHIP;
}

d2_status d2_emd_cost_batch(d2_handle *h, int64_t nprob, const int64_t *row_offsets,
                            const double *row_weights, const int64_t *col_offsets,
                            const double *col_weights, const double *costs,
                            const int64_t *cost_offsets, int32_t max_rows, int32_t max_cols,
                            const d2_opts *opts, double *dist, const int64_t *plan_offsets,
                            double *plan, int32_t *status, void *ws, size_t ws_bytes,
                            void *stream) {
    (void)ws;
    (void)ws_bytes;
    if (!h || nprob < 0) return D2_EINVAL;
    if (max_rows < 1 || max_cols < 1) return D2_EINVAL;
    if (max_rows > D2_MAX_SUPPORT || max_cols > D2_MAX_SUPPORT) return D2_EUNSUPPORTED;
    KOpts k;
    d2_status st = opts_ok(opts, k);
    if (st != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (nprob > 0 && (!row_offsets || !row_weights || !col_offsets || !col_weights || !costs ||
                      !cost_offsets || !dist))
        return D2_EINVAL;
    if ((plan == nullptr) != (plan_offsets == nullptr)) return D2_EINVAL;
    if ((st = bind_device(h)) != D2_OK) return st;
    const int cls = sched_of(opts) == D2_SCHED_PLAIN ? 3 : d2::class_for(max_rows, max_cols);
    hipError_t e = d2::launch_emd_cost(ctx(h, (hipStream_t)stream), cls, nprob, row_offsets, row_weights,
                                       col_offsets, col_weights, costs, cost_offsets, max_rows, max_cols, k,
                                       dist, plan_offsets, plan, status);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_centroid_update(d2_handle *h, const d2_set *X, const d2_set *Z, const int32_t *labels,
                             const double *obj_weights, const d2_opts *opts, double *z_new,
                             double *eps_step1, double *eps_step3, int32_t *counts,
                             int32_t *obj_status, void *ws, size_t ws_bytes, void *stream) {
    if (!h) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, Z);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (X->n > 0 && !labels) return D2_EINVAL;
    if (Z->n > 0 && !z_new) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    if (Z->n > 0 && (const void *)z_new == Z->points) return D2_EINVAL;
    const size_t need = d2::update_ws_bytes(X->n, Z->n, X->d, ms(X), ms(Z));
    if (!ws || ws_bytes < need) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    if (X->n == 0 && Z->n == 0) return D2_OK;
    const int cls = sched_of(opts) == D2_SCHED_PLAIN ? 3 : d2::class_for(ms(X), ms(Z));
    hipError_t e = d2::launch_update(ctx(h, (hipStream_t)stream), cls, kset(X), kset(Z), ms(X), ms(Z), k,
                                     labels, obj_weights, z_new, eps_step1, eps_step3, counts, obj_status, ws);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_centroid_update_free(d2_handle *h, const d2_set *X, const d2_set *Z, const int32_t *labels,
                                  const double *obj_weights, int32_t max_members, const d2_opts *opts,
                                  double *z_new, double *w_new, double *eps_step1, double *eps_step3,
                                  int32_t *counts, int32_t *obj_status, int32_t *cluster_status,
                                  int32_t *cluster_pivots, int32_t *basis_io, int64_t basis_stride, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (!h) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, Z);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (max_members < 1) return D2_EINVAL;
    if (basis_io && basis_stride < 2) return D2_EINVAL;
    if (X->n > 0 && !labels) return D2_EINVAL;
    if (Z->n > 0 && (!z_new || !w_new)) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    if (Z->n > 0 && ((const void *)z_new == Z->points || (const void *)w_new == Z->weights)) return D2_EINVAL;
    if (d2::update_free_slab_bytes(max_members, ms(X), ms(Z), X->d) > kMaxFreeSlab) return D2_EUNSUPPORTED;
    const size_t need = d2::update_free_ws_bytes(X->n, Z->n, X->d, ms(X), ms(Z), max_members, h->cu_count, nullptr);
    if (!ws || ws_bytes < need) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    if (X->n == 0 && Z->n == 0) return D2_OK;
    hipError_t e = d2::launch_update_free(ctx(h, (hipStream_t)stream), kset(X), kset(Z), ms(X), ms(Z),
                                          max_members, k, labels, obj_weights, z_new, w_new, eps_step1, eps_step3,
                                          counts, obj_status, cluster_status, cluster_pivots, basis_io,
                                          basis_stride, ws);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_merge_level(d2_handle *h, const d2_set *Z, int64_t n, const int32_t *labels, const double *omega,
                         int64_t n0, int32_t *C, int64_t *kept, int64_t *new_offsets, void *new_points,
                         void *new_weights, double *new_omega, void *ws, size_t ws_bytes, void *stream) {
    if (!h || !set_ok(Z) || n < 0 || n0 < 0) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    if (!kept || !new_offsets) return D2_EINVAL;
    if (n > 0 && !labels) return D2_EINVAL;
    if (n0 > 0 && !C) return D2_EINVAL;
    if (Z->n > 0 && (!new_points || !new_weights || !new_omega)) return D2_EINVAL;
    if (Z->n > 0 && (new_points == Z->points || new_weights == Z->weights)) return D2_EINVAL;
    if (n0 > 0 && n > 0 && (const void *)C == (const void *)labels) return D2_EINVAL;
    const size_t need = d2::merge_ws_bytes(n, Z->n);
    if (!ws || ws_bytes < need) return D2_EWORKSPACE;
    if (bind_device(h) != D2_OK) return D2_EHIP;
    hipError_t e = d2::launch_merge_level(ctx(h, (hipStream_t)stream), kset(Z), n, labels, omega, n0, C, kept,
                                          new_offsets, new_points, new_weights, new_omega, ws);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_assign_multi(d2_handle *h, int32_t ntypes, const d2_set *X, const d2_set *Z,
                          const d2_opts *opts, int32_t *labels, double *best, double *all,
                          int32_t *row_status, void *ws, size_t ws_bytes, void *stream) {
    if (!h) return D2_EINVAL;
    KOpts k;
    d2_status st = opts_ok(opts, k);
    if (st != D2_OK) return st;
    d2::AssignPlan plans[kMaxTypes];
    size_t ab = 0;
    if ((st = multi_plans(h, ntypes, X, Z, sched_of(opts), k.cost_mode, plans, &ab)) != D2_OK) return st;
    const int64_t n = X[0].n, K = Z[0].n;
    if (n > 0 && (!labels || !best)) return D2_EINVAL;
    if (n > 0 && K < 1) return D2_EINVAL;
    if (K > INT32_MAX) return D2_EUNSUPPORTED;
    const size_t need = d2::multi_ws_bytes(n, K, ab);
    if (!ws || ws_bytes < need) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    KSet kx[kMaxTypes], kz[kMaxTypes];
    for (int m = 0; m < ntypes; ++m) { kx[m] = kset(&X[m]); kz[m] = kset(&Z[m]); }
    hipError_t e = d2::launch_assign_multi(ctx(h, (hipStream_t)stream), ntypes, plans, kx, kz, k, labels, best,
                                           all, row_status, ws, ab);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_assign_segmented(d2_handle *h, const d2_set *X, const d2_set *Z, const int32_t *seg,
                              int64_t nseg, const int64_t *zseg_offsets, const d2_opts *opts,
                              int32_t *labels, double *best, int32_t *row_status, void *stream) {
    if (!h || nseg < 0) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, Z);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (X->n > 0 && (!seg || !labels || !best || (nseg > 0 && !zseg_offsets))) return D2_EINVAL;
    if (Z->n > INT32_MAX) return D2_EUNSUPPORTED;
    if ((st = bind_device(h)) != D2_OK) return st;
    const int cls = sched_of(opts) == D2_SCHED_PLAIN ? 3 : d2::class_for(ms(X), ms(Z));
    hipError_t e = d2::launch_assign_seg(ctx(h, (hipStream_t)stream), cls, kset(X), kset(Z), k, seg, nseg,
                                         zseg_offsets, labels, best, row_status);
    return e == hipSuccess ? D2_OK : D2_EHIP;
}

d2_status d2_pairwise(d2_handle *h, const d2_set *X, const d2_opts *opts, double *condensed,
                      int32_t *pair_status, void *ws, size_t ws_bytes, void *stream) {
    if (!h) return D2_EINVAL;
    if (X && set_ok(X) && large_pairs(X, X)) {
        // supports beyond the lane-group shapes: the workgroup simplex
        d2_status st = large_sets_ok(X, X);
        if (st != D2_OK) return st;
        KOpts k;
        if ((st = opts_ok(opts, k)) != D2_OK) return st;
        if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
        if (X->n > 1 && !condensed) return D2_EINVAL;
        if (X->n > 1 && (!ws || ws_bytes < d2::wg_pairwise_bytes(X->n, ms(X), h->cu_count))) return D2_EWORKSPACE;
        if ((st = bind_device(h)) != D2_OK) return st;
        if (X->n < 2) return D2_OK;
        hipError_t e = d2::launch_pairwise_wg(ctx(h, (hipStream_t)stream), kset(X), k, ms(X), condensed,
                                              pair_status, ws);
        return e == hipSuccess ? D2_OK : D2_EHIP;
    }
    d2_status st = pair_sets_ok(X, X);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (X->n > 1 && !condensed) return D2_EINVAL;
    KSet kx = kset(X);
    d2::PairwisePlan p = d2::plan_pairwise(kx, ms(X), sched_of(opts));
    if (p.ws_bytes > 0 && (!ws || ws_bytes < p.ws_bytes)) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    if (X->n < 2) return D2_OK;
    const d2::Schedule sch = schedule_for(h, X, k);
    uint64_t key[24];
    memset(key, 0, sizeof(key));
    int n = 0;
    key_set(key, n, X);
    key_opts(key, n, k);
    key[n++] = (uint64_t)(uintptr_t)condensed;
    key[n++] = (uint64_t)(uintptr_t)pair_status;
    key[n++] = (uint64_t)(uintptr_t)ws;
    key[n++] = (uint64_t)sched_of(opts);
    for (int c = 0; c < 4; ++c)
        key[n++] = ((uint64_t)(uint32_t)sch.blocks_per_cu[c] << 42) | ((uint64_t)(uint32_t)sch.chunk[c] << 21) |
                   (uint32_t)sch.tile[c];
    key[n++] = ((uint64_t)(uint32_t)sch.edge[0] << 32) | (uint32_t)sch.edge[1];
    return run_graph(h, 3, key, eager_of(opts), (hipStream_t)stream, [&](hipStream_t s) {
        return d2::launch_pairwise(ctx(h, s), p, kx, k, condensed, pair_status, ws, sch);
    });
}

d2_status d2_tune_pairwise(d2_handle *h, const d2_set *X, const d2_opts *opts, double *condensed,
                           int32_t *pair_status, void *ws, size_t ws_bytes, void *stream,
                           double *best_ms) {
    if (!h) return D2_EINVAL;
    d2_status st = pair_sets_ok(X, X);
    if (st != D2_OK) return st;
    KOpts k;
    if ((st = opts_ok(opts, k)) != D2_OK) return st;
    if (k.cost_mode != D2_COST_F64_DIRECT) return D2_EUNSUPPORTED;
    if (sched_of(opts) != D2_SCHED_AUTO) return D2_EINVAL;
    if (X->n > 1 && !condensed) return D2_EINVAL;
    KSet kx = kset(X);
    d2::PairwisePlan p = d2::plan_pairwise(kx, ms(X), D2_SCHED_AUTO);
    if (p.ws_bytes > 0 && (!ws || ws_bytes < p.ws_bytes)) return D2_EWORKSPACE;
    if ((st = bind_device(h)) != D2_OK) return st;
    if (X->n < 2) { if (best_ms) *best_ms = 0.0; return D2_OK; }
    hipStream_t s = (hipStream_t)stream;
    // The classes run one after another, so each is tuned on its own launch
    // (the sort plus that class): persistent workgroups per CU x work-queue
    // chunk x tile width, coordinate by coordinate from the defaults.  Then
    // the bin edges of classes 0 and 1 (moving objects of support just below
    // an edge into the next, wider shape), timed on the whole call.
    static const int kBlocks[] = {2, 4, 8};
    static const int kChunk[] = {1, 4, 16};
    static const int kTile[] = {128, 512, 2048};
    static const int kEdge0[] = {16, 12, 8};
    static const int kEdge1[] = {32, 24};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return D2_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return D2_EHIP; }
    hipError_t e = hipSuccess;
    auto timed = [&](const d2::Schedule &sch, int only) -> float {
        float ms_ = 1e30f;
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = d2::launch_pairwise(ctx(h, s), p, kx, k, condensed, pair_status, ws, sch, only);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms_, e0, e1);
        return e == hipSuccess ? ms_ : 1e30f;
    };
    d2::Schedule best_sch = default_schedule();
    for (int c = 0; c < 4 && e == hipSuccess; ++c) {
        float bc = timed(best_sch, c);
        for (int bi = 0; bi < 3; ++bi) {
            d2::Schedule t = best_sch;
            t.blocks_per_cu[c] = kBlocks[bi];
            const float m = timed(t, c);
            if (m < bc) { bc = m; best_sch = t; }
        }
        for (int ci = 0; ci < 3; ++ci) {
            d2::Schedule t = best_sch;
            t.chunk[c] = kChunk[ci];
            const float m = timed(t, c);
            if (m < bc) { bc = m; best_sch = t; }
        }
        for (int ti = 0; ti < 3; ++ti) {
            d2::Schedule t = best_sch;
            t.tile[c] = kTile[ti];
            const float m = timed(t, c);
            if (m < bc) { bc = m; best_sch = t; }
        }
    }
    float best = timed(best_sch, -1);
    for (int a0 = 0; a0 < 3 && e == hipSuccess; ++a0)
        for (int a1 = 0; a1 < 2 && e == hipSuccess; ++a1) {
            d2::Schedule t = best_sch;
            t.edge[0] = kEdge0[a0];
            t.edge[1] = kEdge1[a1];
            if (t.edge[0] == best_sch.edge[0] && t.edge[1] == best_sch.edge[1]) continue;
            const float m = timed(t, -1);
            if (m < best) { best = m; best_sch = t; }
        }
    // the condensed output holds the chosen schedule's full result
    if (e == hipSuccess) best = timed(best_sch, -1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return D2_EHIP;
    bool found = false;
    for (auto &t : h->tuned)
        if (t.n == X->n && t.d == X->d && t.dtype == X->dtype && t.max_support == X->max_support &&
            t.init == k.init) { t.sch = best_sch; found = true; }
    if (!found) {
        TuneEntry t;
        t.n = X->n; t.d = X->d; t.dtype = X->dtype; t.max_support = X->max_support; t.init = k.init;
        t.sch = best_sch;
        h->tuned.push_back(t);
    }
    if (best_ms) *best_ms = best;
    return D2_OK;
}

}  // extern "C"
