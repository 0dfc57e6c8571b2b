// Host side of the C ABI declared in include/spoly.h: argument checks, the
// context (device buffers it owns) and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "../../include/spoly.h"
#include "onebounce.hpp"
#include "twobounce.hpp"
#include "sqrt_table.inc"
#include "pruner.hpp"
#include "mixed.hpp"
#include "tail.hpp"
#include "order.hpp"

struct spoly_ctx {
    int device;
    float4* tri_cone;      // 2 float4 per triangle, grown on demand
    int64_t tri_cone_cap;  // in triangles
    int2* pairs;           // two-vertex cull: (T1, T2) pairs of one light
    int64_t pairs_cap;
    unsigned long long* pair_count;
    spoly::PrunerWork pw;  // pruner training activations
    void* pw_block;
    int cus;               // compute units of the device
    void* ob_block;        // two-phase one-vertex workspace: counters, items, full list
    int64_t ob_cap;
    void* ob_rblock;       // r(v) of the candidates listed for isolation, list and status
    int64_t ob_rbytes;
    hipEvent_t stage_ev[5];  // timing events of the last one-vertex solve with SPOLY_FLAG_STAGE_TIMES
    int stage_n;             // kernels timed by stage_ev (0: none yet)
    void* ord_block;         // workspace of SPOLY_FLAG_DETERMINISTIC_ORDER, grown on demand
    size_t ord_bytes;
    float* tri_feat;         // pruner scorer: per-triangle feature rows, grown on demand
    int64_t tri_feat_cap;    // in triangles
};

namespace {

bool mesh_ok(const spoly_mesh* m)
{
    return m && m->px && m->py && m->pz && m->nx && m->ny && m->nz && m->tri && m->n_vertices > 0 && m->n_tris > 0;
}
bool pts_ok(const spoly_points* p) { return p && p->x && p->y && p->z && p->n > 0; }

spoly_status dev_err(hipError_t e) { return e == hipSuccess ? SPOLY_OK : SPOLY_E_DEVICE; }

// SPOLY_FLAG_DETERMINISTIC_ORDER: sort the records the solve just wrote (same stream)
spoly_status sort_output(spoly_ctx* ctx, spoly_solution* out, int64_t cap, const unsigned long long* count,
                         hipStream_t s)
{
    if (cap <= 0) return SPOLY_OK;
    const size_t need = spoly::sort_solutions_bytes(cap);
    if (ctx->ord_bytes < need) {
        if (ctx->ord_block) (void)hipFree(ctx->ord_block);
        ctx->ord_block = nullptr;
        ctx->ord_bytes = 0;
        if (hipMalloc(&ctx->ord_block, need) != hipSuccess) return SPOLY_E_DEVICE;
        ctx->ord_bytes = need;
    }
    return dev_err(spoly::sort_solutions(out, cap, count, ctx->ord_block, ctx->ord_bytes, s));
}

}  // namespace

static spoly_status ob_args(const spoly_mesh* mesh, const spoly_points* x0s, const spoly_points* x2s,
                            const int32_t* q_x0, const int32_t* q_x2, const int32_t* q_tri, int64_t n_queries,
                            spoly_event ev, double eta0, double eta1, spoly_precision prec,
                            const spoly_params* params, spoly_solution* out, int64_t out_capacity,
                            unsigned long long* out_count, unsigned long long* counters, int32_t* diag_q,
                            spoly::OneBounceArgs& A);

extern "C" {

void spoly_default_params(spoly_params* p)
{
    if (!p) return;
    p->pieces = 100;
    p->bisect_iters = 10;
    p->iso_eps = 1e-9;
    p->tau = 1e-6;
    p->u_margin = 1e-4;
    p->dedup = 1e-8;
    p->polish_iters = 6;
    p->flags = 0;
}

void spoly_tt_default_params(spoly_params* p)
{
    if (!p) return;
    spoly_default_params(p);
    p->u_margin = 0.05;
}

const char* spoly_status_str(spoly_status s)
{
    switch (s) {
    case SPOLY_OK: return "ok";
    case SPOLY_E_INVALID_ARG: return "invalid argument";
    case SPOLY_E_CAPACITY: return "output capacity exceeded";
    case SPOLY_E_DEVICE: return "device error";
    case SPOLY_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

spoly_status spoly_ctx_create(spoly_ctx** ctx, int device)
{
    if (!ctx) return SPOLY_E_INVALID_ARG;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SPOLY_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly_ctx* c = static_cast<spoly_ctx*>(std::calloc(1, sizeof(spoly_ctx)));
    if (!c) return SPOLY_E_DEVICE;
    c->device = device;
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->cus <= 0)
        c->cus = 256;
    *ctx = c;
    return SPOLY_OK;
}

void spoly_ctx_destroy(spoly_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->tri_cone) (void)hipFree(ctx->tri_cone);
    if (ctx->pairs) (void)hipFree(ctx->pairs);
    if (ctx->pair_count) (void)hipFree(ctx->pair_count);
    if (ctx->pw_block) (void)hipFree(ctx->pw_block);
    if (ctx->ob_block) (void)hipFree(ctx->ob_block);
    if (ctx->ob_rblock) (void)hipFree(ctx->ob_rblock);
    if (ctx->ord_block) (void)hipFree(ctx->ord_block);
    if (ctx->tri_feat) (void)hipFree(ctx->tri_feat);
    if (ctx->stage_ev[0])
        for (int i = 0; i < 5; ++i) (void)hipEventDestroy(ctx->stage_ev[i]);
    std::free(ctx);
}

int32_t spoly_stage_times(spoly_ctx* ctx, float* ms, int32_t cap)
{
    if (!ctx || (cap > 0 && !ms) || cap < 0) return -1;
    if (ctx->stage_n == 0) return 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return -1;
    if (hipEventSynchronize(ctx->stage_ev[ctx->stage_n]) != hipSuccess) return -1;
    int32_t n = ctx->stage_n < cap ? ctx->stage_n : cap;
    for (int32_t i = 0; i < n; ++i)
        if (hipEventElapsedTime(&ms[i], ctx->stage_ev[i], ctx->stage_ev[i + 1]) != hipSuccess) return -1;
    return n;
}

// Item list between the two phases of the one-vertex solve, and for
// refraction the per-candidate r(v) between its coefficient and isolation
// kernels (grown on demand; growing synchronises the device through
// hipFree/hipMalloc).
static spoly_status grow(void** block, int64_t* cap, int64_t need, size_t per, size_t head)
{
    if (*cap >= need) return SPOLY_OK;
    if (*block) (void)hipFree(*block);
    *block = nullptr;
    *cap = 0;
    if (hipMalloc(block, size_t(need) * per + head) != hipSuccess) {
        *block = nullptr;
        return SPOLY_E_DEVICE;
    }
    *cap = need;
    return SPOLY_OK;
}

// Item list of the two-phase one-vertex solve for `cap` candidates at p:
// [256 B counters | items_v: kObEmit doubles | items_q, items_n, full_q: int32] per candidate
constexpr size_t kObItemBytes = 8 * spoly::kObEmit + 12;
constexpr size_t kObHeadBytes = 256;
static void carve_ob_items(char* p, int64_t cap, spoly::OneBounceArgs& A)
{
    A.items_count = reinterpret_cast<unsigned long long*>(p);
    A.items_v = reinterpret_cast<double*>(p + kObHeadBytes);
    A.items_q = reinterpret_cast<int32_t*>(p + kObHeadBytes + size_t(cap) * 8 * spoly::kObEmit);
    A.items_n = A.items_q + cap;
    A.full_q = A.items_n + cap;
    A.items_cap = cap;
}
// r(v) list of the refraction front for `cap` candidates at p:
// [r(v): coef_bytes | iso_q, iso_st: int32] per candidate
static void carve_ob_rlist(char* p, int64_t cap, size_t coef_bytes, spoly::OneBounceArgs& A)
{
    A.rlist = p;
    A.iso_q = reinterpret_cast<int32_t*>(p + coef_bytes * size_t(cap));
    A.iso_st = A.iso_q + cap;
}

static spoly_status ensure_ob_items(spoly_ctx* ctx, int64_t need, size_t coef_bytes, spoly::OneBounceArgs& A)
{
    spoly_status st = grow(&ctx->ob_block, &ctx->ob_cap, need, kObItemBytes, kObHeadBytes);
    if (st != SPOLY_OK) return st;
    carve_ob_items(static_cast<char*>(ctx->ob_block), ctx->ob_cap, A);
    // [r(v) of listed candidates: coef_bytes | iso_q, iso_st: int32] per candidate, same capacity
    A.rlist = nullptr;
    A.iso_q = nullptr;
    A.iso_st = nullptr;
    if (coef_bytes == 0) return SPOLY_OK;
    const int64_t per = int64_t(coef_bytes) + 8;
    if (ctx->ob_rbytes < per * ctx->ob_cap) {
        if (ctx->ob_rblock) (void)hipFree(ctx->ob_rblock);
        ctx->ob_rblock = nullptr;
        ctx->ob_rbytes = 0;
        if (hipMalloc(&ctx->ob_rblock, size_t(per) * size_t(ctx->ob_cap)) != hipSuccess) {
            ctx->ob_rblock = nullptr;
            return SPOLY_E_DEVICE;
        }
        ctx->ob_rbytes = per * ctx->ob_cap;
    }
    carve_ob_rlist(static_cast<char*>(ctx->ob_rblock), ctx->ob_cap, coef_bytes, A);
    return SPOLY_OK;
}

static spoly_status ensure_cones(spoly_ctx* ctx, const spoly_mesh* mesh, hipStream_t s)
{
    if (ctx->tri_cone_cap < mesh->n_tris) {
        if (ctx->tri_cone) (void)hipFree(ctx->tri_cone);
        ctx->tri_cone = nullptr;
        ctx->tri_cone_cap = 0;
        if (hipMalloc(&ctx->tri_cone, sizeof(float4) * 2 * size_t(mesh->n_tris)) != hipSuccess) return SPOLY_E_DEVICE;
        ctx->tri_cone_cap = mesh->n_tris;
    }
    return dev_err(spoly::launch_tri_cones(mesh->px, mesh->py, mesh->pz, mesh->nx, mesh->ny, mesh->nz, mesh->tri,
                                           mesh->n_tris, ctx->tri_cone, s));
}

spoly_status spoly_cull_1bounce(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_points* x0s,
                                const spoly_points* x2s, double eta0, double eta1, double margin, int32_t* out_x0,
                                int32_t* out_x2, int32_t* out_tri, int64_t out_capacity,
                                unsigned long long* out_count, void* stream)
{
    if (!ctx || !mesh_ok(mesh) || !pts_ok(x0s) || !pts_ok(x2s) || !out_count || out_capacity < 0) return SPOLY_E_INVALID_ARG;
    if (out_capacity > 0 && (!out_x0 || !out_x2 || !out_tri)) return SPOLY_E_INVALID_ARG;
    if (!(eta0 > 0.0) || !(eta1 > 0.0) || !(margin >= 0.0)) return SPOLY_E_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly_status st = ensure_cones(ctx, mesh, s);
    if (st != SPOLY_OK) return st;
    spoly::CullArgs A;
    A.tri_cone = ctx->tri_cone;
    A.n_tris = mesh->n_tris;
    A.x0x = x0s->x; A.x0y = x0s->y; A.x0z = x0s->z;
    A.x2x = x2s->x; A.x2y = x2s->y; A.x2z = x2s->z;
    A.n0 = x0s->n; A.n2 = x2s->n;
    A.eta0 = float(eta0); A.eta1 = float(eta1); A.margin = float(margin);
    A.out_x0 = out_x0; A.out_x2 = out_x2; A.out_tri = out_tri;
    A.cap = out_capacity;
    A.out_count = out_count;
    return dev_err(spoly::launch_cull_1bounce(A, s));
}

spoly_status spoly_solve_1bounce(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_points* x0s,
                                 const spoly_points* x2s, const int32_t* q_x0, const int32_t* q_x2,
                                 const int32_t* q_tri, int64_t n_queries, spoly_event ev, double eta0, double eta1,
                                 spoly_precision prec, const spoly_params* params, spoly_solution* out,
                                 int64_t out_capacity, unsigned long long* out_count, unsigned long long* counters,
                                 int32_t* diag_q, void* stream)
{
    if (!ctx) return SPOLY_E_INVALID_ARG;
    spoly::OneBounceArgs A;
    spoly_status st = ob_args(mesh, x0s, x2s, q_x0, q_x2, q_tri, n_queries, ev, eta0, eta1, prec, params, out,
                              out_capacity, out_count, counters, diag_q, A);
    if (st != SPOLY_OK) return st;
    if (params->flags & SPOLY_FLAG_FORCE_FP64) prec = SPOLY_FP64;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    // the refraction front lists r(v) (13 doubles) of candidates between its two kernels
    const size_t coef_bytes = ev == SPOLY_T ? 13 * 8 : 0;
    st = ensure_ob_items(ctx, n_queries, coef_bytes, A);
    if (st != SPOLY_OK) return st;
    hipEvent_t* evs = nullptr;
    if (params->flags & SPOLY_FLAG_STAGE_TIMES) {
        if (!ctx->stage_ev[0])
            for (int i = 0; i < 5; ++i)
                if (hipEventCreate(&ctx->stage_ev[i]) != hipSuccess) return SPOLY_E_DEVICE;
        evs = ctx->stage_ev;
        ctx->stage_n = n_queries > 0 ? (ev == SPOLY_T ? 4 : 3) : 0;
    }
    st = dev_err(spoly::launch_onebounce_2phase(A, int(ev), int(prec), ctx->cus * 4,
                                                static_cast<hipStream_t>(stream), evs));
    if (st != SPOLY_OK || !(params->flags & SPOLY_FLAG_DETERMINISTIC_ORDER)) return st;
    return sort_output(ctx, out, out_capacity, out_count, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Argument checks and kernel arguments shared by the one-vertex entry points
// (the workspace pointers are filled by the caller).
static spoly_status ob_args(const spoly_mesh* mesh, const spoly_points* x0s, const spoly_points* x2s,
                            const int32_t* q_x0, const int32_t* q_x2, const int32_t* q_tri, int64_t n_queries,
                            spoly_event ev, double eta0, double eta1, spoly_precision prec,
                            const spoly_params* params, spoly_solution* out, int64_t out_capacity,
                            unsigned long long* out_count, unsigned long long* counters, int32_t* diag_q,
                            spoly::OneBounceArgs& A)
{
    if (!mesh_ok(mesh) || !pts_ok(x0s) || !pts_ok(x2s) || !params || !out_count) return SPOLY_E_INVALID_ARG;
    if (n_queries < 0 || out_capacity < 0 || (out_capacity > 0 && !out)) return SPOLY_E_INVALID_ARG;
    if (n_queries > 0 && (!q_x0 || !q_x2 || !q_tri)) return SPOLY_E_INVALID_ARG;
    if (ev != SPOLY_R && ev != SPOLY_T) return SPOLY_E_INVALID_ARG;
    if (prec != SPOLY_FP64 && prec != SPOLY_FP32_POLISH64) return SPOLY_E_INVALID_ARG;
    if (!(eta0 > 0.0) || !(eta1 > 0.0)) return SPOLY_E_INVALID_ARG;
    if (!(params->tau > 0.0) || !(params->iso_eps > 0.0) || params->polish_iters < 0 || !(params->u_margin >= 0.0) ||
        !(params->dedup >= 0.0))
        return SPOLY_E_INVALID_ARG;
    if (params->flags & ~(SPOLY_FLAG_FORCE_FP64 | SPOLY_FLAG_STAGE_TIMES | SPOLY_FLAG_DETERMINISTIC_ORDER))
        return SPOLY_E_INVALID_ARG;
    if (params->flags & SPOLY_FLAG_FORCE_FP64) prec = SPOLY_FP64;
    A.px = mesh->px; A.py = mesh->py; A.pz = mesh->pz;
    A.nx = mesh->nx; A.ny = mesh->ny; A.nz = mesh->nz;
    A.tri = mesh->tri;
    A.x0x = x0s->x; A.x0y = x0s->y; A.x0z = x0s->z;
    A.x2x = x2s->x; A.x2y = x2s->y; A.x2z = x2s->z;
    A.q_x0 = q_x0; A.q_x2 = q_x2; A.q_tri = q_tri;
    A.nq = n_queries;
    A.eta0 = eta0; A.eta1 = eta1;
    A.iso_eps = params->iso_eps; A.tau = params->tau; A.u_margin = params->u_margin; A.dedup = params->dedup;
    A.polish_iters = params->polish_iters;
    A.out = out; A.cap = out_capacity; A.out_count = out_count;
    A.counters = counters; A.diag_q = diag_q;
    A.refine_v = (ev == SPOLY_R && prec == SPOLY_FP32_POLISH64) ? 1 : 0;
    return SPOLY_OK;
}

// ---------------------------------------------------------------- no-allocation variant
// The two-phase workspace of spoly_solve_1bounce_noalloc lives in this
// file-scope device array; each device holds its own copy until the process
// ends.  Host code never uses the array's name as an address: its device
// address is looked up per device (hipGetSymbolAddress, with that device
// current) on the first call on that device and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[SPOLY_NOALLOC_SCRATCH_BYTES];
static_assert(kObHeadBytes + kObItemBytes * size_t(SPOLY_NOALLOC_MAX_QUERIES_R) <= SPOLY_NOALLOC_SCRATCH_BYTES,
              "reflection workspace exceeds the scratch array");
static_assert((kObHeadBytes + kObItemBytes * size_t(SPOLY_NOALLOC_MAX_QUERIES_T) + 255) / 256 * 256 +
                      (13 * 8 + 8) * size_t(SPOLY_NOALLOC_MAX_QUERIES_T) <= SPOLY_NOALLOC_SCRATCH_BYTES,
              "refraction workspace exceeds the scratch array");

namespace {
constexpr int kMaxDevices = 64;
struct ScratchSlot {
    void* ptr;
    int cus;
};
ScratchSlot g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

spoly_status scratch_for_current_device(ScratchSlot& slot)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPOLY_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot& s = g_scratch[dev];
    if (!s.ptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPOLY_E_DEVICE;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        s.cus = cus;
        s.ptr = p;
    }
    slot = s;
    return SPOLY_OK;
}
}  // namespace

extern "C" {

spoly_status spoly_solve_1bounce_noalloc(const spoly_mesh* mesh, const spoly_points* x0s, const spoly_points* x2s,
                                         const int32_t* q_x0, const int32_t* q_x2, const int32_t* q_tri,
                                         int64_t n_queries, spoly_event ev, double eta0, double eta1,
                                         spoly_precision prec, const spoly_params* params, spoly_solution* out,
                                         int64_t out_capacity, unsigned long long* out_count,
                                         unsigned long long* counters, int32_t* diag_q, void* stream)
{
    spoly::OneBounceArgs A;
    spoly_status st = ob_args(mesh, x0s, x2s, q_x0, q_x2, q_tri, n_queries, ev, eta0, eta1, prec, params, out,
                              out_capacity, out_count, counters, diag_q, A);
    if (st != SPOLY_OK) return st;
    // the sort needs a workspace sized by the output capacity
    if (params->flags & SPOLY_FLAG_DETERMINISTIC_ORDER) return SPOLY_E_UNSUPPORTED;
    if (params->flags & SPOLY_FLAG_FORCE_FP64) prec = SPOLY_FP64;
    const int64_t max_q = ev == SPOLY_T ? SPOLY_NOALLOC_MAX_QUERIES_T : SPOLY_NOALLOC_MAX_QUERIES_R;
    if (n_queries > max_q) return SPOLY_E_CAPACITY;
    ScratchSlot slot;
    st = scratch_for_current_device(slot);
    if (st != SPOLY_OK) return st;
    // [items for max_q candidates | refraction r(v) list for max_q candidates]; the layout uses the
    // largest query count of the event, so its size does not depend on n_queries
    const size_t coef_bytes = ev == SPOLY_T ? 13 * 8 : 0;
    char* base = static_cast<char*>(slot.ptr);
    carve_ob_items(base, max_q, A);
    A.rlist = nullptr;
    A.iso_q = nullptr;
    A.iso_st = nullptr;
    if (coef_bytes) {
        const size_t items = kObHeadBytes + kObItemBytes * size_t(max_q);
        const size_t off = (items + 255) / 256 * 256;
        carve_ob_rlist(base + off, max_q, coef_bytes, A);
    }
    return dev_err(spoly::launch_onebounce_2phase(A, int(ev), int(prec), slot.cus * 4,
                                                  static_cast<hipStream_t>(stream)));
}

}  // extern "C"

extern "C" {

spoly_status spoly_cull_2bounce(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_points* x0s,
                                const spoly_points* x3s, const double* eta, double margin, int32_t* out_x0,
                                int32_t* out_x3, int32_t* out_t1, int32_t* out_t2, int64_t out_capacity,
                                unsigned long long* out_count, void* stream)
{
    if (!ctx || !mesh_ok(mesh) || !pts_ok(x0s) || !pts_ok(x3s) || !eta || !out_count || out_capacity < 0)
        return SPOLY_E_INVALID_ARG;
    if (out_capacity > 0 && (!out_x0 || !out_x3 || !out_t1 || !out_t2)) return SPOLY_E_INVALID_ARG;
    if (!(eta[0] > 0.0) || !(eta[1] > 0.0) || !(eta[2] > 0.0) || !(margin >= 0.0)) return SPOLY_E_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly_status st = ensure_cones(ctx, mesh, s);
    if (st != SPOLY_OK) return st;
    const int64_t npair = int64_t(mesh->n_tris) * mesh->n_tris;
    if (ctx->pairs_cap < npair) {
        if (ctx->pairs) (void)hipFree(ctx->pairs);
        ctx->pairs = nullptr;
        ctx->pairs_cap = 0;
        if (hipMalloc(&ctx->pairs, sizeof(int2) * size_t(npair)) != hipSuccess) return SPOLY_E_DEVICE;
        ctx->pairs_cap = npair;
    }
    if (!ctx->pair_count && hipMalloc(&ctx->pair_count, sizeof(unsigned long long)) != hipSuccess)
        return SPOLY_E_DEVICE;
    spoly::CullTTArgs A;
    A.tri_cone = ctx->tri_cone;
    A.n_tris = mesh->n_tris;
    A.x0x = x0s->x; A.x0y = x0s->y; A.x0z = x0s->z;
    A.x3x = x3s->x; A.x3y = x3s->y; A.x3z = x3s->z;
    A.n0 = x0s->n; A.n3 = x3s->n;
    A.eta0 = float(eta[0]); A.eta1 = float(eta[1]); A.eta2 = float(eta[2]); A.margin = float(margin);
    A.pairs = ctx->pairs; A.pair_cap = ctx->pairs_cap; A.pair_count = ctx->pair_count;
    A.out_x0 = out_x0; A.out_x3 = out_x3; A.out_t1 = out_t1; A.out_t2 = out_t2;
    A.cap = out_capacity; A.out_count = out_count;
    for (int j3 = 0; j3 < x3s->n; ++j3) {
        if (spoly::launch_zero_u64(ctx->pair_count, s) != hipSuccess) return SPOLY_E_DEVICE;
        if (spoly::launch_tt_pairs(A, j3, s) != hipSuccess) return SPOLY_E_DEVICE;
        unsigned long long np = 0;
        if (hipMemcpyAsync(&np, ctx->pair_count, sizeof(np), hipMemcpyDeviceToHost, s) != hipSuccess) return SPOLY_E_DEVICE;
        if (hipStreamSynchronize(s) != hipSuccess) return SPOLY_E_DEVICE;
        if (np > (unsigned long long)ctx->pairs_cap) np = (unsigned long long)ctx->pairs_cap;
        if (spoly::launch_tt_cull(A, j3, int64_t(np), s) != hipSuccess) return SPOLY_E_DEVICE;
    }
    return SPOLY_OK;
}

spoly_status spoly_solve_nbounce(spoly_ctx* ctx, const spoly_mesh* mesh, int32_t k, const spoly_event* chain,
                                 const double* eta, const spoly_points* x0s, const spoly_points* x3s,
                                 const int32_t* q_x0, const int32_t* q_x3, const int32_t* q_tris, int64_t n_queries,
                                 spoly_precision prec, const spoly_params* params, const double* sqrt_table,
                                 spoly_solution* out, int64_t out_capacity, unsigned long long* out_count,
                                 unsigned long long* counters, int32_t* diag_q, void* stream)
{
    if (!ctx || !mesh_ok(mesh) || !pts_ok(x0s) || !pts_ok(x3s) || !params || !out_count || !chain || !eta)
        return SPOLY_E_INVALID_ARG;
    if (n_queries < 0 || out_capacity < 0 || (out_capacity > 0 && !out)) return SPOLY_E_INVALID_ARG;
    if (n_queries > 0 && (!q_x0 || !q_x3 || !q_tris)) return SPOLY_E_INVALID_ARG;
    if (k != 2) return SPOLY_E_UNSUPPORTED;
    for (int i = 0; i < 2; ++i)
        if (chain[i] != SPOLY_R && chain[i] != SPOLY_T) return SPOLY_E_INVALID_ARG;
    if (prec != SPOLY_FP64) return SPOLY_E_UNSUPPORTED;
    if (!(eta[0] > 0.0) || !(eta[1] > 0.0) || !(eta[2] > 0.0)) return SPOLY_E_INVALID_ARG;
    // a reflection keeps its medium: equal IORs on its two segments
    for (int i = 0; i < 2; ++i)
        if (chain[i] == SPOLY_R && eta[i] != eta[i + 1]) return SPOLY_E_INVALID_ARG;
    if (params->flags & ~(SPOLY_FLAG_FORCE_FP64 | SPOLY_FLAG_DETERMINISTIC_ORDER)) return SPOLY_E_INVALID_ARG;
    if (params->pieces < 1 || params->pieces > spoly::kMaxPieces || params->bisect_iters < 0 ||
        params->bisect_iters > spoly::kMaxBisect ||
        params->polish_iters < 0 ||
        !(params->tau > 0.0) || !(params->u_margin >= 0.0) || !(params->dedup >= 0.0))
        return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly::TTArgs A;
    A.px = mesh->px; A.py = mesh->py; A.pz = mesh->pz;
    A.nx = mesh->nx; A.ny = mesh->ny; A.nz = mesh->nz;
    A.tri = mesh->tri;
    A.x0x = x0s->x; A.x0y = x0s->y; A.x0z = x0s->z;
    A.x3x = x3s->x; A.x3y = x3s->y; A.x3z = x3s->z;
    A.q_x0 = q_x0; A.q_x3 = q_x3; A.q_tris = q_tris;
    A.nq = n_queries;
    A.ev1 = chain[0]; A.ev2 = chain[1];
    A.eta0 = eta[0]; A.eta1 = eta[1]; A.eta2 = eta[2];
    const double* tb = sqrt_table ? sqrt_table : nullptr;
    for (int i = 0; i < 7; ++i) A.sqrt_bp[i] = tb ? tb[i] : kSqrtPieceEnds[i];
    for (int i = 0; i < 24; ++i) A.sqrt_c[i] = tb ? tb[7 + i] : kSqrtCoef[i];
    A.pieces = params->pieces; A.bisect_iters = params->bisect_iters; A.polish_iters = params->polish_iters;
    A.tau = params->tau; A.u_margin = params->u_margin; A.dedup = params->dedup;
    A.out = out; A.cap = out_capacity; A.out_count = out_count;
    A.counters = counters; A.diag_q = diag_q;
    spoly_status st = dev_err(spoly::launch_tt_solve(A, static_cast<hipStream_t>(stream)));
    if (st != SPOLY_OK || !(params->flags & SPOLY_FLAG_DETERMINISTIC_ORDER)) return st;
    return sort_output(ctx, out, out_capacity, out_count, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

bool fill_io(spoly::PrunerIO& io, const spoly_mesh* mesh, const spoly_points* x0s, const spoly_points* x3s,
             const int32_t* q_x0, const int32_t* q_x3, const int32_t* q_tris, int64_t n)
{
    if (!mesh_ok(mesh) || !pts_ok(x0s) || !pts_ok(x3s) || n < 0) return false;
    if (n > 0 && (!q_x0 || !q_x3 || !q_tris)) return false;
    io.px = mesh->px; io.py = mesh->py; io.pz = mesh->pz;
    io.nx = mesh->nx; io.ny = mesh->ny; io.nz = mesh->nz;
    io.tri = mesh->tri;
    io.x0x = x0s->x; io.x0y = x0s->y; io.x0z = x0s->z;
    io.x3x = x3s->x; io.x3y = x3s->y; io.x3z = x3s->z;
    io.q_x0 = q_x0; io.q_x3 = q_x3; io.q_tris = q_tris;
    io.n = n;
    return true;
}

spoly_status ensure_pruner_work(spoly_ctx* ctx, int64_t n)
{
    if (ctx->pw_block && ctx->pw.cap >= n) return SPOLY_OK;
    if (ctx->pw_block) (void)hipFree(ctx->pw_block);
    ctx->pw_block = nullptr;
    const int64_t cap = n < 1024 ? 1024 : n;
    const size_t bf = 2, f4 = 4;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~size_t(255); return o; };
    size_t oX = take(cap * spoly::kFeat * bf), oPb = take(size_t(spoly::kNParams) * bf);
    size_t oH1 = take(cap * spoly::kHid * bf), oH2 = take(cap * spoly::kHid * bf), oH3 = take(cap * spoly::kHid * bf);
    size_t odZ4 = take(cap * 16 * bf), odZ = take(cap * spoly::kHid * bf);
    size_t oZ1 = take(cap * spoly::kHid * f4), oZ2 = take(cap * spoly::kHid * f4), oZ3 = take(cap * spoly::kHid * f4);
    size_t oZ4 = take(cap * 16 * f4), odH = take(cap * spoly::kHid * f4);
    size_t opart = take(size_t(spoly::kGemmSplitMax) * spoly::kHid * spoly::kHid * f4);
    if (hipMalloc(&ctx->pw_block, off) != hipSuccess) { ctx->pw_block = nullptr; return SPOLY_E_DEVICE; }
    char* b = static_cast<char*>(ctx->pw_block);
    spoly::PrunerWork& W = ctx->pw;
    W.cap = cap;
    W.X = (unsigned short*)(b + oX); W.Pb = (unsigned short*)(b + oPb);
    W.H1 = (unsigned short*)(b + oH1); W.H2 = (unsigned short*)(b + oH2); W.H3 = (unsigned short*)(b + oH3);
    W.dZ4 = (unsigned short*)(b + odZ4); W.dZ = (unsigned short*)(b + odZ);
    W.Z1 = (float*)(b + oZ1); W.Z2 = (float*)(b + oZ2); W.Z3 = (float*)(b + oZ3); W.Z4 = (float*)(b + oZ4);
    W.dH = (float*)(b + odH);
    W.part = (float*)(b + opart);
    return SPOLY_OK;
}

}  // namespace

extern "C" {

spoly_status spoly_prune_score(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_points* x0s,
                               const spoly_points* x3s, const int32_t* q_x0, const int32_t* q_x3,
                               const int32_t* q_tris, int64_t n, const float* params, float threshold, float* scores,
                               int32_t* keep_idx, int64_t keep_capacity, unsigned long long* keep_count, void* stream)
{
    spoly::PrunerIO io;
    if (!ctx || !params || !keep_count || keep_capacity < 0 || (keep_capacity > 0 && !keep_idx)) return SPOLY_E_INVALID_ARG;
    if (!fill_io(io, mesh, x0s, x3s, q_x0, q_x3, q_tris, n)) return SPOLY_E_INVALID_ARG;
    if (!(threshold >= 0.0f) || !(threshold <= 1.0f)) return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    if (ctx->tri_feat_cap < mesh->n_tris) {
        if (ctx->tri_feat) (void)hipFree(ctx->tri_feat);
        ctx->tri_feat = nullptr;
        ctx->tri_feat_cap = 0;
        if (hipMalloc(&ctx->tri_feat, sizeof(float) * spoly::kTriFeat * size_t(mesh->n_tris)) != hipSuccess)
            return SPOLY_E_DEVICE;
        ctx->tri_feat_cap = mesh->n_tris;
    }
    return dev_err(spoly::launch_prune_score(io, params, threshold, scores, keep_idx, keep_capacity, keep_count,
                                             ctx->tri_feat, mesh->n_tris, static_cast<hipStream_t>(stream)));
}

spoly_status spoly_pruner_fwd_bwd(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_points* x0s,
                                  const spoly_points* x3s, const int32_t* q_x0, const int32_t* q_x3,
                                  const int32_t* q_tris, int64_t n, const float* labels, float pos_weight,
                                  const float* params, float* grads, float* loss, void* stream)
{
    spoly::PrunerIO io;
    if (!ctx || !labels || !params || !grads || !loss || n <= 0 || n > 65536) return SPOLY_E_INVALID_ARG;
    if (!fill_io(io, mesh, x0s, x3s, q_x0, q_x3, q_tris, n)) return SPOLY_E_INVALID_ARG;
    if (!(pos_weight > 0.0f)) return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly_status st = ensure_pruner_work(ctx, n);
    if (st != SPOLY_OK) return st;
    return dev_err(spoly::pruner_fwd_bwd(io, labels, pos_weight, params, grads, loss, ctx->pw,
                                         static_cast<hipStream_t>(stream)));
}

spoly_status spoly_pruner_step(spoly_ctx* ctx, float* params, const float* grads, float* adam_m, float* adam_v,
                               int64_t step, float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!ctx || !params || !grads || !adam_m || !adam_v || step < 1) return SPOLY_E_INVALID_ARG;
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    return dev_err(spoly::pruner_adam(params, grads, adam_m, adam_v, step, lr, beta1, beta2, eps,
                                      static_cast<hipStream_t>(stream)));
}

spoly_status spoly_pruner_features(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_points* x0s,
                                   const spoly_points* x3s, const int32_t* q_x0, const int32_t* q_x3,
                                   const int32_t* q_tris, int64_t n, float* features, void* stream)
{
    spoly::PrunerIO io;
    if (!ctx || !features) return SPOLY_E_INVALID_ARG;
    if (!fill_io(io, mesh, x0s, x3s, q_x0, q_x3, q_tris, n)) return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly_status st = ensure_pruner_work(ctx, n);
    if (st != SPOLY_OK) return st;
    return dev_err(spoly::launch_gather(io, ctx->pw.X, features, static_cast<hipStream_t>(stream)));
}

}  // extern "C"

extern "C" spoly_status spoly_solve_mixed(spoly_ctx* ctx, const spoly_mesh* mesh1, const spoly_points* x0s1,
                                         const spoly_points* x2s1, const int32_t* q1_x0, const int32_t* q1_x2,
                                         const int32_t* q1_tri, int64_t n1, spoly_event ev1, double eta0,
                                         double eta1, const spoly_mesh* mesh2, const spoly_points* x0s2,
                                         const spoly_points* x3s2, const int32_t* q2_x0, const int32_t* q2_x3,
                                         const int32_t* q2_tris, int64_t n2, const double* eta2,
                                         spoly_precision prec, const spoly_params* params,
                                         const spoly_mixed_shape* shape, unsigned long long* queue,
                                         spoly_solution* out, int64_t out_capacity, unsigned long long* out_count,
                                         void* stream)
{
    if (!ctx || !params || !shape || !queue || !out_count || !eta2) return SPOLY_E_INVALID_ARG;
    if (!mesh_ok(mesh1) || !pts_ok(x0s1) || !pts_ok(x2s1) || !mesh_ok(mesh2) || !pts_ok(x0s2) || !pts_ok(x3s2))
        return SPOLY_E_INVALID_ARG;
    if (n1 < 0 || n2 < 0 || out_capacity < 0 || (out_capacity > 0 && !out)) return SPOLY_E_INVALID_ARG;
    if ((n1 > 0 && (!q1_x0 || !q1_x2 || !q1_tri)) || (n2 > 0 && (!q2_x0 || !q2_x3 || !q2_tris)))
        return SPOLY_E_INVALID_ARG;
    if (ev1 != SPOLY_R && ev1 != SPOLY_T) return SPOLY_E_INVALID_ARG;
    if (prec != SPOLY_FP64 && prec != SPOLY_FP32_POLISH64) return SPOLY_E_INVALID_ARG;
    if (!(eta0 > 0.0) || !(eta1 > 0.0) || !(eta2[0] > 0.0) || !(eta2[1] > 0.0) || !(eta2[2] > 0.0))
        return SPOLY_E_INVALID_ARG;
    if (shape->workgroups_per_cu < 1 || shape->workgroups_per_cu > 32 || shape->r_tile < 64 ||
        shape->r_tile > 4096 || (shape->r_tile % 64) != 0 || shape->order < 0 || shape->order > 2)
        return SPOLY_E_INVALID_ARG;
    if (params->flags & SPOLY_FLAG_DETERMINISTIC_ORDER) return SPOLY_E_UNSUPPORTED;
    if (params->flags & ~SPOLY_FLAG_FORCE_FP64) return SPOLY_E_INVALID_ARG;
    if (params->flags & SPOLY_FLAG_FORCE_FP64) prec = SPOLY_FP64;
    if (params->pieces < 1 || params->pieces > spoly::kMaxPieces || params->bisect_iters < 0 ||
        params->bisect_iters > spoly::kMaxBisect ||
        params->polish_iters < 0 || !(params->tau > 0.0) || !(params->iso_eps > 0.0) || !(params->u_margin >= 0.0) ||
        !(params->dedup >= 0.0))
        return SPOLY_E_INVALID_ARG;
    if (n1 + n2 > 2147483647LL) return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        return SPOLY_E_DEVICE;
    spoly::MixedArgs M;
    spoly::OneBounceArgs& A = M.r;
    A.px = mesh1->px; A.py = mesh1->py; A.pz = mesh1->pz;
    A.nx = mesh1->nx; A.ny = mesh1->ny; A.nz = mesh1->nz;
    A.tri = mesh1->tri;
    A.x0x = x0s1->x; A.x0y = x0s1->y; A.x0z = x0s1->z;
    A.x2x = x2s1->x; A.x2y = x2s1->y; A.x2z = x2s1->z;
    A.q_x0 = q1_x0; A.q_x2 = q1_x2; A.q_tri = q1_tri;
    A.nq = n1;
    A.eta0 = eta0; A.eta1 = eta1;
    A.iso_eps = params->iso_eps; A.tau = params->tau; A.u_margin = params->u_margin; A.dedup = params->dedup;
    A.polish_iters = params->polish_iters;
    A.refine_v = (ev1 == SPOLY_R && prec == SPOLY_FP32_POLISH64) ? 1 : 0;
    A.out = out; A.cap = out_capacity; A.out_count = out_count;
    A.counters = nullptr; A.diag_q = nullptr;
    A.items_q = nullptr; A.items_n = nullptr; A.items_v = nullptr; A.full_q = nullptr; A.items_cap = 0;
    A.rlist = nullptr; A.iso_q = nullptr; A.iso_st = nullptr;
    A.items_count = nullptr;
    spoly::TTArgs& T = M.t;
    T.px = mesh2->px; T.py = mesh2->py; T.pz = mesh2->pz;
    T.nx = mesh2->nx; T.ny = mesh2->ny; T.nz = mesh2->nz;
    T.tri = mesh2->tri;
    T.x0x = x0s2->x; T.x0y = x0s2->y; T.x0z = x0s2->z;
    T.x3x = x3s2->x; T.x3y = x3s2->y; T.x3z = x3s2->z;
    T.q_x0 = q2_x0; T.q_x3 = q2_x3; T.q_tris = q2_tris;
    T.nq = n2;
    T.ev1 = SPOLY_T; T.ev2 = SPOLY_T;
    T.eta0 = eta2[0]; T.eta1 = eta2[1]; T.eta2 = eta2[2];
    for (int i = 0; i < 7; ++i) T.sqrt_bp[i] = kSqrtPieceEnds[i];
    for (int i = 0; i < 24; ++i) T.sqrt_c[i] = kSqrtCoef[i];
    T.pieces = params->pieces; T.bisect_iters = params->bisect_iters; T.polish_iters = params->polish_iters;
    T.tau = params->tau; T.u_margin = 0.05; T.dedup = params->dedup;
    T.out = out; T.cap = out_capacity; T.out_count = out_count;
    T.counters = nullptr; T.diag_q = nullptr;
    M.r_tile = shape->r_tile;
    M.order = shape->order;
    M.n_r_tiles = (n1 + shape->r_tile - 1) / shape->r_tile;
    M.n_items = M.n_r_tiles + n2;
    M.queue = queue;
    return dev_err(spoly::launch_mixed(M, int(ev1), int(prec), cus * shape->workgroups_per_cu,
                                       static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ path-phase tail

struct spoly_bvh {
    int device;
    spoly::BvhStore store;
};

extern "C" {

spoly_status spoly_bvh_build(spoly_ctx* ctx, const spoly_mesh* mesh, spoly_bvh** out, void* stream)
{
    if (!ctx || !mesh_ok(mesh) || !out) return SPOLY_E_INVALID_ARG;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly_bvh* b = static_cast<spoly_bvh*>(std::calloc(1, sizeof(spoly_bvh)));
    if (!b) return SPOLY_E_DEVICE;
    b->device = ctx->device;
    if (spoly::bvh_build(mesh->px, mesh->py, mesh->pz, mesh->tri, mesh->n_tris, &b->store,
                         static_cast<hipStream_t>(stream)) != hipSuccess) {
        std::free(b);
        return SPOLY_E_DEVICE;
    }
    *out = b;
    return SPOLY_OK;
}

void spoly_bvh_destroy(spoly_bvh* bvh)
{
    if (!bvh) return;
    (void)hipSetDevice(bvh->device);
    spoly::bvh_free(&bvh->store);
    std::free(bvh);
}

void spoly_tail_default_params(spoly_tail_params* p)
{
    if (!p) return;
    p->intensity = 1.0;
    p->reflectance = 1.0;
    p->t_eps = 1e-6;
    p->rcv_normal[0] = p->rcv_normal[1] = p->rcv_normal[2] = 0.0;
}

spoly_status spoly_path_tail(spoly_ctx* ctx, const spoly_mesh* mesh, const spoly_bvh* bvh, int32_t k,
                             const spoly_event* chain, const double* eta, const spoly_points* x0s,
                             const spoly_points* xls, const int32_t* q_x0, const int32_t* q_xl,
                             const spoly_solution* sols, int64_t n_sols, const unsigned long long* sol_count,
                             const spoly_tail_params* params, int32_t* mask, double* contrib, double* image,
                             void* stream)
{
    if (!ctx || !mesh_ok(mesh) || !bvh || !chain || !eta || !pts_ok(x0s) || !pts_ok(xls) || !params)
        return SPOLY_E_INVALID_ARG;
    if (k < 1 || k > 2) return SPOLY_E_UNSUPPORTED;
    if (bvh->device != ctx->device || bvh->store.n_tris != mesh->n_tris) return SPOLY_E_INVALID_ARG;
    if (n_sols < 0 || (n_sols > 0 && (!sols || !q_x0 || !q_xl))) return SPOLY_E_INVALID_ARG;
    for (int i = 0; i < k; ++i) {
        if (chain[i] != SPOLY_R && chain[i] != SPOLY_T) return SPOLY_E_INVALID_ARG;
        if (chain[i] == SPOLY_R && eta[i] != eta[i + 1]) return SPOLY_E_INVALID_ARG;
    }
    for (int i = 0; i <= k; ++i)
        if (!(eta[i] > 0.0)) return SPOLY_E_INVALID_ARG;
    if (!(params->intensity >= 0.0) || !(params->reflectance >= 0.0) || !(params->t_eps >= 0.0) ||
        !(params->t_eps < 0.5))
        return SPOLY_E_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPOLY_E_DEVICE;
    spoly::TailArgs A;
    A.bvh.nodes = bvh->store.nodes;
    A.bvh.tris = bvh->store.tris;
    A.bvh.n_tris = bvh->store.n_tris;
    A.px = mesh->px; A.py = mesh->py; A.pz = mesh->pz;
    A.nx = mesh->nx; A.ny = mesh->ny; A.nz = mesh->nz;
    A.tri = mesh->tri;
    A.x0x = x0s->x; A.x0y = x0s->y; A.x0z = x0s->z;
    A.xlx = xls->x; A.xly = xls->y; A.xlz = xls->z;
    A.q_x0 = q_x0; A.q_xl = q_xl;
    A.sols = sols; A.n = n_sols; A.count = sol_count;
    A.k = k;
    A.ev[0] = chain[0]; A.ev[1] = k > 1 ? chain[1] : SPOLY_R;
    A.eta[0] = eta[0]; A.eta[1] = eta[1]; A.eta[2] = k > 1 ? eta[2] : eta[1];
    A.intensity = params->intensity; A.rho = params->reflectance; A.teps = params->t_eps;
    A.use_rn = params->rcv_normal[0] != 0.0 || params->rcv_normal[1] != 0.0 || params->rcv_normal[2] != 0.0;
    double rl = std::sqrt(params->rcv_normal[0] * params->rcv_normal[0] + params->rcv_normal[1] * params->rcv_normal[1] +
                          params->rcv_normal[2] * params->rcv_normal[2]);
    for (int i = 0; i < 3; ++i) A.rn[i] = A.use_rn ? params->rcv_normal[i] / rl : 0.0;
    A.mask = mask; A.contrib = contrib; A.image = image;
    return dev_err(spoly::launch_tail(A, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
