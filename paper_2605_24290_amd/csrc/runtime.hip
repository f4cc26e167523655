// C-ABI entry points of librxgs: context, scene and MLP upload, the render
// pipeline (Alg. 1 of RxGS with a view index in the sort key), exports.
#include "device_common.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

using namespace rxgs;

namespace {

thread_local std::string g_create_err;

rxgs_status fail(rxgs_ctx *ctx, rxgs_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

rxgs_status hip_fail(rxgs_ctx *ctx, hipError_t e, const char *what)
{
    (void)hipGetLastError();
    const rxgs_status st = (e == hipErrorOutOfMemory) ? RXGS_E_OOM : RXGS_E_DEVICE;
    return fail(ctx, st, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                   \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// a buffer of the context (scene, MLP, staging)
#define GROW(ctx, buf, bytes)                                                     \
    do {                                                                          \
        if (!grow((buf), (bytes), &(ctx)->alloc))                                 \
            return fail(ctx, RXGS_E_OOM, "device allocation failed: " #buf);      \
    } while (0)

// a buffer of workspace w (its own allocator, else the context's)
#define WGROW(ctx, w, buf, bytes)                                                 \
    do {                                                                          \
        (w).req_bytes += (bytes);                                                 \
        if (!grow((buf), (bytes), (w).al ? (w).al : &(ctx)->alloc))               \
            return fail(ctx, RXGS_E_OOM, (w).al && (w).al->base                   \
                                             ? "scratch region exhausted: " #buf  \
                                             : "device allocation failed: " #buf); \
    } while (0)

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DeviceScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

__global__ void k_count_nonfinite(const float *__restrict__ p, size_t n, unsigned *__restrict__ cnt)
{
    size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * BLOCK;
    unsigned c = 0;
    for (; i < n; i += stride) c += !isfinite(p[i]);
    if (c) atomicAdd(cnt, c);
}

// largest |p[i]| as FP32 bits (non-negative floats order like their bits)
__global__ void k_absmax_bits(const float *__restrict__ p, size_t n, unsigned *__restrict__ out)
{
    size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * BLOCK;
    unsigned m = 0;
    for (; i < n; i += stride) m = max(m, __float_as_uint(fabsf(p[i])));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

// AoS inputs -> SoA planes (x, y, z, ls0, ls1, ls2, qw, qx, qy, qz, logit)
__global__ void k_to_soa(const float *__restrict__ means, const float *__restrict__ ls,
                         const float *__restrict__ q, const float *__restrict__ lg, int64_t K,
                         float *__restrict__ soa)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    for (int a = 0; a < 3; a++) soa[a * K + k] = means[3 * k + a];
    for (int a = 0; a < 3; a++) soa[(3 + a) * K + k] = ls[3 * k + a];
    for (int a = 0; a < 4; a++) soa[(6 + a) * K + k] = q[4 * k + a];
    soa[10 * K + k] = lg[k];
}

bool all_finite_host(const float *p, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int bits_for(uint64_t n)
{
    int b = 0;
    while ((1ull << b) < n) b++;
    return b;
}

// pinned host staging of the workspace (grow-only)
bool ensure_pinned(Workspace &ws, size_t bytes)
{
    if (ws.h_pinned_cap >= bytes) return true;
    if (ws.fixed_host) return false;   // made at set-up, never regrown
    if (ws.h_pinned) (void)hipHostFree(ws.h_pinned);
    ws.h_pinned = nullptr;
    ws.h_pinned_cap = 0;
    size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
    if (hipHostMalloc(&ws.h_pinned, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ws.h_pinned = nullptr;
        return false;
    }
    ws.h_pinned_cap = want;
    return true;
}

// Size (bytes of the 2-D record gradients) above which the backward clears
// its per-position accumulators at visible positions only (256 MiB);
// RXGS_ZERO_VISIBLE_MIN overrides it (0: always), so that tests can take
// that path on small scenes.
size_t zero_visible_min()
{
    const char *e = std::getenv("RXGS_ZERO_VISIBLE_MIN");
    return (e && e[0]) ? (size_t)std::strtoull(e, nullptr, 10) : ((size_t)256 << 20);
}

// every device buffer of a workspace released (carved ones only forgotten)
void release_buffers(Workspace &ws)
{
    DevBuf *bufs[] = {&ws.centres, &ws.rxpos,   &ws.desc,   &ws.ext,     &ws.rawkey, &ws.opac,
                      &ws.skey[0], &ws.skey[1], &ws.sval[0], &ws.sval[1], &ws.srec,    &ws.ggeo,
                      &ws.qcull,   &ws.sbox,    &ws.vorder, &ws.poff, &ws.torder,
                      &ws.pkey[0], &ws.pkey[1], &ws.pval[0], &ws.pval[1], &ws.ranges, &ws.rad,
                      &ws.Lp,      &ws.Gp,      &ws.items,  &ws.Tfin,   &ws.nlast,  &ws.part,
                      &ws.counters, &ws.hist,   &ws.nvis_d, &ws.dS,    &ws.g2d,    &ws.dL,
                      &ws.dG,      &ws.mpart,   &ws.w1part,  &ws.mred,   &ws.live,   &ws.items_live, &ws.vflag,
                      &ws.items_far, &ws.frec, &ws.fcnt,  &ws.ftile,  &ws.hist_b, &ws.gfeat_tmp, &ws.gmlp_tmp,
                      &ws.rgam,    &ws.rab,     &ws.rloc,    &ws.gP,     &ws.dSP,
                      &ws.oinv,    &ws.rank,    &ws.lcnt,    &ws.dLv,     &ws.dGp,    &ws.bins,
                      &ws.pterm,   &ws.pacc};
    for (DevBuf *b : bufs) release(*b);
}

void free_workspace(Workspace &ws)
{
    release_buffers(ws);
    if (ws.staged) (void)hipEventDestroy(ws.staged);
    if (ws.counted) (void)hipEventDestroy(ws.counted);
    if (ws.done) (void)hipEventDestroy(ws.done);
    ws.staged = nullptr;
    ws.counted = nullptr;
    ws.done = nullptr;
    if (ws.h_pinned) (void)hipHostFree(ws.h_pinned);
    ws.h_pinned = nullptr;
    ws.h_pinned_cap = 0;
    ws.valid = false;
}

// waits for the last render or backward into ws (on whatever stream it ran)
hipError_t wait_workspace(const Workspace &ws)
{
    return ws.done ? hipEventSynchronize(ws.done) : hipSuccess;
}

// the context's private stream (non-blocking: it never waits for, nor stalls,
// the caller's or a server slot's streams)
hipError_t aux_stream(rxgs_ctx *ctx, hipStream_t &out)
{
    if (!ctx->aux) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ctx->aux = nullptr;
            return e;
        }
    }
    out = ctx->aux;
    return hipSuccess;
}

// synchronous copy on the context's private stream
hipError_t aux_copy(rxgs_ctx *ctx, void *dst, const void *src, size_t n, hipMemcpyKind kind)
{
    hipStream_t a = nullptr;
    hipError_t e = aux_stream(ctx, a);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, kind, a);
    if (e == hipSuccess) e = hipStreamSynchronize(a);
    return e;
}

}  // namespace

// ============================================================================
// stage timing
namespace rxgs {

int Profiler::stage_id(const char *name)
{
    for (size_t i = 0; i < names.size(); i++)
        if (names[i] == name) return (int)i;
    names.emplace_back(name);
    launches.push_back(0);
    ms.push_back(0.0);
    return (int)names.size() - 1;
}

hipEvent_t Profiler::take()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void Profiler::flush()
{
    for (const Pending &q : pending) {
        float t = 0.f;
        if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&t, q.a, q.b) == hipSuccess) {
            launches[q.stage] += 1;
            ms[q.stage] += t;
        } else {
            (void)hipGetLastError();
        }
        pool.push_back(q.a);
        pool.push_back(q.b);
    }
    pending.clear();
}

void Profiler::release_all()
{
    flush();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

StageMark::StageMark(Profiler &prof, const char *name, hipStream_t s) : p(&prof), st(s)
{
    if (!p->on) return;
    if (p->pending.size() > 65536) p->flush();
    stage = p->stage_id(name);
    a = p->take();
    if (a && hipEventRecord(a, st) != hipSuccess) {
        (void)hipGetLastError();
        p->pool.push_back(a);
        a = nullptr;
    }
}

StageMark::~StageMark()
{
    if (!a) return;
    hipEvent_t b = p->take();
    if (!b || hipEventRecord(b, st) != hipSuccess) {
        (void)hipGetLastError();
        p->pool.push_back(a);
        if (b) p->pool.push_back(b);
        return;
    }
    p->pending.push_back({stage, a, b});
}

}  // namespace rxgs

#define STAGE(ctx, name, expr)                              \
    do {                                                    \
        rxgs::StageMark sm_((ctx)->prof, name, st);         \
        HIPCHK(ctx, (expr));                                \
    } while (0)

extern "C" rxgs_status rxgs_profile_enable(rxgs_ctx *ctx, int on)
{
    if (!ctx) return RXGS_E_INVALID;
    DeviceScope ds(ctx->device);
    if (on && !ctx->prof.dcount) {
        void *p = nullptr;
        if (hipMalloc(&p, 64) != hipSuccess) return fail(ctx, RXGS_E_OOM, "profile counters: device allocation failed");
        ctx->prof.dcount = static_cast<unsigned long long *>(p);
        HIPCHK(ctx, hipMemset(p, 0, 64));
    }
    ctx->prof.on = on != 0;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_profile_counts(rxgs_ctx *ctx, rxgs_work_counts *out, int reset, void *stream)
{
    if (!ctx || !out) return RXGS_E_INVALID;
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    unsigned long long h[3] = {0, 0, 0};
    if (ctx->prof.dcount) {
        HIPCHK(ctx, hipMemcpyAsync(h, ctx->prof.dcount, sizeof h, hipMemcpyDeviceToHost, st));
        if (reset) HIPCHK(ctx, hipMemsetAsync(ctx->prof.dcount, 0, sizeof h, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    }
    out->mlp_items = (int64_t)h[0];
    out->mlp_pairs = (int64_t)h[1];
    out->mlp_slots = (int64_t)h[2];
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_profile_read(rxgs_ctx *ctx, rxgs_stage_time *out, int max_entries, int *n_entries,
                                         int reset)
{
    if (!ctx || max_entries < 0 || (max_entries > 0 && !out)) return RXGS_E_INVALID;
    DeviceScope ds(ctx->device);
    Profiler &p = ctx->prof;
    p.flush();
    const int n = (int)p.names.size();
    for (int i = 0; i < n && i < max_entries; i++) {
        std::memset(out[i].name, 0, sizeof out[i].name);
        std::strncpy(out[i].name, p.names[i].c_str(), sizeof out[i].name - 1);
        out[i].launches = p.launches[i];
        out[i].total_ms = p.ms[i];
    }
    if (n_entries) *n_entries = n;
    if (reset)
        for (int i = 0; i < n; i++) {
            p.launches[i] = 0;
            p.ms[i] = 0.0;
        }
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_set_near_cut(rxgs_ctx *ctx, int on)
{
    if (!ctx) return RXGS_E_INVALID;
    ctx->near_cut = on != 0;
    return RXGS_OK;
}

extern "C" int64_t rxgs_views_redone(const rxgs_ctx *ctx) { return ctx ? ctx->views_redone : -1; }

extern "C" rxgs_status rxgs_view_flags(rxgs_ctx *ctx, uint32_t *out, int32_t max_views, int32_t *n_views)
{
    if (!ctx || (max_views > 0 && !out)) return RXGS_E_INVALID;
    const Workspace &ws = ctx->ws;
    const int n = ws.vflag.p ? std::min<int>(ws.V, std::max(max_views, 0)) : 0;
    if (n_views) *n_views = ws.vflag.p ? ws.V : 0;
    if (n == 0) return RXGS_OK;
    DeviceScope ds(ctx->device);
    HIPCHK(ctx, wait_workspace(ws));
    HIPCHK(ctx, aux_copy(ctx, out, ws.vflag.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return RXGS_OK;
}

extern "C" const char *rxgs_version(void) { return "rxgs 0.1 (gfx950)"; }

extern "C" const char *rxgs_last_error(const rxgs_ctx *ctx)
{
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

// ============================================================================
// Scratch of the allocation-free entry point (rxgs_render_noalloc): one
// static array that every GPU the library runs on holds for the life of the
// process.  Host code never uses its name as an address: each device's copy
// is resolved once, with that device current, by hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[RXGS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
constexpr size_t NOALLOC_PINNED = (size_t)1 << 20;   // host staging of the counts and descriptors
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// this device's copy of the scratch array (the device must be current)
hipError_t scratch_address(int device, void **out)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// the allocation-free workspace of a context: carved from the device's
// scratch array, with its pinned staging and events made here, at set-up
rxgs_status setup_noalloc(rxgs_ctx *ctx)
{
    void *sp = nullptr;
    hipError_t e = scratch_address(ctx->device, &sp);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress(scratch)");
    ctx->fixed.base = static_cast<char *>(sp);
    ctx->fixed.cap = RXGS_NOALLOC_SCRATCH_BYTES;
    ctx->fixed.used = 0;
    ctx->fixed.device = ctx->device;
    rxgs_saved *s = new (std::nothrow) rxgs_saved();
    if (!s) return fail(ctx, RXGS_E_OOM, "out of host memory");
    s->ctx = ctx;
    s->keep = false;
    s->ws.al = &ctx->fixed;
    ctx->noalloc = s;
    Workspace &ws = s->ws;
    e = hipHostMalloc(&ws.h_pinned, NOALLOC_PINNED, hipHostMallocDefault);
    if (e != hipSuccess) {
        ws.h_pinned = nullptr;
        return hip_fail(ctx, e, "pinned staging of the allocation-free workspace");
    }
    ws.h_pinned_cap = NOALLOC_PINNED;
    ws.fixed_host = true;
    HIPCHK(ctx, hipEventCreateWithFlags(&ws.staged, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ws.counted, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ws.done, hipEventDisableTiming));
    return RXGS_OK;
}
}  // namespace

extern "C" rxgs_status rxgs_create(int device, const rxgs_grid *grid, rxgs_ctx **out)
{
    if (!out) {
        g_create_err = "out is NULL";
        return RXGS_E_INVALID;
    }
    *out = nullptr;
    if (!grid || grid->H < 1 || grid->W < 2 || (grid->W & 1) || grid->reserved != 0 ||
        !std::isfinite(grid->el0) || !std::isfinite(grid->del_el) || !(grid->del_el > 0.0) ||
        (int64_t)grid->H * grid->W > (1ll << 28)) {
        g_create_err = "invalid grid (H >= 1, even W >= 2, finite el0, del_el > 0)";
        return RXGS_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        g_create_err = "no such HIP device";
        return RXGS_E_DEVICE;
    }
    rxgs_ctx *ctx = new (std::nothrow) rxgs_ctx();
    if (!ctx) {
        g_create_err = "out of host memory";
        return RXGS_E_OOM;
    }
    ctx->device = device;
    ctx->alloc.device = device;
    {
        const char *e = std::getenv("RXGS_DETERMINISTIC");
        ctx->deterministic = e && e[0] == '1';
        const char *ps = std::getenv("RXGS_PAIR_SORT");
        ctx->pair_sort = ps && ps[0] == '1';
    }
    ctx->grid = *grid;
    DevGrid &g = ctx->g;
    g.H = grid->H;
    g.W = grid->W;
    g.tiles_x = (grid->W + TILE - 1) / TILE;
    g.tiles_y = (grid->H + TILE - 1) / TILE;
    g.tiles = g.tiles_x * g.tiles_y;
    g.el0 = grid->el0;
    g.del = grid->del_el;
    g.daz = 2.0 * M_PI / (double)grid->W;
    g.idaz = (double)grid->W / (2.0 * M_PI);
    g.idel = 1.0 / grid->del_el;
    {
        DeviceScope ds(device);
        const rxgs_status rs = setup_noalloc(ctx);
        if (rs != RXGS_OK) {
            g_create_err = ctx->err;
            rxgs_destroy(ctx);
            return rs;
        }
    }
    *out = ctx;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_create_with_allocator(int device, const rxgs_grid *grid, rxgs_alloc_fn alloc,
                                                  rxgs_free_fn free_fn, void *user, rxgs_ctx **out)
{
    if (!alloc || !free_fn) {
        g_create_err = "allocator callbacks must both be given";
        if (out) *out = nullptr;
        return RXGS_E_INVALID;
    }
    rxgs_status rs = rxgs_create(device, grid, out);
    if (rs != RXGS_OK) return rs;
    (*out)->alloc.alloc = alloc;
    (*out)->alloc.free = free_fn;
    (*out)->alloc.user = user;
    return RXGS_OK;
}

extern "C" void rxgs_destroy(rxgs_ctx *ctx)
{
    if (!ctx) return;
    DeviceScope ds(ctx->device);
    (void)wait_workspace(ctx->ws);
    if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
    ctx->prof.release_all();
    if (ctx->prof.dcount) (void)hipFree(ctx->prof.dcount);
    free_workspace(ctx->ws);
    release(ctx->scene.soa);
    release(ctx->scene.rad);
    release(ctx->scene.feat);
    release(ctx->mlp.raw);
    release(ctx->mlp.w2a);
    release(ctx->mlp.w2b);
    release(ctx->mlp.tab);
    release(ctx->mlp.w2h);
    release(ctx->mlp.tabh);
    release(ctx->mlp.w1h);
    release(ctx->mlp.b1tab);
    release_rxcond(ctx->rxc);
    release(ctx->stage);
    if (ctx->noalloc) {
        (void)wait_workspace(ctx->noalloc->ws);
        free_workspace(ctx->noalloc->ws);
        delete ctx->noalloc;
        ctx->noalloc = nullptr;
    }
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    delete ctx;
}

extern "C" rxgs_status rxgs_saved_create(rxgs_ctx *ctx, rxgs_saved **out)
{
    if (!ctx || !out) return fail(ctx, RXGS_E_INVALID, "NULL argument");
    rxgs_saved *s = new (std::nothrow) rxgs_saved();
    if (!s) return fail(ctx, RXGS_E_OOM, "out of host memory");
    s->ctx = ctx;
    ctx->saved.push_back(s);
    *out = s;
    return RXGS_OK;
}

extern "C" void rxgs_saved_destroy(rxgs_saved *s)
{
    if (!s) return;
    rxgs_ctx *ctx = s->ctx;
    DeviceScope ds(ctx->device);
    (void)wait_workspace(s->ws);
    if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
    free_workspace(s->ws);
    auto &v = ctx->saved;
    v.erase(std::remove(v.begin(), v.end(), s), v.end());
    delete s;
}

extern "C" rxgs_status rxgs_scene_upload(rxgs_ctx *ctx, int64_t K, const float *means, const float *log_scales,
                                         const float *quats, const float *logits, const float *radiance,
                                         const float *features, int src_on_device, void *stream)
{
    if (!ctx) return RXGS_E_INVALID;
    if (K < 0 || K > (1ll << 27)) return fail(ctx, RXGS_E_INVALID, "K out of range [0, 2^27]");
    if (radiance && features) return fail(ctx, RXGS_E_INVALID, "at most one of radiance and features may be given");
    if (K > 0 && (!means || !log_scales || !quats || !logits))
        return fail(ctx, RXGS_E_INVALID, "NULL scene array");
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Scene &sc = ctx->scene;
    sc.valid = false;
    const bool feat = features != nullptr;
    const bool geo = !feat && !radiance;   // geometry only: radiance from a conditioning model
    const size_t nrad = geo ? 0 : (size_t)K * (feat ? FEAT : 2);
    const float *radsrc = feat ? features : radiance;
    const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (!src_on_device) {
        if (!all_finite_host(means, 3 * K) || !all_finite_host(log_scales, 3 * K) ||
            !all_finite_host(quats, 4 * K) || !all_finite_host(logits, K) || !all_finite_host(radsrc, nrad))
            return fail(ctx, RXGS_E_INVALID, "non-finite value in the scene");
        for (int64_t k = 0; k < K; k++) {
            const float *q = quats + 4 * k;
            if (q[0] == 0.f && q[1] == 0.f && q[2] == 0.f && q[3] == 0.f)
                return fail(ctx, RXGS_E_INVALID, "zero quaternion");
        }
    }
    GROW(ctx, sc.soa, (size_t)11 * std::max<int64_t>(K, 1) * 4);
    GROW(ctx, ctx->stage, (size_t)12 * std::max<int64_t>(K, 1) * 4 + 256);
    float *stg = ctx->stage.as<float>();
    if (K > 0) {
        HIPCHK(ctx, hipMemcpyAsync(stg, means, 12 * K, kind, st));
        HIPCHK(ctx, hipMemcpyAsync(stg + 3 * K, log_scales, 12 * K, kind, st));
        HIPCHK(ctx, hipMemcpyAsync(stg + 6 * K, quats, 16 * K, kind, st));
        HIPCHK(ctx, hipMemcpyAsync(stg + 10 * K, logits, 4 * K, kind, st));
        hipLaunchKernelGGL(k_to_soa, dim3((unsigned)((K + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, stg, stg + 3 * K,
                           stg + 6 * K, stg + 10 * K, K, sc.soa.as<float>());
        HIPCHK(ctx, hipGetLastError());
    }
    DevBuf &dst = feat ? sc.feat : sc.rad;
    GROW(ctx, dst, std::max<size_t>(nrad, 1) * 4);
    if (K > 0 && nrad > 0) HIPCHK(ctx, hipMemcpyAsync(dst.p, radsrc, nrad * 4, kind, st));
    float fmax = 0.f;   // largest |feature|, for the split-FP16 layer-1 path
    if (src_on_device && K > 0) {
        unsigned *cnt = reinterpret_cast<unsigned *>(stg + 11 * K);
        HIPCHK(ctx, hipMemsetAsync(cnt, 0, 8, st));
        const unsigned blocks = (unsigned)std::min<int64_t>((11 * K + BLOCK - 1) / BLOCK, 2048);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks), dim3(BLOCK), 0, st, sc.soa.as<float>(), (size_t)11 * K,
                           cnt);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks), dim3(BLOCK), 0, st, dst.as<float>(), nrad, cnt);
        if (feat) hipLaunchKernelGGL(k_absmax_bits, dim3(blocks), dim3(BLOCK), 0, st, dst.as<float>(), nrad, cnt + 1);
        HIPCHK(ctx, hipGetLastError());
        unsigned h[2] = {0, 0};
        HIPCHK(ctx, hipMemcpyAsync(h, cnt, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        if (h[0]) return fail(ctx, RXGS_E_INVALID, "non-finite value in the scene");
        std::memcpy(&fmax, &h[1], 4);
    } else if (feat) {
        for (size_t i = 0; i < nrad; i++) fmax = std::max(fmax, std::fabs(radsrc[i]));
    }
    sc.fmax = fmax;
    sc.K = K;
    sc.has_features = feat;
    sc.geometry_only = geo && K > 0;
    ctx->rxc.valid = false;   // its occupancy grid and coefficients belong to the old scene
    sc.version = ++ctx->version_counter;
    sc.valid = true;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_mlp_upload(rxgs_ctx *ctx, const float *params, int src_on_device, void *stream)
{
    if (!ctx) return RXGS_E_INVALID;
    if (!params) return fail(ctx, RXGS_E_INVALID, "params is NULL");
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<float> h(RXGS_MLP_NPARAM);
    if (src_on_device) {
        HIPCHK(ctx, hipMemcpyAsync(h.data(), params, sizeof(float) * h.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    } else {
        std::memcpy(h.data(), params, sizeof(float) * h.size());
    }
    if (!all_finite_host(h.data(), h.size())) return fail(ctx, RXGS_E_INVALID, "non-finite MLP parameter");
    const float *W2 = h.data() + HID * MLP_IN + HID;
    const float *b2 = W2 + HID * HID;
    const float *W3 = b2 + HID;
    // MFMA A-operand layouts of W2 (forward) and W2^T (backward):
    //   w2a[mb][t][lane] = W2[32 mb + lane % 32][hid_of(lane / 32, t)]
    //   w2b[ib][t][lane] = W2[hid_of(lane / 32, t)][32 ib + lane % 32]
    std::vector<float> w2a(2 * 32 * 64), w2b(2 * 32 * 64);
    for (int mb = 0; mb < 2; mb++)
        for (int t = 0; t < 32; t++)
            for (int l = 0; l < 64; l++) {
                w2a[(mb * 32 + t) * 64 + l] = W2[(32 * mb + (l & 31)) * HID + hid_of(l >> 5, t)];
                w2b[(mb * 32 + t) * 64 + l] = W2[hid_of(l >> 5, t) * HID + 32 * mb + (l & 31)];
            }
    // per (lane half h, block mb, accumulator register r): hidden index d and
    // its layer-3 weights and layer-2 bias
    std::vector<float> tab(2 * 2 * 16 * 4, 0.f);
    for (int hh = 0; hh < 2; hh++)
        for (int mb = 0; mb < 2; mb++)
            for (int r = 0; r < 16; r++) {
                const int d = 32 * mb + 8 * (r / 4) + 4 * hh + (r % 4);
                float *e = &tab[((hh * 2 + mb) * 16 + r) * 4];
                e[0] = W3[d];
                e[1] = W3[HID + d];
                e[2] = b2[d];
            }
    // split-FP16 copy of W2 for the forward pair kernel: W2 is scaled by an
    // exact power of two so that its largest entry lands just under 2^15
    // (FP16 range, and the low halves stay out of the subnormal range); the
    // scale is undone exactly in the layer-2 bias and the layer-3 weights.
    float wmax = 0.f;
    for (int i = 0; i < HID * HID; i++) wmax = std::max(wmax, std::fabs(W2[i]));
    int e = 0;
    if (wmax > 0.f) std::frexp(wmax, &e);   // wmax < 2^e
    const int wexp = std::min(std::max(15 - e, -120), 120);
    std::vector<_Float16> w2h(2 * 2 * 4 * 64 * 8);
    for (int mb = 0; mb < 2; mb++)
        for (int q = 0; q < 4; q++)
            for (int l = 0; l < 64; l++)
                for (int i = 0; i < 8; i++) {
                    const float w = std::ldexp(W2[(32 * mb + (l & 31)) * HID + hid_of(l >> 5, 8 * q + i)], wexp);
                    const _Float16 hi = (_Float16)w;
                    const _Float16 lo = (_Float16)(w - (float)hi);
                    w2h[(((0 * 2 + mb) * 4 + q) * 64 + l) * 8 + i] = hi;
                    w2h[(((1 * 2 + mb) * 4 + q) * 64 + l) * 8 + i] = lo;
                }
    // split-FP16 copy of the feature block of W1 for computing the Gaussians'
    // layer-1 term inside the pair kernel: W1[:, 36:] * 2^w1exp (largest entry
    // just under 2^15) as FP16 (hi, lo) pairs in the MFMA 32x32x16 A-operand
    // layout, [2 part][2 mb][2 q][64 lane] x 8 halves, element i =
    // W1[32 mb + lane % 32][36 + 16 q + 8 (lane / 32) + i]; b1 in the
    // accumulator order of each lane half; per-row sums of |W1[:, 36:]|
    const float *W1 = h.data();
    const float *b1 = W1 + HID * MLP_IN;
    float w1max = 0.f;
    for (int d = 0; d < HID; d++)
        for (int c = 0; c < FEAT; c++) w1max = std::max(w1max, std::fabs(W1[d * MLP_IN + ENC + c]));
    int e1 = 0;
    if (w1max > 0.f) std::frexp(w1max, &e1);
    const int w1exp = std::min(std::max(15 - e1, -120), 120);
    std::vector<_Float16> w1h(2 * 2 * 2 * 64 * 8);
    for (int mb = 0; mb < 2; mb++)
        for (int q = 0; q < 2; q++)
            for (int l = 0; l < 64; l++)
                for (int i = 0; i < 8; i++) {
                    const float w = std::ldexp(W1[(32 * mb + (l & 31)) * MLP_IN + ENC + 16 * q + 8 * (l >> 5) + i],
                                               w1exp);
                    const _Float16 hi = (_Float16)w;
                    const _Float16 lo = (_Float16)(w - (float)hi);
                    w1h[(((0 * 2 + mb) * 2 + q) * 64 + l) * 8 + i] = hi;
                    w1h[(((1 * 2 + mb) * 2 + q) * 64 + l) * 8 + i] = lo;
                }
    std::vector<float> b1tab(2 * 32);
    bool b1_exact = true;
    for (int hh = 0; hh < 2; hh++)
        for (int t = 0; t < 32; t++) {
            const float x = std::ldexp(b1[hid_of(hh, t)], w1exp);
            if (!std::isfinite(x) || (b1[hid_of(hh, t)] != 0.f && std::fabs(x) < FLT_MIN)) b1_exact = false;
            b1tab[hh * 32 + t] = x;
        }
    std::vector<double> w1abs(HID);
    for (int d = 0; d < HID; d++) {
        double r = 0.0;
        for (int c = 0; c < FEAT; c++) r += std::fabs((double)W1[d * MLP_IN + ENC + c]);
        w1abs[d] = r;
    }

    // the rescaled layer-2 bias and layer-3 weights must stay finite and
    // normal (an exact rescaling); otherwise layer 2 runs on FP32 MFMA
    std::vector<float> tabh(tab);
    bool exact = true;
    for (size_t i = 0; i < tabh.size(); i += 4) {
        for (int c = 0; c < 3; c++) {
            const float x = std::ldexp(tab[i + c], c < 2 ? -wexp : wexp);
            if (!std::isfinite(x) || (tab[i + c] != 0.f && std::fabs(x) < FLT_MIN)) exact = false;
            tabh[i + c] = x;
        }
    }
    Mlp &m = ctx->mlp;
    m.valid = false;
    const char *env = std::getenv("RXGS_MLP_FP32");
    m.fp32 = !exact || (env && env[0] == '1');
    m.wexp = wexp;
    m.w1exp = w1exp;
    m.w1_ok = b1_exact && w1max < 32768.f;
    for (int d = 0; d < HID; d++) {
        m.w1abs[d] = w1abs[d];
        m.b1abs[d] = std::fabs((double)b1[d]);
    }
    GROW(ctx, m.w1h, sizeof(_Float16) * w1h.size());
    GROW(ctx, m.b1tab, sizeof(float) * b1tab.size());
    HIPCHK(ctx, hipMemcpyAsync(m.w1h.p, w1h.data(), sizeof(_Float16) * w1h.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.b1tab.p, b1tab.data(), sizeof(float) * b1tab.size(), hipMemcpyHostToDevice, st));
    GROW(ctx, m.w2h, sizeof(_Float16) * w2h.size());
    GROW(ctx, m.tabh, sizeof(float) * tabh.size());
    HIPCHK(ctx, hipMemcpyAsync(m.w2h.p, w2h.data(), sizeof(_Float16) * w2h.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.tabh.p, tabh.data(), sizeof(float) * tabh.size(), hipMemcpyHostToDevice, st));
    GROW(ctx, m.raw, sizeof(float) * RXGS_MLP_NPARAM);
    GROW(ctx, m.w2a, sizeof(float) * w2a.size());
    GROW(ctx, m.w2b, sizeof(float) * w2b.size());
    GROW(ctx, m.tab, sizeof(float) * tab.size());
    HIPCHK(ctx, hipMemcpyAsync(m.raw.p, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.w2a.p, w2a.data(), sizeof(float) * w2a.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.w2b.p, w2b.data(), sizeof(float) * w2b.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.tab.p, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice, st));
    // (ordered after earlier work on the caller's stream that may still read
    // the old tables; the host vectors must outlive the copies)
    HIPCHK(ctx, hipStreamSynchronize(st));
    m.version = ++ctx->version_counter;
    m.valid = true;
    return RXGS_OK;
}

// ============================================================================
// TX renders whose views have at most this many receivers take the prefix
// radiance path; with more, the weights-only pass (see render_pass).
constexpr int PREFIX_MAX_RX = 128;

// One pass of the forward.  limit caps, per view, the depth-sorted entries
// that are emitted (the nearest ones); the blend flags every view it cut that
// still has a pixel whose transmittance stayed above the stop threshold.
static rxgs_status render_pass(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off, int N,
                               const float *rx, float *C, float *power, float *csum, float *amp, rxgs_saved *saved,
                               void *stream, uint32_t limit, int rsrc = RSRC_SCENE)
{
    if (!ctx) return RXGS_E_INVALID;
    if (mode != RXGS_MODE_TX && mode != RXGS_MODE_RX) return fail(ctx, RXGS_E_INVALID, "unknown mode");
    if (N < 0) return fail(ctx, RXGS_E_INVALID, "N < 0");
    if (N > 0 && (!rx || !C)) return fail(ctx, RXGS_E_INVALID, "rx or C is NULL");
    if (saved && saved->ctx != ctx) return fail(ctx, RXGS_E_INVALID, "saved state of another context");
    const Scene &sc = ctx->scene;
    if (!sc.valid) return fail(ctx, RXGS_E_STATE, "no scene uploaded");
    const bool rxc = rsrc == RSRC_RXCOND;
    if (!rxc && sc.has_features && !ctx->mlp.valid)
        return fail(ctx, RXGS_E_STATE, "MLP scene without an uploaded MLP");
    if (!rxc && sc.geometry_only)
        return fail(ctx, RXGS_E_STATE, "the scene has no radiance of its own: render it with rxgs_render_rxcond");
    if (rxc && (!ctx->rxc.valid || ctx->rxc.scene_version != sc.version))
        return fail(ctx, RXGS_E_STATE, "no conditioning model uploaded for the current scene");
    const int Ch = rxc ? ctx->rxc.C : 1;   // output rows per receiver
    if ((int64_t)N * Ch > (1ll << 30)) return fail(ctx, RXGS_E_INVALID, "too many receiver channels");
    std::vector<int> rxview(N);
    int V = 0;
    if (mode == RXGS_MODE_TX) {
        if (Q < 1 || !tx || !rx_off) return fail(ctx, RXGS_E_INVALID, "TX mode needs Q >= 1, tx and rx_off");
        if (rx_off[0] != 0 || rx_off[Q] != N) return fail(ctx, RXGS_E_INVALID, "rx_off must run from 0 to N");
        for (int q = 0; q < Q; q++) {
            if (rx_off[q + 1] < rx_off[q]) return fail(ctx, RXGS_E_INVALID, "rx_off must be non-decreasing");
            for (int j = rx_off[q]; j < rx_off[q + 1]; j++) rxview[j] = q;
        }
        V = Q;
    } else {
        for (int j = 0; j < N; j++) rxview[j] = j;
        V = N;
    }
    if (N == 0) return RXGS_OK;
    const int NR = N * Ch;   // rows (receiver, channel), receiver-major
    const DevGrid &g = ctx->g;
    const int64_t K = sc.K;
    const int64_t Kp = round_up(std::max<int64_t>(K, 1), SORT_TILE);
    if ((uint64_t)V * (uint64_t)Kp >= (1ull << 32) || (uint64_t)V * (uint64_t)g.tiles >= (1ull << 32))
        return fail(ctx, RXGS_E_INVALID, "views x Gaussians exceeds 2^32; split the receivers");
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Workspace &ws = saved ? saved->ws : ctx->ws;
    const bool save = saved && saved->keep;   // keep state for the backward and the exports
    ws.valid = false;
    ws.req_bytes = 0;
    // a deterministic backward needs every position's radiance (no prefix,
    // whose far-position work list is built in arrival order)
    ws.det = save && ctx->deterministic && rsrc == RSRC_SCENE;
    if (!ws.staged) {
        HIPCHK(ctx, hipEventCreateWithFlags(&ws.staged, hipEventDisableTiming));
        HIPCHK(ctx, hipEventCreateWithFlags(&ws.counted, hipEventDisableTiming));
        HIPCHK(ctx, hipEventCreateWithFlags(&ws.done, hipEventDisableTiming));
    } else {
        // the previous render's host-to-device copies out of the staging buffer
        HIPCHK(ctx, hipEventSynchronize(ws.staged));
    }
    const size_t VK = (size_t)V * Kp;
    ws.mode = mode;
    ws.V = V;
    ws.N = NR;
    ws.Nrx = N;
    ws.Ch = Ch;
    ws.rsrc = rsrc;
    ws.Q = Q;
    ws.K = K;
    ws.Kp = Kp;
    ws.g = g;
    ws.use_mlp = !rxc && sc.has_features;
    ws.use_items = ws.use_mlp || rxc;
    std::vector<int> rowview(NR);   // view of each output row
    for (int j = 0; j < N; j++)
        for (int c = 0; c < Ch; c++) rowview[(size_t)j * Ch + c] = rxview[j];
    ws.h_rxview = rowview;
    ws.limit = limit;
    WGROW(ctx, ws, ws.vflag, (size_t)V * 4);

    if (save) {
        // the backward needs the view centres and receiver positions later
        WGROW(ctx, ws, ws.centres, (size_t)V * 12);
        WGROW(ctx, ws, ws.rxpos, (size_t)N * 12);
    }
    // (a saved state's binning boxes, raw keys and opacities are computed
    // when first exported: the backward does not read them)
    ws.exports_ready = false;
    for (int b = 0; b < 2; b++) {
        WGROW(ctx, ws, ws.skey[b], VK * 4);
        WGROW(ctx, ws, ws.sval[b], VK * 4);
    }
    WGROW(ctx, ws, ws.srec, VK * 32);
    WGROW(ctx, ws, ws.sbox, VK * 16);
    WGROW(ctx, ws, ws.vorder, VK * 4);
    WGROW(ctx, ws, ws.poff, VK * 4);
    WGROW(ctx, ws, ws.ggeo, (size_t)std::max<int64_t>(K, 1) * 48);
    WGROW(ctx, ws, ws.qcull, (size_t)std::max<int64_t>(K, 1) * 4);
    // per view (visible count, pair count); slots for the largest |layer-1
    // term| of the receivers and of the Gaussians (FP32 bits); render
    // statistics; the emission's ticket, error word and look-back status
    const size_t emit_words_n = emit_word_count(V, Kp);
    const size_t cnt_words = (size_t)4 * V + AMAX_SLOTS + 2 * STAT_WORDS + emit_words_n + 16;   // + far-item count
    WGROW(ctx, ws, ws.counters, cnt_words * 4);
    WGROW(ctx, ws, ws.hist, sort_ws_bytes((uint32_t)VK, 32, V));
    // grids of at most BIN_MAX_TILES tiles: the first emission counts its
    // pairs per tile and the pairs are placed in their tile lists directly
    ws.direct_bins = g.tiles <= BIN_MAX_TILES && !ctx->pair_sort;
    emit1_chunking(ws);
    if (ws.direct_bins) WGROW(ctx, ws, ws.bins, bins_bytes(V, ws.em_cpv));

    if (save) {
        HIPCHK(ctx, hipMemcpyAsync(ws.centres.p, mode == RXGS_MODE_TX ? tx : rx, (size_t)V * 12,
                                   hipMemcpyDeviceToDevice, st));
        HIPCHK(ctx, hipMemcpyAsync(ws.rxpos.p, rx, (size_t)N * 12, hipMemcpyDeviceToDevice, st));
        ws.centres_p = ws.centres.as<float>();
        ws.rxpos_p = ws.rxpos.as<float>();
    } else {
        ws.centres_p = mode == RXGS_MODE_TX ? tx : rx;
        ws.rxpos_p = rx;
    }

    // stage 1: depth keys (with the cheap culls), the per-view depth sort,
    // then the exact projection in depth order, which compacts the visible
    // entries and counts them and their pairs; the host waits only for those
    // counts
    // (the projection-terms kernel also clears the counters and the depth
    // sort's scratch; the key kernel adds the keys' digits to the sort's totals)
    const size_t depth_sort_words = sort_ws_bytes((uint32_t)VK, 32, V) / 4;
    STAGE(ctx, "project",
          launch_project(sc, ws.centres_p, V, Kp, g, ws, cnt_words, depth_sort_words, st));
    int cur = 0;
    STAGE(ctx, "sort_depth",
          sort_pairs_u32(ws.skey, ws.sval, ws.hist, cur, (uint32_t)VK, 32, V, Kp, nullptr, st, true, true,
                         emit_words(ws) + KEPT_STRIDE, SORT_VALS_INDEX | SORT_VALS_ONLY));
    ws.sorted_buf = cur;
    STAGE(ctx, "emit_records", launch_emit1(sc, ws, g, st));
    // one copy: the per-view counts up to and including the emission's error word
    const size_t head_bytes = (size_t)(emit_words(ws) - ws.counters.as<uint32_t>() + 1) * 4;
    if (!ensure_pinned(ws, head_bytes + 64)) return fail(ctx, RXGS_E_OOM, "pinned allocation failed");
    unsigned long long *h_cnt = static_cast<unsigned long long *>(ws.h_pinned);
    const uint32_t *h_err = static_cast<const uint32_t *>(ws.h_pinned) + (head_bytes / 4 - 1);
    HIPCHK(ctx, hipMemcpyAsync(h_cnt, ws.counters.p, head_bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipEventRecord(ws.counted, st));
    // each chunk's start in every tile list, and the views' list lengths
    if (ws.direct_bins) STAGE(ctx, "bin_scan", launch_bin_scan(ws, g, st));
    // the receivers' layer-1 term depends on nothing above: it runs while the
    // host waits for the counts
    if (ws.use_mlp) {
        WGROW(ctx, ws, ws.Gp, (size_t)N * HID * 4);
        STAGE(ctx, "mlp_global", launch_mlp_global_term(ctx->mlp, ws, st));
    }
    if (rxc) {
        // the conditioning's receiver terms: the encoding into the global
        // MLP and its modulation of every component (O(L) per receiver)
        WGROW(ctx, ws, ws.rgam, (size_t)N * RXGS_RXCOND_HIDDEN * 4);
        WGROW(ctx, ws, ws.rab, (size_t)N * ctx->rxc.L * Ch * 16);
        STAGE(ctx, "rxcond_global", launch_rxcond_receivers(ctx->rxc, ws, st));
    }

    // receiver chunks of the blend (independent of the counters: built while
    // the GPU projects and sorts); the receivers of a view are consecutive
    std::vector<int> vfirst(V, 0), vnrx(V, 0);
    for (int j = N - 1; j >= 0; j--) {
        vfirst[rxview[j]] = j;
        vnrx[rxview[j]]++;
    }
    // (in rows: a view's receivers, and each receiver's channels, are consecutive)
    const bool shared_view = mode == RXGS_MODE_TX || Ch > 1;   // several rows share a view's weights
    int maxr = 1;
    ws.rx_max = 1;
    for (int v = 0; v < V; v++) {
        maxr = std::max(maxr, vnrx[v] * Ch);
        ws.rx_max = std::max(ws.rx_max, vnrx[v]);
    }
    ws.R_max = maxr;
    int R = 1;
    if (shared_view)
        while (R < 16 && R < maxr) R *= 2;
    ws.R = R;
    std::vector<int4> chunks;
    for (int v = 0; v < V; v++)
        for (int a = 0; a < vnrx[v] * Ch; a += R) {
            const int j = vfirst[v] * Ch + a;
            const int tslot = shared_view ? (a == 0 ? v : -1) : j;
            chunks.push_back(make_int4(v, j, std::min(R, vnrx[v] * Ch - a), tslot));
        }
    ws.n_chunks = (int)chunks.size();
    ws.n_tslots = shared_view ? V : N;
    // Lazy radiance (TX mode, several receivers per view, nothing saved): the
    // weights do not depend on the receiver, so one weights-only pass per view
    // marks the position blocks some pixel composites and the pair MLP runs
    // on those blocks only.  Saved states keep every visible position's
    // radiance (it is exported).
    std::vector<int4> wchunks;
    if (mode == RXGS_MODE_TX && !save && ws.use_items)
        for (int v = 0; v < V; v++)
            if (vnrx[v] >= LAZY_MIN_RX) wchunks.push_back(make_int4(v, 0, 0, -1));
    ws.n_wchunks = (int)wchunks.size();
    ws.lazy = ws.n_wchunks > 0 && R >= 2;   // the colour pass is the multi-receiver one
    if (!ws.lazy) {
        wchunks.clear();
        ws.n_wchunks = 0;
    }

    HIPCHK(ctx, hipEventSynchronize(ws.counted));
    if (*h_err & 2u) return fail(ctx, RXGS_E_INVALID, "more than 2^32 - 1 pairs in one view; use a coarser grid");
    if (*h_err) return fail(ctx, RXGS_E_DEVICE, "emission look-back did not complete");

    // pairs per view; each view's pairs get a segment padded to whole sort blocks
    uint64_t D = 0, Dpad = 0;
    ws.h_pbase.assign(V, 0);
    ws.h_pcount.assign(V, 0);
    std::vector<int4> segtab;
    for (int v = 0; v < V; v++) {
        const uint64_t dv = h_cnt[2 * v + 1];
        ws.h_pbase[v] = (uint32_t)Dpad;
        ws.h_pcount[v] = (uint32_t)dv;
        const uint64_t nb = (dv + SORT_TILE - 1) / SORT_TILE;
        for (uint64_t b = 0; b < nb; b++)
            segtab.push_back(make_int4((int)(Dpad / SORT_TILE), (int)nb, v, 0));
        D += dv;
        Dpad += nb * SORT_TILE;
        if (Dpad >= (1ull << 32) - SORT_TILE) return fail(ctx, RXGS_E_INVALID, "more than 2^32 pairs; split the receivers");
    }
    ws.D = (int64_t)D;
    ws.Dpad = (int64_t)Dpad;
    ws.h_nvis.assign(V, 0);
    ws.nvis_total = 0;
    for (int v = 0; v < V; v++) {
        ws.h_nvis[v] = (int)h_cnt[2 * v];
        ws.nvis_total += ws.h_nvis[v];
    }
    // Prefix radiance (TX-mode MLP renders without saved state): compositing stops
    // at T < 1e-4, so in thick scenes a view composites only its nearest few
    // hundred Gaussians.  The pair MLP first runs on the PREFIX_POS nearest
    // sorted positions of each view; the blend gives the others zero radiance
    // and flags any view that composites one of them; those views get the
    // rest of their radiance and are blended again (all on the device).
    // A lane that composites an entry past the prefix records it (T w and
    // position, up to FAR_RECORDS per pixel); once the rest of the view's
    // radiance exists, a second launch adds the recorded terms in list order
    // (after the prefix's, as in one pass: the tile lists are in depth order),
    // and blends again only views whose pixels recorded more.  With many
    // receivers on a TX view the prefix costs PREFIX_POS MLP pairs per
    // receiver, while the weights-only pass costs one blend of the view
    // whatever the receiver count: such renders keep the weights pass.
    ws.mpos = 0xFFFFFFFFu;
    const uint32_t prefix = mode == RXGS_MODE_TX ? PREFIX_POS : PREFIX_POS_RX;
    // Saved states take it too: the transmittances, stop indices and
    // statistics come from the first pass (weights do not depend on the
    // radiance), the backward reads the radiance of composited entries only,
    // and a radiance export evaluates the rest first.
    if (ws.use_items && !ws.det && (mode == RXGS_MODE_RX || maxr < PREFIX_MAX_RX))
        for (int v = 0; v < V; v++)
            if ((uint32_t)ws.h_nvis[v] > prefix) ws.mpos = prefix;
    ws.rad_complete = ws.mpos == 0xFFFFFFFFu;
    if (ws.mpos != 0xFFFFFFFFu && ws.lazy) {   // the prefix replaces the weights-only pass
        ws.lazy = false;
        wchunks.clear();
        ws.n_wchunks = 0;
    }

    // MLP work items, per view: (32 sorted positions) x (16 receivers),
    // position-major; only their per-view offsets are built here, the items
    // themselves on the device
    std::vector<uint32_t> item_off(V + 1, 0);
    std::vector<int4> vinfo(V);   // (first receiver, receivers, visible, takes the weights pass)
    int64_t nfar = 0;
    for (int v = 0; v < V; v++) {
        const int64_t nb = (ws.h_nvis[v] + MLP_PAIRS - 1) / MLP_PAIRS, nrg = (vnrx[v] + MLP_RG - 1) / MLP_RG;
        const int64_t nb0 = std::min<int64_t>(nb, ws.mpos / MLP_PAIRS);
        const int64_t ni = ws.use_items ? nb0 * nrg : 0;
        nfar += ws.use_items ? (nb - nb0) * nrg : 0;
        if ((int64_t)item_off[v] + ni >= (1ll << 31)) return fail(ctx, RXGS_E_INVALID, "too many MLP work items");
        item_off[v + 1] = item_off[v] + (uint32_t)ni;
        vinfo[v] = make_int4(vfirst[v], vnrx[v], ws.h_nvis[v], ws.lazy && vnrx[v] >= LAZY_MIN_RX ? 1 : 0);
    }
    ws.n_items = (int)item_off[V];
    if (nfar >= (1ll << 31)) return fail(ctx, RXGS_E_INVALID, "too many MLP work items");
    ws.n_items_far = (int)nfar;
    // pair-emission chunks: EM2_CHUNK visible entries of one view each; or,
    // with direct binning, the workgroups placing each view's pairs (groups of
    // up to bin_group units of BIN_WIN pair slots of one chunk): at most one
    // per BIN_WIN x bin_group of its pairs plus one per chunk of the first emission
    std::vector<uint32_t> chunk_off(V + 1, 0);
    for (int v = 0; v < V; v++) {
        const uint64_t gs = (uint64_t)BIN_WIN * (uint64_t)ws.bin_group;
        const uint64_t n = ws.direct_bins ? (ws.h_pcount[v] + gs - 1) / gs + (uint64_t)ws.em_cpv
                                          : (uint64_t)((ws.h_nvis[v] + EM2_CHUNK - 1) / EM2_CHUNK);
        if ((uint64_t)chunk_off[v] + n >= (1ull << 31)) return fail(ctx, RXGS_E_INVALID, "too many pair-emission chunks");
        chunk_off[v + 1] = chunk_off[v] + (uint32_t)n;
    }
    ws.n_emit_chunks = (int)chunk_off[V];

    const size_t P = (size_t)g.H * g.W;
    WGROW(ctx, ws, ws.pval[0], std::max<uint64_t>(Dpad, 1) * 4);
    if (!ws.direct_bins) {
        WGROW(ctx, ws, ws.pkey[0], std::max<uint64_t>(Dpad, 1) * 4);
        WGROW(ctx, ws, ws.pkey[1], std::max<uint64_t>(Dpad, 1) * 4);
        WGROW(ctx, ws, ws.pval[1], std::max<uint64_t>(Dpad, 1) * 4);
        WGROW(ctx, ws, ws.hist_b, sort_ws_bytes((uint32_t)Dpad, std::max(bits_for((uint64_t)g.tiles), 1), V));
    }
    WGROW(ctx, ws, ws.ranges, (size_t)V * g.tiles * 8);
    WGROW(ctx, ws, ws.torder, (size_t)V * g.tiles * 4);
    WGROW(ctx, ws, ws.rad, (size_t)NR * Kp * 8);
    WGROW(ctx, ws, ws.Tfin, (size_t)ws.n_tslots * P * 4);
    WGROW(ctx, ws, ws.nlast, (size_t)ws.n_tslots * P * 4);
    WGROW(ctx, ws, ws.part, (size_t)NR * g.tiles * 48);   // per sub-tile with one receiver per chunk
    if (ws.use_mlp) WGROW(ctx, ws, ws.Lp, (size_t)std::max<int64_t>(K, 1) * HID * 4);
    if (ws.use_items) WGROW(ctx, ws, ws.items, (size_t)std::max(ws.n_items, 1) * 16);
    if (rxc) WGROW(ctx, ws, ws.rloc, (size_t)N * Kp * Ch * 16);
    if (ws.lazy) {
        WGROW(ctx, ws, ws.items_live, (size_t)std::max(ws.n_items, 1) * 16);
        WGROW(ctx, ws, ws.live, live_count_offset(ws) + 64);
    }
    if (ws.mpos != 0xFFFFFFFFu) {
        WGROW(ctx, ws, ws.items_far, (size_t)std::max(ws.n_items_far, 1) * 16);
        WGROW(ctx, ws, ws.frec, (size_t)V * P * FAR_RECORDS * 8);
        WGROW(ctx, ws, ws.fcnt, (size_t)V * P);
        WGROW(ctx, ws, ws.ftile, (size_t)V * g.tiles * 4);
        WGROW(ctx, ws, ws.live, live_count_offset(ws) + 64);   // marks of the blocks records point into
    }

    // the small descriptors, packed (16-byte aligned parts) into one host-to-device copy
    auto al16 = [](size_t b) { return (b + 15) / 16 * 16; };
    const size_t o_chunks = al16((size_t)NR * 4);
    const size_t o_vinfo = o_chunks + chunks.size() * 16;
    const size_t o_ioff = o_vinfo + (size_t)V * 16;
    const size_t o_coff = o_ioff + al16((size_t)(V + 1) * 4);
    const size_t o_pbase = o_coff + al16((size_t)(V + 1) * 4);
    const size_t o_pcount = o_pbase + al16((size_t)V * 4);
    const size_t o_segtab = o_pcount + al16((size_t)V * 4);
    const size_t o_wchunks = o_segtab + segtab.size() * 16;
    const size_t stage_bytes = o_wchunks + wchunks.size() * 16;
    const size_t cnt_bytes = head_bytes;   // the counts and the emission error word
    const size_t off0 = (cnt_bytes + 63) / 64 * 64;
    if (!ensure_pinned(ws, off0 + stage_bytes + 64)) return fail(ctx, RXGS_E_OOM, "pinned allocation failed");
    WGROW(ctx, ws, ws.desc, stage_bytes);
    char *hp = static_cast<char *>(ws.h_pinned) + off0;
    std::memcpy(hp, rowview.data(), (size_t)NR * 4);
    std::memcpy(hp + o_chunks, chunks.data(), chunks.size() * 16);
    std::memcpy(hp + o_vinfo, vinfo.data(), (size_t)V * 16);
    std::memcpy(hp + o_ioff, item_off.data(), (size_t)(V + 1) * 4);
    std::memcpy(hp + o_coff, chunk_off.data(), (size_t)(V + 1) * 4);
    std::memcpy(hp + o_pbase, ws.h_pbase.data(), (size_t)V * 4);
    std::memcpy(hp + o_pcount, ws.h_pcount.data(), (size_t)V * 4);
    std::memcpy(hp + o_segtab, segtab.data(), segtab.size() * 16);
    if (!wchunks.empty()) std::memcpy(hp + o_wchunks, wchunks.data(), wchunks.size() * 16);
    char *dd = ws.desc.as<char>();
    ws.d_rxview = reinterpret_cast<int *>(dd);
    ws.d_chunks = reinterpret_cast<int4 *>(dd + o_chunks);
    ws.d_vinfo = reinterpret_cast<int4 *>(dd + o_vinfo);
    ws.d_item_off = reinterpret_cast<uint32_t *>(dd + o_ioff);
    ws.d_chunk_off = reinterpret_cast<uint32_t *>(dd + o_coff);
    ws.d_pbase = reinterpret_cast<uint32_t *>(dd + o_pbase);
    ws.d_pcount = reinterpret_cast<uint32_t *>(dd + o_pcount);
    ws.d_segtab = reinterpret_cast<int4 *>(dd + o_segtab);
    ws.d_wchunks = reinterpret_cast<int4 *>(dd + o_wchunks);
    HIPCHK(ctx, hipMemcpyAsync(dd, hp, stage_bytes, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipEventRecord(ws.staged, st));

    // pairs: placed in their tile lists directly, or emitted in depth order
    // and stably sorted by (view, tile); then the tile ranges
    int pcur = 0;
    if (D > 0 && ws.direct_bins) {
        STAGE(ctx, "emit_pairs", launch_bin_pairs(ws, g, st));
        ws.pair_bits = 0;
    } else if (D > 0) {
        // (the emission kernel also clears the pair sort's scratch)
        const int sbits = std::max(bits_for((uint64_t)g.tiles), 1);
        STAGE(ctx, "emit_pairs", launch_emit2(ws, g, sort_ws_bytes((uint32_t)Dpad, sbits, V) / 4, st));
        STAGE(ctx, "sort_pairs", sort_pairs_u32(ws.pkey, ws.pval, ws.hist_b, pcur, (uint32_t)Dpad, sbits, V, 0,
                                                ws.d_segtab, st, true));
        ws.pair_bits = sbits;
    } else {
        ws.pair_bits = 0;
    }
    ws.pairs_buf = pcur;
    STAGE(ctx, "ranges", launch_ranges(ws, g, st));

    // stage 2: radiance per (receiver, sorted position)
    if (ws.use_mlp) {
        if (!ws.items_built) STAGE(ctx, "mlp_items", launch_mlp_items(ws, st));
        if (ws.lazy) STAGE(ctx, "blend_weights", launch_blend_weights(ws, st));
        // the stored Gaussian term: for the backward, or when the pair kernel
        // cannot compute it itself
        if (save || !mlp_fused_ok(sc, ctx->mlp)) STAGE(ctx, "mlp_local", launch_mlp_local(sc, ctx->mlp, ws, st));
        STAGE(ctx, "mlp_pairs", launch_mlp_pairs(sc, ctx->mlp, ws, st));
        if (ctx->prof.on) HIPCHK(ctx, launch_count_items(ws, false, ctx->prof.dcount, st));
    } else if (rxc) {
        if (!ws.items_built) STAGE(ctx, "mlp_items", launch_mlp_items(ws, st));
        if (ws.lazy) STAGE(ctx, "blend_weights", launch_blend_weights(ws, st));
        STAGE(ctx, "rxcond_pairs", launch_rxcond_pairs(sc, ctx->rxc, ws, st, false));
        if (ctx->prof.on) HIPCHK(ctx, launch_count_items(ws, false, ctx->prof.dcount, st));
    } else {
        STAGE(ctx, "rad_direct", launch_rad_direct(sc, ws, st));
    }

    // stage 3: compositing, then the per-receiver reductions
    if (ws.mpos != 0xFFFFFFFFu && !ws.live_cleared)
        HIPCHK(ctx, launch_fill_u32(ws.live.as<uint32_t>(), 0u, (live_count_offset(ws) + 3) / 4, st));
    STAGE(ctx, "blend_fwd", launch_blend_fwd(ws, C, save, st));
    if (ws.mpos != 0xFFFFFFFFu) {
        // views that composited a position past the prefix: the rest of their
        // radiance, then their recorded terms added, or their blend again
        // (the workgroups of other tiles return at once)
        STAGE(ctx, "far_items", launch_far_items(ws, st));
        STAGE(ctx, "mlp_far", rxc ? launch_rxcond_pairs(sc, ctx->rxc, ws, st, true)
                                  : launch_mlp_pairs(sc, ctx->mlp, ws, st, true));
        if (ctx->prof.on) HIPCHK(ctx, launch_count_items(ws, true, ctx->prof.dcount, st));
        STAGE(ctx, "blend_far", launch_blend_fwd(ws, C, false, st, true));
    }
    STAGE(ctx, "reduce", launch_reduce_outputs(ws, power, csum, st));
    if (amp) STAGE(ctx, "amplitude", launch_amplitude(C, amp, NR, P, st));
    HIPCHK(ctx, hipEventRecord(ws.done, st));
    ws.scene_version = sc.version;
    ws.mlp_version = ctx->mlp.version;
    ws.rxc_version = ctx->rxc.version;
    ws.valid = !saved || save;
    return RXGS_OK;
}

// Front-to-back compositing stops at a pixel once its transmittance falls
// below the threshold (Alg. 1), so in optically thick scenes a view's result
// depends only on its nearest Gaussians.  The forward therefore emits, per
// view, only the NEAR_LIMIT nearest depth-sorted entries; a view whose every
// pixel stopped inside that prefix has exactly the result (and, its tile lists
// being prefixes of the full ones, exactly the saved state) of the full list.
// The other views are redone over all their entries: one by one without
// saved state, all of them with it.
extern "C" rxgs_status rxgs_render(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off, int N,
                                   const float *rx, float *C, float *power, float *csum, float *amp,
                                   rxgs_saved *saved, void *stream)
{
    const bool cut = ctx && ctx->scene.valid && ctx->scene.K > NEAR_LIMIT && N > 0 && ctx->near_cut;
    rxgs_status rs = render_pass(ctx, mode, Q, tx, rx_off, N, rx, C, power, csum, amp, saved, stream,
                                 cut ? (uint32_t)NEAR_LIMIT : 0xFFFFFFFFu);
    if (rs != RXGS_OK || !cut) return rs;
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Workspace &ws = saved ? saved->ws : ctx->ws;
    const int V = ws.V;
    if (ws.h_pinned_cap < (size_t)V * 4) return fail(ctx, RXGS_E_STATE, "flag staging too small");
    uint32_t *hf = static_cast<uint32_t *>(ws.h_pinned);
    HIPCHK(ctx, hipMemcpyAsync(hf, ws.vflag.p, (size_t)V * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    std::vector<int> redo;
    for (int v = 0; v < V; v++)
        if ((hf[v] & 3u) == 3u) redo.push_back(v);
    ctx->views_redone += (int64_t)redo.size();
    if (redo.empty()) return RXGS_OK;
    if (saved) return render_pass(ctx, mode, Q, tx, rx_off, N, rx, C, power, csum, amp, saved, stream, 0xFFFFFFFFu);
    const size_t P2 = (size_t)2 * ctx->g.H * ctx->g.W;
    for (int v : redo) {
        rxgs::StageMark sm_(ctx->prof, "redo_views", st);   // one launch per view redone
        int j0 = v, n = 1;
        const float *cen = nullptr;
        int32_t off[2] = {0, 1};
        if (mode == RXGS_MODE_TX) {
            j0 = rx_off[v];
            n = rx_off[v + 1] - rx_off[v];
            off[1] = n;
            cen = tx + 3 * (size_t)v;
        }
        if (n == 0) continue;
        rs = render_pass(ctx, mode, mode == RXGS_MODE_TX ? 1 : 0, cen, mode == RXGS_MODE_TX ? off : nullptr, n,
                         rx + 3 * (size_t)j0, C + P2 * j0, power ? power + j0 : nullptr,
                         csum ? csum + 2 * (size_t)j0 : nullptr, amp ? amp + P2 / 2 * j0 : nullptr, nullptr, stream,
                         0xFFFFFFFFu);
        if (rs != RXGS_OK) return rs;
    }
    return RXGS_OK;
}

// ============================================================================
// rxgs_render without allocations: the workspace is carved, in order, from
// this device's scratch array, rewound at every call; its pinned staging and
// events were made by rxgs_create.  A render that needs more than the array
// holds fails with E_OOM ("scratch region exhausted") before writing any output.
extern "C" rxgs_status rxgs_render_noalloc(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off,
                                           int N, const float *rx, float *C, float *power, float *csum, float *amp,
                                           void *stream)
{
    if (!ctx) return RXGS_E_INVALID;
    if (!ctx->noalloc || !ctx->fixed.base) return fail(ctx, RXGS_E_STATE, "no allocation-free workspace");
    Workspace &ws = ctx->noalloc->ws;
    // the last call's carve is forgotten and the region rewound (its work is
    // ordered before this call's on one stream; calls that overlap race)
    release_buffers(ws);
    ctx->fixed.used = 0;
    return render_pass(ctx, mode, Q, tx, rx_off, N, rx, C, power, csum, amp, ctx->noalloc, stream, 0xFFFFFFFFu);
}

// ============================================================================
// The paper's conditioned radiance (Sec. 4.3.2; App. E.2, E.5)

static bool rc_desc_ok(const rxgs_rxcond_desc *d)
{
    return d && (d->basis == RXGS_BASIS_FLE || d->basis == RXGS_BASIS_SH) && d->lmax >= 0 && d->lmax <= 12 &&
           d->channels >= 1 && d->channels <= 32 && d->bands >= 1 && d->bands <= 16 &&
           d->hidden == RXGS_RXCOND_HIDDEN && d->probes >= 2 && d->probes <= 64 && d->grid >= 1 && d->grid <= 512 &&
           d->reserved == 0;
}

extern "C" int64_t rxgs_rxcond_param_count(const rxgs_rxcond_desc *d)
{
    if (!rc_desc_ok(d)) return -1;
    const int L = (d->lmax + 1) * (d->lmax + 1);
    return (int64_t)rc_offsets(L, d->channels, d->bands).total;
}

extern "C" rxgs_status rxgs_rxcond_upload(rxgs_ctx *ctx, const rxgs_rxcond_desc *d, const float *coeffs,
                                          const float *params, int src_on_device, void *stream)
{
    if (!ctx) return RXGS_E_INVALID;
    if (!rc_desc_ok(d))
        return fail(ctx, RXGS_E_INVALID,
                    "invalid conditioning descriptor (basis FLE or SH, lmax 0..12, channels 1..32, bands 1..16, "
                    "hidden 64, probes 2..64, grid 1..512, reserved 0)");
    const Scene &sc = ctx->scene;
    if (!sc.valid) return fail(ctx, RXGS_E_STATE, "no scene uploaded");
    const int64_t K = sc.K;
    if (!params || (K > 0 && !coeffs)) return fail(ctx, RXGS_E_INVALID, "coefficients or parameters are NULL");
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    RxCond &m = ctx->rxc;
    m.valid = false;
    m.kind = d->basis;
    m.lmax = d->lmax;
    m.L = (d->lmax + 1) * (d->lmax + 1);
    m.C = d->channels;
    m.F = d->bands;
    m.S = d->probes;
    m.G = d->grid;
    m.off = rc_offsets(m.L, m.C, m.F);
    const int L = m.L, C = m.C, F = m.F, G = m.G, H = RXGS_RXCOND_HIDDEN;
    const size_t np = m.off.total;
    const size_t ncoef = (size_t)K * L * C * 2;
    std::vector<float> hp(np);
    if (src_on_device) {
        HIPCHK(ctx, hipMemcpyAsync(hp.data(), params, np * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    } else {
        std::memcpy(hp.data(), params, np * 4);
        if (!all_finite_host(coeffs, ncoef)) return fail(ctx, RXGS_E_INVALID, "non-finite coefficient");
    }
    if (!all_finite_host(hp.data(), np)) return fail(ctx, RXGS_E_INVALID, "non-finite conditioning parameter");
    // walk order: half 0 takes the even |m|, half 1 the odd; m ascending, then
    // the degree, (l, +m) before (l, -m)
    std::vector<int> walk;
    for (int h = 0; h < 2; h++) {
        for (int mm = h; mm <= m.lmax; mm += 2)
            for (int l = mm; l <= m.lmax; l++) {
                walk.push_back(l * l + l + mm);
                if (mm > 0) walk.push_back(l * l + l - mm);
            }
        if (h == 0) m.n0 = (int)walk.size();
    }
    // layer-1 term of each component of the global MLP, in walk order:
    // b1 + W1[:, 6F] deg / m + W1[:, 6F + 1] ord / m + W1[:, 6F + 2 ..] e_l
    const int gin = 6 * F + 2 + RXGS_RXCOND_EMB;
    const double dn = m.lmax > 0 ? (double)m.lmax : 1.0;
    std::vector<float> comp((size_t)L * H);
    for (int w = 0; w < L; w++) {
        const int idx = walk[w];
        int l = 0;
        while ((l + 1) * (l + 1) <= idx) l++;
        const int ord = idx - l * l - l;
        for (int u = 0; u < H; u++) {
            const float *row = hp.data() + m.off.g1 + (size_t)u * gin;
            double a = hp[m.off.gb1 + u];
            a += (double)row[6 * F] * ((double)l / dn);
            a += (double)row[6 * F + 1] * ((double)ord / dn);
            for (int e = 0; e < RXGS_RXCOND_EMB; e++)
                a += (double)row[6 * F + 2 + e] * (double)hp[m.off.e + (size_t)idx * RXGS_RXCOND_EMB + e];
            comp[(size_t)w * H + u] = (float)a;
        }
    }
    // orthonormal factors and the recurrence constants of the associated
    // Legendre functions, per (l, m)
    std::vector<float> ctab(13 * 13 * 4, 0.f);
    for (int l = 0; l <= 12; l++)
        for (int mm = 0; mm <= l; mm++) {
            double r = (2.0 * l + 1.0) / (4.0 * M_PI);
            for (int i = l - mm + 1; i <= l + mm; i++) r /= (double)i;
            float *t = &ctab[(l * 13 + mm) * 4];
            t[0] = (float)std::sqrt(r);
            if (l > mm) {
                t[1] = (float)((2.0 * l - 1.0) / (double)(l - mm));
                t[2] = (float)((double)(l + mm - 1) / (double)(l - mm));
            }
        }
    // the local MLP's W2 in the FP32 MFMA A-operand layout
    std::vector<float> w2t(2 * 32 * 64);
    for (int b = 0; b < 2; b++)
        for (int t = 0; t < 32; t++)
            for (int lane = 0; lane < 64; lane++)
                w2t[(b * 32 + t) * 64 + lane] = hp[m.off.l2 + (size_t)(32 * b + lane % 32) * H + 2 * t + lane / 32];
    std::vector<double> tp(m.S);
    for (int i = 0; i < m.S; i++) {
        double t = 0.9 * (double)i;
        t = t / (double)(m.S - 1);
        tp[i] = 0.05 + t;
    }
    GROW(ctx, m.params, np * 4);
    GROW(ctx, m.comp, comp.size() * 4);
    GROW(ctx, m.walk, (size_t)L * 4);
    GROW(ctx, m.ctab, ctab.size() * 4);
    GROW(ctx, m.w2t, w2t.size() * 4);
    GROW(ctx, m.tprobe, tp.size() * 8);
    GROW(ctx, m.coef, std::max<size_t>(ncoef, 2) * 4);
    GROW(ctx, m.occ, (size_t)G * G * G * 4);
    HIPCHK(ctx, hipMemcpyAsync(m.params.p, hp.data(), np * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.comp.p, comp.data(), comp.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.walk.p, walk.data(), (size_t)L * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.ctab.p, ctab.data(), ctab.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.w2t.p, w2t.data(), w2t.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(m.tprobe.p, tp.data(), tp.size() * 8, hipMemcpyHostToDevice, st));
    // coefficients into walk order (through the staging buffer from the host)
    DevBuf tmp;
    const size_t n3 = (size_t)G * G * G;
    if (!grow(tmp, std::max<size_t>(n3 * 8, 64), &ctx->alloc)) return fail(ctx, RXGS_E_OOM, "occupancy accumulator");
    struct TmpGuard {
        DevBuf &b;
        ~TmpGuard() { release(b); }
    } guard{tmp};
    unsigned *words = tmp.as<unsigned>();   // first used for the checks and the bounds
    if (K > 0) {
        const float *src = coeffs;
        if (!src_on_device) {
            GROW(ctx, ctx->stage, ncoef * 4);
            HIPCHK(ctx, hipMemcpyAsync(ctx->stage.p, coeffs, ncoef * 4, hipMemcpyHostToDevice, st));
            src = ctx->stage.as<float>();
        } else {
            HIPCHK(ctx, hipMemsetAsync(words, 0, 4, st));
            const unsigned blocks = (unsigned)std::min<size_t>((ncoef + BLOCK - 1) / BLOCK, 2048);
            hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks), dim3(BLOCK), 0, st, coeffs, ncoef, words);
            HIPCHK(ctx, hipGetLastError());
            unsigned bad = 0;
            HIPCHK(ctx, hipMemcpyAsync(&bad, words, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(ctx, hipStreamSynchronize(st));
            if (bad) return fail(ctx, RXGS_E_INVALID, "non-finite coefficient");
        }
        HIPCHK(ctx, launch_rc_coef_perm(src, K, m, st));
    }
    // occupancy grid over the box of the means
    unsigned keys[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
    if (K > 0) {
        HIPCHK(ctx, hipMemcpyAsync(words, keys, 24, hipMemcpyHostToDevice, st));
        HIPCHK(ctx, launch_rc_bounds(sc, words, st));
        HIPCHK(ctx, hipMemcpyAsync(keys, words, 24, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    }
    for (int a = 0; a < 3; a++) {
        m.lo[a] = K > 0 ? (double)rc_key_value(keys[a]) : 0.0;
        m.hi[a] = K > 0 ? (double)rc_key_value(keys[3 + a]) : 0.0;
        if (!(m.hi[a] - m.lo[a] >= 1e-6)) m.hi[a] = m.lo[a] + 1e-6;
        m.vs[a] = (m.hi[a] - m.lo[a]) / G;
        m.inv[a] = (double)G / (m.hi[a] - m.lo[a]);
    }
    unsigned long long *acc = tmp.as<unsigned long long>();
    HIPCHK(ctx, hipMemsetAsync(acc, 0, n3 * 8, st));
    HIPCHK(ctx, launch_rc_splat(sc, m, acc, st));
    HIPCHK(ctx, launch_rc_finish(m, acc, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    m.version = ++ctx->version_counter;
    m.scene_version = sc.version;
    m.valid = true;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_rxcond_export(rxgs_ctx *ctx, int what, void *dst, int64_t bytes, int dst_on_device)
{
    if (!ctx) return RXGS_E_INVALID;
    if (!dst || bytes < 0) return fail(ctx, RXGS_E_INVALID, "NULL destination");
    const RxCond &m = ctx->rxc;
    if (!m.valid) return fail(ctx, RXGS_E_STATE, "no conditioning model");
    DeviceScope ds(ctx->device);
    if (what == RXGS_RXCOND_BOX) {
        if (bytes < 48) return fail(ctx, RXGS_E_INVALID, "destination too small");
        double box[6] = {m.lo[0], m.lo[1], m.lo[2], m.hi[0], m.hi[1], m.hi[2]};
        if (dst_on_device) HIPCHK(ctx, aux_copy(ctx, dst, box, 48, hipMemcpyHostToDevice));
        else std::memcpy(dst, box, 48);
        return RXGS_OK;
    }
    if (what != RXGS_RXCOND_OCCUPANCY) return fail(ctx, RXGS_E_INVALID, "unknown export");
    const size_t n = (size_t)m.G * m.G * m.G * 4;
    if ((size_t)bytes < n) return fail(ctx, RXGS_E_INVALID, "destination too small");
    HIPCHK(ctx, aux_copy(ctx, dst, m.occ.p, n, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_render_rxcond(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off,
                                          int N, const float *rx, float *C, float *power, float *csum, float *amp,
                                          rxgs_saved *saved, void *stream)
{
    return render_pass(ctx, mode, Q, tx, rx_off, N, rx, C, power, csum, amp, saved, stream, 0xFFFFFFFFu,
                       RSRC_RXCOND);
}

// ============================================================================
extern "C" rxgs_status rxgs_render_chunked(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off,
                                           int N, const float *rx, float *C, float *power, float *csum, float *amp,
                                           int64_t budget_bytes, int32_t *n_chunks, void *stream)
{
    if (!ctx) return RXGS_E_INVALID;
    if (mode != RXGS_MODE_TX && mode != RXGS_MODE_RX) return fail(ctx, RXGS_E_INVALID, "unknown mode");
    if (N < 0) return fail(ctx, RXGS_E_INVALID, "N < 0");
    if (n_chunks) *n_chunks = 0;
    if (N == 0) return RXGS_OK;
    if (!rx || !C) return fail(ctx, RXGS_E_INVALID, "rx or C is NULL");
    if (!ctx->scene.valid) return fail(ctx, RXGS_E_STATE, "no scene uploaded");
    std::vector<int> owner(N, 0);   // transmitter of each receiver (TX mode)
    if (mode == RXGS_MODE_TX) {
        if (Q < 1 || !tx || !rx_off) return fail(ctx, RXGS_E_INVALID, "TX mode needs Q >= 1, tx and rx_off");
        if (rx_off[0] != 0 || rx_off[Q] != N) return fail(ctx, RXGS_E_INVALID, "rx_off must run from 0 to N");
        for (int q = 0; q < Q; q++) {
            if (rx_off[q + 1] < rx_off[q]) return fail(ctx, RXGS_E_INVALID, "rx_off must be non-decreasing");
            for (int j = rx_off[q]; j < rx_off[q + 1]; j++) owner[j] = q;
        }
    }
    if (budget_bytes <= 0) {
        DeviceScope ds(ctx->device);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return hip_fail(ctx, hipGetLastError(), "hipMemGetInfo");
        budget_bytes = (int64_t)(free_b / 2);
    }
    const int64_t K = ctx->scene.K;
    const int H = ctx->g.H, W = ctx->g.W;
    const size_t P2 = (size_t)2 * H * W;
    int32_t chunks = 0;
    for (int a = 0; a < N;) {
        // transmitters the chunk [a, b) spans
        auto views_of = [&](int b) { return mode == RXGS_MODE_TX ? owner[b - 1] - owner[a] + 1 : 0; };
        auto fits = [&](int b) {
            return rxgs_workspace_estimate(mode, views_of(b), b - a, K, H, W) <= budget_bytes;
        };
        if (!fits(a + 1)) return fail(ctx, RXGS_E_OOM, "one receiver's workspace exceeds the budget");
        int lo = a + 1, hi = N;   // largest b in [lo, hi] that fits (the estimate grows with b)
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (fits(mid)) lo = mid;
            else hi = mid - 1;
        }
        const int b = lo;
        rxgs_status rs;
        if (mode == RXGS_MODE_TX) {
            const int q0 = owner[a], q1 = owner[b - 1];
            std::vector<int32_t> off(q1 - q0 + 2);
            off[0] = 0;
            for (int q = q0; q <= q1; q++) off[q - q0 + 1] = std::min(rx_off[q + 1], b) - a;
            rs = rxgs_render(ctx, mode, q1 - q0 + 1, tx + 3 * (size_t)q0, off.data(), b - a, rx + 3 * (size_t)a,
                             C + P2 * a, power ? power + a : nullptr, csum ? csum + 2 * (size_t)a : nullptr,
                             amp ? amp + P2 / 2 * a : nullptr, nullptr, stream);
        } else {
            rs = rxgs_render(ctx, mode, 0, nullptr, nullptr, b - a, rx + 3 * (size_t)a, C + P2 * a,
                             power ? power + a : nullptr, csum ? csum + 2 * (size_t)a : nullptr,
                             amp ? amp + P2 / 2 * a : nullptr, nullptr, stream);
        }
        if (rs != RXGS_OK) return rs;
        chunks++;
        a = b;
    }
    if (n_chunks) *n_chunks = chunks;
    return RXGS_OK;
}

// ============================================================================
// The deterministic backward: the blend backward stores one partial per
// (pair, receiver block) at the pair's emission slot instead of adding
// atomically; gathers add them per (view, position) and per (row, position)
// in emission order, the MLP backward's terms
// per Gaussian and per receiver in view and block order, and the projection
// gradients per Gaussian over the views in order.  The outputs are written
// (or added, accumulate = 1) once each.
static rxgs_status backward_det(rxgs_ctx *ctx, Workspace &ws, const float *C, const float *dC, const float *dP,
                                const float *dA, const rxgs_grads &gr, ZeroRanges &zr, hipStream_t st)
{
    const Scene &sc = ctx->scene;
    const int64_t K = ws.K;
    const bool accum = gr.accumulate == 1;
    const size_t VK = (size_t)ws.V * ws.Kp;
    const int Rd = det_block_rows(ws);
    const size_t nblk = (size_t)(ws.R_max + Rd - 1) / Rd;
    const size_t Dp = (size_t)std::max<int64_t>(ws.Dpad, 1);
    zr.n = 0;   // outputs are written, not accumulated into
    WGROW(ctx, ws, ws.dS, (size_t)ws.N * ws.Kp * 8);
    WGROW(ctx, ws, ws.g2d, VK * 32);
    WGROW(ctx, ws, ws.live, VK / MLP_PAIRS + 4);
    WGROW(ctx, ws, ws.gP, nblk * Dp * 32);
    WGROW(ctx, ws, ws.dSP, (size_t)ws.R_max * Dp * 8);
    WGROW(ctx, ws, ws.oinv, (size_t)ws.V * std::max<int64_t>(K, 1) * 4);
    zr.add(ws.live.p, (VK / MLP_PAIRS + 3) / 4);
    zr.add(ws.gP.p, nblk * Dp * 8);
    zr.add(ws.dSP.p, (size_t)ws.R_max * Dp * 2);
    float *gfeat = gr.features, *gmlp = gr.mlp;
    if (ws.use_mlp) {
        WGROW(ctx, ws, ws.dL, (size_t)K * HID * 4);
        WGROW(ctx, ws, ws.dG, (size_t)ws.N * HID * 4);
        WGROW(ctx, ws, ws.mpart, mlp_part_bytes(ws));
        WGROW(ctx, ws, ws.w1part, w1b_part_bytes(K));
        WGROW(ctx, ws, ws.mred, mlp_red_bytes());
        WGROW(ctx, ws, ws.rank, (VK / MLP_PAIRS + 1) * 4);
        WGROW(ctx, ws, ws.lcnt, live_rank_words(ws) * 4);
        if (accum && gfeat) {
            WGROW(ctx, ws, ws.gfeat_tmp, (size_t)K * FEAT * 4);
            gfeat = ws.gfeat_tmp.as<float>();
        }
        if (accum && gmlp) {
            WGROW(ctx, ws, ws.gmlp_tmp, (size_t)RXGS_MLP_NPARAM * 4);
            gmlp = ws.gmlp_tmp.as<float>();
        }
    }
    HIPCHK(ctx, launch_zero_ranges(zr, st));
    HIPCHK(ctx, launch_fill_u32(ws.oinv.as<uint32_t>(), 0xFFFFFFFFu, (size_t)ws.V * K, st));
    STAGE(ctx, "blend_bwd", launch_blend_bwd(ws, C, dC, dP, dA, st));
    STAGE(ctx, "bwd_misc", launch_det_gather(ws, st));
    if (ws.use_mlp) {
        // one slot per marked position block, in index order
        HIPCHK(ctx, launch_live_rank(ws, st));
        if (!ensure_pinned(ws, 64)) return fail(ctx, RXGS_E_OOM, "pinned allocation failed");
        const size_t nchunk = live_rank_words(ws) - 1;
        HIPCHK(ctx, hipMemcpyAsync(ws.h_pinned, ws.lcnt.as<uint32_t>() + nchunk, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        const size_t nslot = std::max<uint32_t>(*static_cast<uint32_t *>(ws.h_pinned), 1u);
        const size_t nrg = (size_t)(ws.R_max + MLP_RG - 1) / MLP_RG;
        WGROW(ctx, ws, ws.dLv, nslot * nrg * MLP_PAIRS * HID * 4);
        WGROW(ctx, ws, ws.dGp, nslot * (size_t)ws.R_max * HID * 4);
        HIPCHK(ctx, launch_fill_u32(ws.dGp.as<uint32_t>(), 0u, nslot * (size_t)ws.R_max * HID, st));
        STAGE(ctx, "mlp_bwd", launch_mlp_bwd(sc, ctx->mlp, ws, gfeat, gmlp, st));
    } else {
        STAGE(ctx, "bwd_misc", launch_det_rad(sc, ws, gr.radiance, gr.accumulate, st));
    }
    STAGE(ctx, "project_bwd", launch_det_project(sc, ws, gr, st));
    if (accum && ws.use_mlp) {
        if (gr.features) HIPCHK(ctx, launch_add_f32(gr.features, gfeat, (size_t)K * FEAT, st));
        if (gr.mlp) HIPCHK(ctx, launch_add_f32(gr.mlp, gmlp, RXGS_MLP_NPARAM, st));
    }
    if (ws.done) HIPCHK(ctx, hipEventRecord(ws.done, st));
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_set_deterministic(rxgs_ctx *ctx, int on)
{
    if (!ctx) return RXGS_E_INVALID;
    ctx->deterministic = on != 0;
    return RXGS_OK;
}

// ============================================================================
extern "C" rxgs_status rxgs_render_backward(rxgs_ctx *ctx, const rxgs_saved *saved, const float *C, const float *dC,
                                            const float *dP, const float *dA, const rxgs_grads *grads, void *stream)
{
    if (!ctx) return RXGS_E_INVALID;
    if (!saved || !grads) return fail(ctx, RXGS_E_INVALID, "saved or grads is NULL");
    if (saved->ctx != ctx) return fail(ctx, RXGS_E_INVALID, "saved state of another context");
    // the backward uses scratch buffers of the saved state: calls on one saved state must not overlap
    Workspace &ws = const_cast<rxgs_saved *>(saved)->ws;
    if (ws.valid && ws.rsrc == RSRC_RXCOND)
        return fail(ctx, RXGS_E_STATE, "no backward through the conditioned radiance: the state is for exports only");
    const Scene &sc = ctx->scene;
    if (!ws.valid) return fail(ctx, RXGS_E_STATE, "no forward state in saved");
    if (ws.scene_version != sc.version || (ws.use_mlp && ws.mlp_version != ctx->mlp.version))
        return fail(ctx, RXGS_E_STATE, "scene or MLP changed since the forward");
    if (ws.N > 0 && !C) return fail(ctx, RXGS_E_INVALID, "C is NULL");
    if (grads->accumulate != 0 && grads->accumulate != 1) return fail(ctx, RXGS_E_INVALID, "accumulate must be 0 or 1");
    DeviceScope ds(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const rxgs_grads &gr = *grads;
    const bool accum = gr.accumulate == 1;
    const int64_t K = ws.K;
    // gradients accumulate with atomics: clear them first (unless the caller
    // asked to add into its buffers)
    struct {
        float *p;
        size_t n;
    } outs[] = {{gr.means, (size_t)K * 3}, {gr.log_scales, (size_t)K * 3}, {gr.quats, (size_t)K * 4},
                {gr.logits, (size_t)K},   {ws.use_mlp ? nullptr : gr.radiance, (size_t)K * 2}};
    // (one launch zeroes the outputs and, below, the backward's accumulators)
    ZeroRanges zr;
    if (!accum)
        for (auto &o : outs) zr.add(o.p, o.n);
    if (ws.N == 0 || K == 0) {
        if (accum) return RXGS_OK;   // nothing to add
        HIPCHK(ctx, launch_zero_ranges(zr, st));
        if (ws.use_mlp && gr.features) HIPCHK(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(gr.features), 0u, (size_t)K * FEAT, st));
        if (ws.use_mlp && gr.mlp) HIPCHK(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(gr.mlp), 0u, RXGS_MLP_NPARAM, st));
        return RXGS_OK;
    }
    const size_t VK = (size_t)ws.V * ws.Kp;
    if (ws.det) return backward_det(ctx, ws, C, dC, dP, dA, gr, zr, st);
    WGROW(ctx, ws, ws.dS, (size_t)ws.N * ws.Kp * 8);
    WGROW(ctx, ws, ws.g2d, VK * 32);
    WGROW(ctx, ws, ws.live, VK / MLP_PAIRS + 4);
    // dL/ds and the 2-D record gradients are written and read at visible
    // positions only; when they are large, only those are cleared
    const bool rows = VK * 32 > zero_visible_min() && ws.N <= 65535 && ws.V <= 65535;
    if (rows) {
        const unsigned long long *cnt = ws.counters.as<unsigned long long>();
        HIPCHK(ctx, launch_zero_visible(ws.dS.as<uint32_t>(), ws.Kp, 2, cnt, ws.d_rxview, ws.N, st));
        HIPCHK(ctx, launch_zero_visible(ws.g2d.as<uint32_t>(), ws.Kp, 8, cnt, nullptr, ws.V, st));
    } else {
        zr.add(ws.dS.p, (size_t)ws.N * ws.Kp * 2);
        zr.add(ws.g2d.p, VK * 8);
    }
    zr.add(ws.live.p, (VK / MLP_PAIRS + 3) / 4);
    WGROW(ctx, ws, ws.pterm, (size_t)K * PROJ_TERM_BYTES);
    WGROW(ctx, ws, ws.pacc, (size_t)K * PACC_STRIDE * 4);
    zr.add(ws.pacc.p, (size_t)K * PACC_STRIDE);
    if (ws.use_mlp) {
        WGROW(ctx, ws, ws.dL, (size_t)K * HID * 4);
        WGROW(ctx, ws, ws.dG, (size_t)ws.N * HID * 4);
        WGROW(ctx, ws, ws.mpart, mlp_part_bytes(ws));
        WGROW(ctx, ws, ws.w1part, w1b_part_bytes(K));
        WGROW(ctx, ws, ws.mred, mlp_red_bytes());
        zr.add(ws.dL.p, (size_t)K * HID);
        zr.add(ws.dG.p, (size_t)ws.N * HID);
    }
    // features and MLP gradients are stored, not added, by their kernels: to
    // accumulate, they go to scratch first and are added afterwards
    float *gfeat = gr.features, *gmlp = gr.mlp;
    if (accum && ws.use_mlp) {
        if (gfeat) {
            WGROW(ctx, ws, ws.gfeat_tmp, (size_t)K * FEAT * 4);
            gfeat = ws.gfeat_tmp.as<float>();
        }
        if (gmlp) {
            WGROW(ctx, ws, ws.gmlp_tmp, (size_t)RXGS_MLP_NPARAM * 4);
            gmlp = ws.gmlp_tmp.as<float>();
        }
    }
    HIPCHK(ctx, launch_zero_ranges(zr, st));
    STAGE(ctx, "blend_bwd", launch_blend_bwd(ws, C, dC, dP, dA, st));
    if (ws.use_mlp)
        STAGE(ctx, "mlp_bwd", launch_mlp_bwd(sc, ctx->mlp, ws, gfeat, gmlp, st));
    else
        STAGE(ctx, "bwd_misc", launch_rad_bwd(sc, ws, gr.radiance, st));
    STAGE(ctx, "project_bwd", launch_project_bwd(sc, ws, gr, st));
    if (accum && ws.use_mlp) {
        if (gr.features) HIPCHK(ctx, launch_add_f32(gr.features, gfeat, (size_t)K * FEAT, st));
        if (gr.mlp) HIPCHK(ctx, launch_add_f32(gr.mlp, gmlp, RXGS_MLP_NPARAM, st));
    }
    if (ws.done) HIPCHK(ctx, hipEventRecord(ws.done, st));
    return RXGS_OK;
}

// ============================================================================
extern "C" rxgs_status rxgs_saved_info(const rxgs_saved *s, rxgs_saved_info_t *out)
{
    if (!s || !out) return RXGS_E_INVALID;
    const Workspace &ws = s->ws;
    if (!ws.valid) return RXGS_E_STATE;
    out->K = ws.K;
    out->K_pad = ws.Kp;
    out->V = ws.V;
    out->N = ws.N;
    out->D = ws.D;
    out->n_visible = ws.nvis_total;
    out->tiles = ws.g.tiles;
    out->tiles_x = ws.g.tiles_x;
    // composited-pair statistics of the forward: wait for it (its own event,
    // not the device), then sum the slots
    rxgs_ctx *ctx = s->ctx;
    DeviceScope dsc(ctx->device);
    if (wait_workspace(ws) != hipSuccess) return hip_fail(ctx, hipGetLastError(), "saved info: wait");
    std::vector<unsigned long long> h(4 * STAT_SLOTS);
    Workspace &w = const_cast<Workspace &>(ws);
    HIPCHK(ctx, aux_copy(ctx, h.data(), stat_words(w), h.size() * 8, hipMemcpyDeviceToHost));
    out->n_composited_px = out->n_composited = out->n_evaluated_px = out->n_walked_px = 0;
    for (int i = 0; i < STAT_SLOTS; i++) {
        out->n_composited_px += (int64_t)h[i];
        out->n_composited += (int64_t)h[STAT_SLOTS + i];
        out->n_evaluated_px += (int64_t)h[2 * STAT_SLOTS + i];
        out->n_walked_px += (int64_t)h[3 * STAT_SLOTS + i];
    }
    out->workspace_bytes = (int64_t)ws.req_bytes;
    out->n_sort_fallbacks = 0;
    const uint32_t *fw[2] = {sort_fallback_word(w.hist, (uint32_t)((size_t)ws.V * ws.Kp), 32, ws.V),
                             sort_fallback_word(w.hist_b, (uint32_t)ws.Dpad, ws.pair_bits, ws.V)};
    for (const uint32_t *p : fw) {
        if (!p) continue;
        uint32_t c = 0;
        HIPCHK(ctx, aux_copy(ctx, &c, p, 4, hipMemcpyDeviceToHost));
        out->n_sort_fallbacks += c;
    }
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_saved_export(const rxgs_saved *s, int what, void *dst, int64_t bytes, int dst_on_device)
{
    if (!s || !dst || bytes < 0) return RXGS_E_INVALID;
    const Workspace &ws = s->ws;
    rxgs_ctx *ctx = s->ctx;
    if (!ws.valid) return fail(ctx, RXGS_E_STATE, "no forward state");
    const size_t VK = (size_t)ws.V * ws.Kp;
    const size_t P = (size_t)ws.g.H * ws.g.W;
    if ((what == RXGS_EXPORT_BIN || what == RXGS_EXPORT_KEYS || what == RXGS_EXPORT_OPACITY) && !ws.exports_ready) {
        // computed from the saved view centres and the scene's projection
        // terms (a cached part of the state, hence the cast)
        if (ws.scene_version != ctx->scene.version)
            return fail(ctx, RXGS_E_STATE, "scene changed since the forward");
        Workspace &w = const_cast<Workspace &>(ws);
        DeviceScope ds0(ctx->device);
        WGROW(ctx, w, w.ext, VK * 16);
        WGROW(ctx, w, w.rawkey, VK * 4);
        WGROW(ctx, w, w.opac, VK * 4);
        hipStream_t a = nullptr;
        HIPCHK(ctx, aux_stream(ctx, a));
        HIPCHK(ctx, wait_workspace(ws));   // the render, on the caller's stream
        HIPCHK(ctx, launch_project_exports(w, a));
        HIPCHK(ctx, hipStreamSynchronize(a));
        w.exports_ready = true;
    }
    const void *src = nullptr;
    size_t n = 0;
    std::vector<int> tmp;
    switch (what) {
    case RXGS_EXPORT_BIN: src = ws.ext.p; n = VK * 16; break;
    case RXGS_EXPORT_KEYS: src = ws.rawkey.p; n = VK * 4; break;
    case RXGS_EXPORT_OPACITY: src = ws.opac.p; n = VK * 4; break;
    case RXGS_EXPORT_ORDER: src = ws.vorder.p; n = VK * 4; break;
    case RXGS_EXPORT_NVIS:
        tmp = ws.h_nvis;
        src = tmp.data();
        n = tmp.size() * 4;
        break;
    case RXGS_EXPORT_PAIRS: n = (size_t)ws.D * 4; break;
    case RXGS_EXPORT_RANGES: n = (size_t)ws.V * ws.g.tiles * 8; break;
    case RXGS_EXPORT_RADIANCE: src = ws.rad.p; n = (size_t)ws.N * ws.Kp * 8; break;
    case RXGS_EXPORT_TFINAL: src = ws.Tfin.p; n = (size_t)ws.n_tslots * P * 4; break;
    case RXGS_EXPORT_NLAST: src = ws.nlast.p; n = (size_t)ws.n_tslots * P * 4; break;
    case RXGS_EXPORT_RECORDS: src = ws.srec.p; n = VK * 32; break;
    default: return fail(ctx, RXGS_E_INVALID, "unknown export");
    }
    if ((size_t)bytes < n) return fail(ctx, RXGS_E_INVALID, "destination too small");
    if (n == 0) return RXGS_OK;
    DeviceScope ds(ctx->device);
    if (what == RXGS_EXPORT_RADIANCE && !ws.rad_complete) {
        // the prefix render evaluated only the radiance the blend needed:
        // evaluate the rest (it completes a cached part of the state; nothing
        // the state describes changes, hence the cast)
        const bool rxc = ws.rsrc == RSRC_RXCOND;
        if (ws.scene_version != ctx->scene.version ||
            (rxc ? ws.rxc_version != ctx->rxc.version || !ctx->rxc.valid : ws.mlp_version != ctx->mlp.version))
            return fail(ctx, RXGS_E_STATE, "scene or radiance model changed since the forward");
        Workspace &w = const_cast<Workspace &>(ws);
        hipStream_t a = nullptr;
        HIPCHK(ctx, aux_stream(ctx, a));
        HIPCHK(ctx, wait_workspace(ws));   // the render, on the caller's stream
        HIPCHK(ctx, launch_far_all(w, a));
        HIPCHK(ctx, launch_far_items(w, a));
        if (rxc) HIPCHK(ctx, launch_rxcond_pairs(ctx->scene, ctx->rxc, w, a, true));
        else HIPCHK(ctx, launch_mlp_pairs(ctx->scene, ctx->mlp, w, a, true));
        HIPCHK(ctx, hipStreamSynchronize(a));
        w.rad_complete = true;
    }
    HIPCHK(ctx, wait_workspace(ws));
    if (what == RXGS_EXPORT_PAIRS || what == RXGS_EXPORT_RANGES) {
        // pairs without the per-view padding, ranges in those compact indices
        std::vector<uint32_t> hv((size_t)ws.Dpad);
        std::vector<uint32_t> out;
        if (ws.Dpad) HIPCHK(ctx, aux_copy(ctx, hv.data(), ws.pval[ws.pairs_buf].p, hv.size() * 4, hipMemcpyDeviceToHost));
        if (what == RXGS_EXPORT_PAIRS) {
            // each view's pairs are the first pcount entries of its segment
            // (the sort does not write the padding slots)
            out.reserve((size_t)ws.D);
            for (int v = 0; v < ws.V; v++)
                for (uint32_t i = 0; i < ws.h_pcount[v]; i++) out.push_back(hv[(size_t)ws.h_pbase[v] + i]);
        } else {
            std::vector<uint32_t> rg((size_t)ws.V * ws.g.tiles * 2);
            HIPCHK(ctx, aux_copy(ctx, rg.data(), ws.ranges.p, rg.size() * 4, hipMemcpyDeviceToHost));
            uint32_t cbase = 0;
            for (int v = 0; v < ws.V; v++) {
                for (int t = 0; t < ws.g.tiles; t++) {
                    uint32_t *r = &rg[((size_t)v * ws.g.tiles + t) * 2];
                    if (r[1] > r[0]) {
                        r[0] = r[0] - ws.h_pbase[v] + cbase;
                        r[1] = r[1] - ws.h_pbase[v] + cbase;
                    }
                }
                cbase += ws.h_pcount[v];
            }
            out.swap(rg);
        }
        if (out.size() * 4 != n) return fail(ctx, RXGS_E_STATE, "pair export size mismatch");
        if (dst_on_device)
            HIPCHK(ctx, aux_copy(ctx, dst, out.data(), n, hipMemcpyHostToDevice));
        else
            std::memcpy(dst, out.data(), n);
        return RXGS_OK;
    }
    if (what == RXGS_EXPORT_NVIS) {
        if (dst_on_device)
            HIPCHK(ctx, aux_copy(ctx, dst, src, n, hipMemcpyHostToDevice));
        else
            std::memcpy(dst, src, n);
        return RXGS_OK;
    }
    HIPCHK(ctx, aux_copy(ctx, dst, src, n, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return RXGS_OK;
}
