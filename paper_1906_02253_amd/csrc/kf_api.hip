// C-ABI entry points of libkfmi.so: argument validation, context and
// workspace management, dispatch to the kernel launchers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>

#include "kf_find.hpp"
#include "kf_mlp_api.hpp"

namespace {

thread_local std::string g_err;

int fail(kf_ctx* ctx, int code, const char* fmt, ...)
    __attribute__((format(printf, 3, 4)));

int fail(kf_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_err = buf;
    return code;
}

int hip_fail(kf_ctx* ctx, hipError_t e, const char* where)
{
    return fail(ctx, KF_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool bad_ld(int64_t n, int64_t ld) { return n < 0 || ld < n || (ld % 64) != 0; }

int check_tracks(kf_ctx* ctx, const kf_tracks* t, const char* what)
{
    if (!t) return fail(ctx, KF_EINVAL, "%s: null track descriptor", what);
    if (bad_ld(t->n, t->ld))
        return fail(ctx, KF_EINVAL, "%s: need 0 <= n <= ld and ld %% 64 == 0 (n=%lld ld=%lld)", what,
                    (long long)t->n, (long long)t->ld);
    if (t->n > 0 && (!t->par || !t->cov || !t->chi2 || !t->ndf || !t->status))
        return fail(ctx, KF_EINVAL, "%s: null track array", what);
    return KF_OK;
}

int check_hits(kf_ctx* ctx, const kf_hits* h, const char* what)
{
    if (!h) return fail(ctx, KF_EINVAL, "%s: null hit descriptor", what);
    if (h->n < 0) return fail(ctx, KF_EINVAL, "%s: negative hit count", what);
    if (h->n > 0 && (!h->x || !h->y || !h->z || !h->su || !h->sv || !h->layer))
        return fail(ctx, KF_EINVAL, "%s: null hit array", what);
    return KF_OK;
}

}  // namespace

namespace kfmi {

void* Workspace::get(size_t need)
{
    if (need <= bytes && ptr) return ptr;
    release();
    size_t cap = need < (1u << 20) ? (1u << 20) : need + need / 4;
    if (hipMalloc(&ptr, cap) != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        return nullptr;
    }
    bytes = cap;
    return ptr;
}

void Workspace::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}


// Validated, laid-out finding pass: the phases enqueue from this.
struct FindLaunch {
    FindPlan pl;
    FindArgs a;
    int W = 0, grid = 0, prec = 0, largest_first = 0;
    bool learn = false;
    bool clean = false;
    bool dedup = false;
    int32_t* out_hits = nullptr;
    kf_tracks* out = nullptr;
    int64_t n_events = 0;
    const int32_t* seed_hits = nullptr;
    const int32_t* event_off = nullptr;
    const int32_t* seed_event = nullptr;
    const kf_hits* hits = nullptr;
    const kf_tracks* seeds = nullptr;
};

}  // namespace kfmi

namespace {

// Checks the arguments of a finding pass, sizes and takes the workspace and
// fills `L`.  Returns KF_OK or an error code (message set).
int prepare_find(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                 const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
                 int32_t* out_hits, kf_tracks* out, uint64_t* counters, int flags, const char* what,
                 kfmi::FindLaunch* L, void* fixed_ws = nullptr, size_t fixed_bytes = 0)
{
    int r = check_tracks(ctx, seeds, what);
    if (r) return r;
    r = check_tracks(ctx, out, what);
    if (r) return r;
    r = check_hits(ctx, hits, what);
    if (r) return r;
    const int prec = flags & KF_PREC_MASK;
    if (prec == KF_PREC_FP64)
        return fail(ctx, KF_EUNSUPPORTED, "%s: float storage only (MIXED or FP32)", what);
    if (prec != KF_PREC_MIXED && prec != KF_PREC_FP32)
        return fail(ctx, KF_EINVAL, "%s: bad precision flag", what);
    const bool field = ctx->params.field_z0 > 0.0;
    const bool learn = (flags & KF_INIT_MLP) != 0;
    if (learn && !ctx->mlp_loaded) return fail(ctx, KF_EUNSUPPORTED, "%s: no learned model loaded", what);
    if (learn && ctx->d_steer)
        return fail(ctx, KF_EUNSUPPORTED, "%s: steering and the learned guess exclude each other", what);
    if (learn && ctx->find_width < 64)
        return fail(ctx, KF_EUNSUPPORTED, "%s: the learned guess needs a width of at least 64", what);
    if (out->n != seeds->n) return fail(ctx, KF_EINVAL, "%s: out->n must equal seeds->n", what);
    if (n_events < 1 || !event_off) return fail(ctx, KF_EINVAL, "%s: need n_events >= 1 and event_off", what);
    if (hits->n > 0x7fffffffLL) return fail(ctx, KF_EINVAL, "%s: at most 2^31-1 hits", what);
    if (seeds->n > 0x7fffffffLL) return fail(ctx, KF_EINVAL, "%s: at most 2^31-1 seeds", what);
    if (seeds->n > 0 && (!seed_event || !seed_hits || !out_hits))
        return fail(ctx, KF_EINVAL, "%s: null seed_event, seed_hits or out_hits", what);
    const int W = ctx->find_width;
    const int MC = ctx->params.max_cands;
    const int S = kfmi::seeds_per_wg(W, MC);
    const int nl = ctx->n_layers;
    kfmi::FindPlan& pl = L->pl;
    int64_t per_event = 0;
    for (int l = 0; l < nl; ++l) {
        pl.bl.base[l] = (int32_t)per_event;
        per_event += (int64_t)ctx->layers[l].nbin_phi * ctx->layers[l].nbin_2;
    }
    if ((int64_t)n_events * per_event >= 0x7fffffffLL ||
        (int64_t)n_events * 4096 >= 0x7fffffffLL)
        return fail(ctx, KF_EINVAL, "%s: n_events x bins per event exceeds 2^31", what);
    pl.bl.per_event = (int32_t)per_event;
    const size_t lds = kfmi::find_shared_size(W, S, nl, prec);
    if (ctx->max_lds > 0 && lds > (size_t)ctx->max_lds)
        return fail(ctx, KF_EUNSUPPORTED, "%s: width %d needs %zu bytes of LDS, device allows %d",
                    what, W, lds, ctx->max_lds);
    int lw = 0;
    while ((1 << lw) < W) ++lw;
    const int pi = prec == KF_PREC_FP32 ? 1 : 0;
    const bool mat = ctx->mat.x0 != nullptr;
    const bool steer = ctx->d_steer != nullptr;
    int& occ = ctx->occ_cache[field ? 1 : 0][steer ? 1 : 0][mat ? 1 : 0][learn ? 1 : 0][pi][lw];
    if (occ == 0) {
        hipError_t e = kfmi::find_max_blocks_per_cu(W, S, nl, prec, learn, mat, steer, field, &occ);
        if (e != hipSuccess) return hip_fail(ctx, e, "find occupancy");
        if (occ < 1) occ = 1;
    }
    const int64_t n_tiles = (seeds->n + S - 1) / S;
    int64_t grid = (int64_t)occ * (ctx->n_cu > 0 ? ctx->n_cu : 1);
    if (grid > n_tiles) grid = n_tiles;
    if (grid < 1) grid = 1;
    const size_t bytes = kfmi::plan_find(&pl, nullptr, hits->n, n_events, seeds->n, nl, (int)grid, S);
    void* base = nullptr;
    if (fixed_ws) {
        if (bytes > fixed_bytes)
            return fail(ctx, KF_EINVAL, "%s: the call needs %zu bytes of scratch, the static scratch "
                        "holds %zu", what, bytes, fixed_bytes);
        base = fixed_ws;
    } else {
        base = ctx->ws.get(bytes);
        if (!base) return fail(ctx, KF_ENOMEM, "%s: workspace of %zu bytes", what, bytes);
    }
    kfmi::plan_find(&pl, base, hits->n, n_events, seeds->n, nl, (int)grid, S);
    kfmi::FindArgs& a = L->a;
    a.bh = (const kfmi::BinnedHit*)pl.binned;
    a.bin_off = pl.off;
    a.bl = pl.bl;
    a.n_hits = hits->n;
    a.hit_layer = hits->layer;
    a.n_seeds = seeds->n;
    a.sld = seeds->ld;
    a.spar = (const float*)seeds->par;
    a.scov = (const float*)seeds->cov;
    a.schi2 = (const float*)seeds->chi2;
    a.sndf = seeds->ndf;
    a.sstatus = seeds->status;
    a.seed_event = seed_event;
    a.n_events = n_events;
    a.seed_hits = seed_hits;
    a.order = pl.tile_order;
    a.out_hits = out_hits;
    a.old = out->ld;
    a.opar = (float*)out->par;
    a.ocov = (float*)out->cov;
    a.ochi2 = (float*)out->chi2;
    a.ondf = out->ndf;
    a.ostatus = out->status;
    a.bp = pl.bp;
    a.tile_counter = pl.tile_counter;
    a.queue_loopers = pl.queue_loopers;
    a.counters = (unsigned long long*)counters;
    a.layers = ctx->d_layers;
    a.n_layers = nl;
    a.prm = ctx->params;
    a.material = (flags & KF_NO_MATERIAL) ? 0 : 1;
    a.mat = ctx->mat;
    a.steer = ctx->d_steer;
    a.n_tiles = (int)n_tiles;
    a.seeds_per_tile = S;
    a.mlp = ctx->mlp.dev();
    L->learn = learn;
    L->clean = (flags & KF_CLEAN_SEEDS) != 0;
    L->dedup = (flags & KF_REMOVE_DUPLICATES) != 0;
    L->out_hits = out_hits;
    L->out = out;
    L->seed_hits = seed_hits;
    L->W = W;
    L->grid = (int)grid;
    L->prec = prec;
    L->largest_first = ctx->find_largest_first;
    L->n_events = n_events;
    L->event_off = event_off;
    L->seed_event = seed_event;
    L->hits = hits;
    L->seeds = seeds;
    return KF_OK;
}

hipError_t phase_bin(const kf_ctx* ctx, const kfmi::FindLaunch& L, hipStream_t s)
{
    return kfmi::launch_bin(L.pl, L.hits, L.event_off, (int)L.n_events, ctx->d_layers,
                            ctx->n_layers, s);
}

hipError_t phase_order(const kf_ctx* ctx, const kfmi::FindLaunch& L, hipStream_t s)
{
    hipError_t e = kfmi::launch_seed_order(L.pl, L.seeds, L.seed_event, L.event_off,
                                           (int)L.n_events, L.largest_first, s);
    if (e == hipSuccess && L.clean)
        e = kfmi::launch_clean(L.pl, L.seeds, L.seed_event, (int)L.n_events, L.seed_hits,
                               L.hits->n, ctx->params, s);
    if (e == hipSuccess) e = kfmi::launch_cost_order(L.pl, L.seeds, L.a.n_tiles, L.a.seeds_per_tile, s);
    if (e == hipSuccess) e = kfmi::launch_fill(L.pl.tile_counter, 64, 0, s);
    return e;
}

hipError_t phase_find(const kf_ctx* ctx, const kfmi::FindLaunch& L, hipStream_t s)
{
    hipError_t e = kfmi::launch_find_kernel(L.a, L.W, L.grid, L.prec, L.learn, s);
    if (e == hipSuccess && L.dedup)
        e = kfmi::launch_dedup(L.pl, L.out->n, ctx->n_layers, L.out_hits, (const float*)L.out->chi2,
                               L.out->status, L.seed_event, L.hits->n, ctx->params.dup_frac, s);
    return e;
}

// Event set of the next timed call, or nullptr when timing is off.
hipEvent_t* timing_set(kf_ctx* ctx)
{
    if (ctx->timing_used >= ctx->timing_n) return nullptr;
    return ctx->ev + kfmi::kPhaseEvents * ctx->timing_used;
}

void release_graph(kf_ctx* ctx)
{
    kfmi::FindGraph& g = ctx->fg;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = kfmi::FindGraph();
}

// Captures what `f` enqueues on the context's capture stream into a new graph.
template <typename F>
hipError_t capture(kf_ctx* ctx, hipGraph_t* out, F f)
{
    *out = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = f(ctx->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    *out = g;
    return hipSuccess;
}

// Static scratch of kf_find_noalloc: one copy per device, alive until the
// process ends.  In host code `scratch` names a host-side stand-in; the
// device address comes from hipGetSymbolAddress, once per device, at
// kf_create.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kfmi::kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up on the
// first call for that device.
hipError_t scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kfmi::kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char* kf_last_error(const kf_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

const char* kf_last_error_global(void) { return g_err.c_str(); }

int kf_create(kf_ctx** out, const kf_layer* layers, int32_t n_layers, const kf_params* params)
{
    if (!out) return fail(nullptr, KF_EINVAL, "kf_create: null output pointer");
    *out = nullptr;
    if (!layers || n_layers <= 0 || n_layers > kfmi::kMaxLayers)
        return fail(nullptr, KF_EINVAL, "kf_create: need 1..%d layers (got %d)", kfmi::kMaxLayers,
                    n_layers);
    for (int i = 0; i < n_layers; ++i) {
        const kf_layer& L = layers[i];
        if ((L.kind != 0 && L.kind != 1) || !(L.hi > L.lo) || L.nbin_phi <= 0 || L.nbin_2 <= 0 ||
            L.nbin_phi * L.nbin_2 > kfmi::kMaxLayerBins || !(L.x0 >= 0.0) ||
            (L.kind == 0 && !(L.r_or_z > 0.0)) || !(L.win_su >= 0.0) || !(L.win_sv >= 0.0))
            return fail(nullptr, KF_EINVAL, "kf_create: invalid layer %d", i);
    }
    kf_params p;
    if (params) {
        p = *params;
    } else {
        p.bz = 3.8;
        p.chi2_cut = 30.0;
        p.max_cands = 6;
        p.max_newton = 10;
        p.newton_tol = 1e-4;
        p.mass = 0.13957;
        p.max_miss = 2;
        p.mlp_max_iter = 3;
        p.field_z0 = 0.0;
        p.field_step = 2.0;
        p.clean_deta = 0.01;
        p.clean_dphi = 0.01;
        p.clean_dc = 0.05;
        p.dup_frac = 0.5;
    }
    if (!(p.bz != 0.0) || !(p.chi2_cut > 0.0) || p.max_cands < 1 || p.max_cands > 8 ||
        p.max_newton < 1 || p.max_newton > 64 || !(p.newton_tol > 0.0) || !(p.mass >= 0.0) ||
        p.max_miss < 0 || p.mlp_max_iter < 1 || p.mlp_max_iter > 64 || !(p.field_z0 >= 0.0) ||
        (p.field_z0 > 0.0 && !(p.field_step > 0.0 && p.field_step <= 1000.0)) ||
        !(p.clean_deta >= 0.0 && p.clean_deta <= 6.0 / 64.0) ||
        !(p.clean_dphi >= 0.0 && p.clean_dphi <= 2.0 * kfmi::kPi / 64.0) ||
        !(p.clean_dc >= 0.0 && p.clean_dc < 1e30) || !(p.dup_frac > 0.0 && p.dup_frac <= 1.0))
        return fail(nullptr, KF_EINVAL, "kf_create: invalid parameters");
    kf_ctx* ctx = new kf_ctx();
    ctx->n_layers = n_layers;
    memcpy(ctx->layers, layers, sizeof(kf_layer) * n_layers);
    ctx->params = p;
    hipError_t e = hipGetDevice(&ctx->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&ctx->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                  ctx->device);
    if (e == hipSuccess) e = scratch_address(ctx->device, &ctx->noalloc_scratch);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_layers, sizeof(kf_layer) * kfmi::kMaxLayers);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_layers, ctx->layers, sizeof(kf_layer) * n_layers, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        int r = hip_fail(nullptr, e, "kf_create");
        if (ctx->d_layers) (void)hipFree(ctx->d_layers);
        delete ctx;
        return r;
    }
    *out = ctx;
    return KF_OK;
}

void kf_destroy(kf_ctx* ctx)
{
    if (!ctx) return;
    release_graph(ctx);
    for (int k = 0; k < kfmi::kPhaseEvents * ctx->timing_cap; ++k) (void)hipEventDestroy(ctx->ev[k]);
    delete[] ctx->ev;
    for (int k = 0; k < kfmi::kPhaseEvents; ++k)
        if (ctx->idle_ev[k]) (void)hipEventDestroy(ctx->idle_ev[k]);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    ctx->mlp_ws.release();
    if (ctx->mlp_mem) (void)hipFree(ctx->mlp_mem);
    ctx->ws.release();
    if (ctx->d_layers) (void)hipFree(ctx->d_layers);
    if (ctx->d_mat) (void)hipFree(ctx->d_mat);
    if (ctx->d_steer) (void)hipFree(ctx->d_steer);
    delete ctx;
}

int kf_seed(kf_ctx* ctx, const kf_hits* hits, const int32_t* seed_hits, kf_tracks* out, int flags,
            void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_seed: null context");
    int r = check_tracks(ctx, out, "kf_seed");
    if (r) return r;
    r = check_hits(ctx, hits, "kf_seed");
    if (r) return r;
    if (out->n > 0 && !seed_hits) return fail(ctx, KF_EINVAL, "kf_seed: null seed_hits");
    hipError_t e = kfmi::launch_seed(ctx, hits, seed_hits, out, flags, (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_seed");
}

int kf_propagate(kf_ctx* ctx, kf_tracks* t, const int32_t* target_layer, float* path_len,
                 int32_t* iters, int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_propagate: null context");
    int r = check_tracks(ctx, t, "kf_propagate");
    if (r) return r;
    if (t->n > 0 && !target_layer) return fail(ctx, KF_EINVAL, "kf_propagate: null target_layer");
    if ((flags & KF_INIT_MLP) && !ctx->mlp_loaded)
        return fail(ctx, KF_EUNSUPPORTED, "kf_propagate: no learned model loaded");
    hipError_t e = kfmi::launch_propagate(ctx, t, target_layer, path_len, iters, flags,
                                          (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_propagate");
}

int kf_fit(kf_ctx* ctx, kf_tracks* t, const kf_hits* hits, const int32_t* layer_seq,
           const int32_t* hit_idx, int32_t max_steps, int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_fit: null context");
    int r = check_tracks(ctx, t, "kf_fit");
    if (r) return r;
    r = check_hits(ctx, hits, "kf_fit");
    if (r) return r;
    if (max_steps < 0 || max_steps > 4096) return fail(ctx, KF_EINVAL, "kf_fit: bad max_steps");
    if (!layer_seq && max_steps > ctx->n_layers)
        return fail(ctx, KF_EINVAL, "kf_fit: max_steps exceeds the layer count with implicit layers");
    if (t->n > 0 && max_steps > 0 && !hit_idx) return fail(ctx, KF_EINVAL, "kf_fit: null hit_idx");
    if ((flags & KF_INIT_MLP) && !ctx->mlp_loaded)
        return fail(ctx, KF_EUNSUPPORTED, "kf_fit: no learned model loaded");
    hipError_t e = kfmi::launch_fit(ctx, t, hits, layer_seq, hit_idx, max_steps, flags,
                                    (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_fit");
}

int kf_set_find_config(kf_ctx* ctx, int32_t width, int32_t largest_first)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_set_find_config: null context");
    if (width != 32 && width != 64 && width != 128 && width != 256)
        return fail(ctx, KF_EINVAL, "kf_set_find_config: width must be 32, 64, 128 or 256");
    if (kfmi::seeds_per_wg(width, ctx->params.max_cands) < 1)
        return fail(ctx, KF_EINVAL, "kf_set_find_config: width below max_cands");
    ctx->find_width = width;
    ctx->find_largest_first = largest_first ? 1 : 0;
    return KF_OK;
}

int kf_get_find_config(kf_ctx* ctx, int32_t* width, int32_t* largest_first)
{
    if (!ctx || !width || !largest_first)
        return fail(ctx, KF_EINVAL, "kf_get_find_config: null argument");
    *width = ctx->find_width;
    *largest_first = ctx->find_largest_first;
    return KF_OK;
}

int kf_set_steering(kf_ctx* ctx, const kf_region* regions, int32_t n_regions)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_set_steering: null context");
    const bool set = regions && n_regions > 0;
    kfmi::SteerDev h{};
    if (set) {
        if (n_regions > kfmi::kMaxRegions)
            return fail(ctx, KF_EINVAL, "kf_set_steering: at most %d regions", kfmi::kMaxRegions);
        h.n = n_regions;
        for (int g = 0; g < n_regions; ++g) {
            const kf_region& R = regions[g];
            if (!(R.eta_lo < R.eta_hi) || R.n_layers < 1 || R.n_layers > kfmi::kMaxPlan)
                return fail(ctx, KF_EINVAL, "kf_set_steering: region %d has a bad eta range or length", g);
            bool seen[kfmi::kMaxLayers] = {};
            for (int q = 0; q < R.n_layers; ++q) {
                const int l = R.layers[q];
                if (l < 0 || l >= ctx->n_layers || seen[l])
                    return fail(ctx, KF_EINVAL, "kf_set_steering: region %d entry %d: bad or repeated layer",
                                g, q);
                seen[l] = true;
                h.layers[g][q] = (uint8_t)l;
            }
            h.len[g] = R.n_layers;
            h.eta_lo[g] = R.eta_lo;
            h.eta_hi[g] = R.eta_hi;
        }
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_set_steering");
    // a captured pass holds the old steering pointer: capture again next time
    release_graph(ctx);
    ctx->setup_gen++;
    if (ctx->d_steer) {
        e = hipFree(ctx->d_steer);
        ctx->d_steer = nullptr;
        if (e != hipSuccess) return hip_fail(ctx, e, "kf_set_steering free");
    }
    if (!set) return KF_OK;
    kfmi::SteerDev* d = nullptr;
    e = hipMalloc(&d, sizeof(kfmi::SteerDev));
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_set_steering alloc");
    e = hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(ctx, e, "kf_set_steering copy");
    }
    ctx->d_steer = d;
    return KF_OK;
}

int kf_set_material(kf_ctx* ctx, const kf_material* m)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_set_material: null context");
    if (m) {
        if (m->nr < 1 || m->nz < 1 || (int64_t)m->nr * m->nz > (1LL << 22) || !(m->r_max > 0.0) ||
            !(m->z_max > m->z_min) || !std::isfinite(m->r_max) || !std::isfinite(m->z_min) ||
            !std::isfinite(m->z_max) || !m->x0 || !m->xi)
            return fail(ctx, KF_EINVAL, "kf_set_material: bad map dimensions or null arrays");
        const int64_t nc = (int64_t)m->nr * m->nz;
        for (int64_t i = 0; i < nc; ++i)
            if (!(m->x0[i] >= 0.0f) || !(m->xi[i] >= 0.0f) || !std::isfinite(m->x0[i]) ||
                !std::isfinite(m->xi[i]))
                return fail(ctx, KF_EINVAL, "kf_set_material: cell %lld is negative or not finite",
                            (long long)i);
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_set_material");
    // a captured pass holds the old map's pointers and sizes by value: capture
    // again next time
    release_graph(ctx);
    ctx->setup_gen++;
    if (ctx->d_mat) {
        e = hipFree(ctx->d_mat);
        ctx->d_mat = nullptr;
        ctx->mat = kfmi::MatMap{};
        if (e != hipSuccess) return hip_fail(ctx, e, "kf_set_material free");
    }
    if (!m) return KF_OK;
    const size_t nc = (size_t)m->nr * m->nz;
    float* d = nullptr;
    e = hipMalloc(&d, 2 * nc * sizeof(float));
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_set_material alloc");
    e = hipMemcpy(d, m->x0, nc * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + nc, m->xi, nc * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(ctx, e, "kf_set_material copy");
    }
    ctx->d_mat = d;
    ctx->mat.x0 = d;
    ctx->mat.xi = d + nc;
    ctx->mat.nr = m->nr;
    ctx->mat.nz = m->nz;
    ctx->mat.r_max = m->r_max;
    ctx->mat.z_min = m->z_min;
    ctx->mat.z_max = m->z_max;
    return KF_OK;
}

int kf_remove_duplicates(kf_ctx* ctx, const kf_hits* hits, kf_tracks* tracks,
                         const int32_t* track_hits, const int32_t* track_event, int flags,
                         void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_remove_duplicates: null context");
    int r = check_tracks(ctx, tracks, "kf_remove_duplicates");
    if (r) return r;
    if (!hits || hits->n < 0) return fail(ctx, KF_EINVAL, "kf_remove_duplicates: bad hits");
    const int prec = flags & KF_PREC_MASK;
    if (prec != KF_PREC_MIXED && prec != KF_PREC_FP32)
        return fail(ctx, KF_EUNSUPPORTED, "kf_remove_duplicates: float storage only (MIXED or FP32)");
    if (hits->n > 0x7ffffffeLL) return fail(ctx, KF_EINVAL, "kf_remove_duplicates: at most 2^31-2 hits");
    if (tracks->n * (int64_t)ctx->n_layers > 0x7fffffffLL)
        return fail(ctx, KF_EINVAL, "kf_remove_duplicates: too many tracks");
    if (tracks->n == 0) return KF_OK;
    if (!track_hits || !track_event)
        return fail(ctx, KF_EINVAL, "kf_remove_duplicates: null track_hits or track_event");
    kfmi::FindPlan pl{};
    pl.bl.per_event = 0;
    const size_t bytes = kfmi::plan_find(&pl, nullptr, hits->n, 1, tracks->n, ctx->n_layers, 1, 1);
    void* base = ctx->ws.get(bytes);
    if (!base) return fail(ctx, KF_ENOMEM, "kf_remove_duplicates: workspace of %zu bytes", bytes);
    kfmi::plan_find(&pl, base, hits->n, 1, tracks->n, ctx->n_layers, 1, 1);
    hipError_t e = kfmi::launch_dedup(pl, tracks->n, ctx->n_layers, track_hits,
                                      (const float*)tracks->chi2, tracks->status, track_event,
                                      hits->n, ctx->params.dup_frac, (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_remove_duplicates");
}

int kf_clean_seeds(kf_ctx* ctx, const kf_hits* hits, int32_t n_events, kf_tracks* seeds,
                   const int32_t* seed_event, const int32_t* seed_hits, int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_clean_seeds: null context");
    int r = check_tracks(ctx, seeds, "kf_clean_seeds");
    if (r) return r;
    if (!hits || hits->n < 0) return fail(ctx, KF_EINVAL, "kf_clean_seeds: bad hits");
    const int prec = flags & KF_PREC_MASK;
    if (prec != KF_PREC_MIXED && prec != KF_PREC_FP32)
        return fail(ctx, KF_EUNSUPPORTED, "kf_clean_seeds: float storage only (MIXED or FP32)");
    if (n_events < 1) return fail(ctx, KF_EINVAL, "kf_clean_seeds: need n_events >= 1");
    if ((int64_t)n_events * 4096 >= 0x7fffffffLL)
        return fail(ctx, KF_EINVAL, "kf_clean_seeds: too many events");
    if (seeds->n > 0x7fffffffLL) return fail(ctx, KF_EINVAL, "kf_clean_seeds: at most 2^31-1 seeds");
    if (seeds->n == 0) return KF_OK;
    if (!seed_event || !seed_hits) return fail(ctx, KF_EINVAL, "kf_clean_seeds: null seed_event or seed_hits");
    kfmi::FindPlan pl{};
    pl.bl.per_event = 0;
    const size_t bytes = kfmi::plan_find(&pl, nullptr, hits->n, n_events, seeds->n, 0, 1, 1);
    void* base = ctx->ws.get(bytes);
    if (!base) return fail(ctx, KF_ENOMEM, "kf_clean_seeds: workspace of %zu bytes", bytes);
    kfmi::plan_find(&pl, base, hits->n, n_events, seeds->n, 0, 1, 1);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = kfmi::launch_seed_order(pl, seeds, seed_event, nullptr, n_events, 0, s);
    if (e == hipSuccess) e = kfmi::launch_clean(pl, seeds, seed_event, n_events, seed_hits, hits->n,
                                                ctx->params, s);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_clean_seeds");
}

int kf_find(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
            const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
            int32_t* out_hits, kf_tracks* out, uint64_t* counters, int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_find: null context");
    kfmi::FindLaunch L;
    int r = prepare_find(ctx, hits, event_off, n_events, seeds, seed_event, seed_hits, out_hits,
                         out, counters, flags, "kf_find", &L);
    if (r) return r;
    if (seeds->n == 0) return KF_OK;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t* ev = timing_set(ctx);
    hipError_t e = hipSuccess;
    // no seeding phase here: its two events coincide
    if (ev) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = phase_bin(ctx, L, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
    if (e == hipSuccess) e = phase_order(ctx, L, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) e = phase_find(ctx, L, s);
    if (e == hipSuccess && ev) {
        e = hipEventRecord(ev[4], s);
        if (e == hipSuccess) ctx->timing_used++;
    }
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_find");
}

int kf_find_noalloc(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                    const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
                    int32_t* out_hits, kf_tracks* out, uint64_t* counters, int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_find_noalloc: null context");
    if (!ctx->noalloc_scratch) return fail(ctx, KF_EHIP, "kf_find_noalloc: no static scratch");
    kfmi::FindLaunch L;
    int r = prepare_find(ctx, hits, event_off, n_events, seeds, seed_event, seed_hits, out_hits,
                         out, counters, flags, "kf_find_noalloc", &L, ctx->noalloc_scratch,
                         kNoAllocScratchBytes);
    if (r) return r;
    if (seeds->n == 0) return KF_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = phase_bin(ctx, L, s);
    if (e == hipSuccess) e = phase_order(ctx, L, s);
    if (e == hipSuccess) e = phase_find(ctx, L, s);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_find_noalloc");
}

int kf_find_batched(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                    const int32_t* seed_hits, const int32_t* seed_layers, const int32_t* seed_event,
                    kf_tracks* seeds, int32_t* out_hits, kf_tracks* out, uint64_t* counters,
                    int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_find_batched: null context");
    if (flags & KF_PER_LAYER) return fail(ctx, KF_EINVAL, "kf_find_batched: KF_PER_LAYER is a fit option");
    kfmi::FindLaunch L;
    int r = prepare_find(ctx, hits, event_off, n_events, seeds, seed_event, seed_hits, out_hits,
                         out, counters, flags, "kf_find_batched", &L);
    if (r) return r;
    if (seeds->n > 0 && !seed_layers) return fail(ctx, KF_EINVAL, "kf_find_batched: null seed_layers");
    if (seeds->n == 0) return KF_OK;
    hipError_t e = hipSuccess;
    if (!ctx->cap_stream) {
        // created together: kept only if all succeed
        hipStream_t cs = nullptr;
        hipEvent_t ie[kfmi::kPhaseEvents] = {};
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        for (int k = 0; k < kfmi::kPhaseEvents && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&ie[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (int k = 0; k < kfmi::kPhaseEvents; ++k)
                if (ie[k]) (void)hipEventDestroy(ie[k]);
            if (cs) (void)hipStreamDestroy(cs);
            return hip_fail(ctx, e, "kf_find_batched setup");
        }
        ctx->cap_stream = cs;
        for (int k = 0; k < kfmi::kPhaseEvents; ++k) ctx->idle_ev[k] = ie[k];
    }
    // everything the captured launches depend on: pointers, sizes, options
    // and the workspace (a grown workspace moves every scratch array)
    uint64_t key[40];
    int nk = 0;
    auto put = [&](uint64_t v) { key[nk++] = v; };
    put((uint64_t)(uintptr_t)hits->x); put((uint64_t)(uintptr_t)hits->y);
    put((uint64_t)(uintptr_t)hits->z); put((uint64_t)(uintptr_t)hits->su);
    put((uint64_t)(uintptr_t)hits->sv); put((uint64_t)(uintptr_t)hits->layer);
    put((uint64_t)hits->n); put((uint64_t)(uintptr_t)event_off); put((uint64_t)n_events);
    put((uint64_t)(uintptr_t)seed_hits); put((uint64_t)(uintptr_t)seed_layers);
    put((uint64_t)(uintptr_t)seed_event);
    put((uint64_t)seeds->n); put((uint64_t)seeds->ld); put((uint64_t)(uintptr_t)seeds->par);
    put((uint64_t)(uintptr_t)seeds->cov); put((uint64_t)(uintptr_t)seeds->chi2);
    put((uint64_t)(uintptr_t)seeds->ndf); put((uint64_t)(uintptr_t)seeds->status);
    put((uint64_t)out->ld); put((uint64_t)(uintptr_t)out->par); put((uint64_t)(uintptr_t)out->cov);
    put((uint64_t)(uintptr_t)out->chi2); put((uint64_t)(uintptr_t)out->ndf);
    put((uint64_t)(uintptr_t)out->status); put((uint64_t)(uintptr_t)out_hits);
    put((uint64_t)(uintptr_t)counters); put((uint64_t)flags); put((uint64_t)L.W);
    put((uint64_t)L.largest_first); put((uint64_t)L.grid);
    put((uint64_t)(uintptr_t)ctx->ws.ptr); put((uint64_t)ctx->ws.bytes);
    put((uint64_t)(uintptr_t)ctx->mat.x0);
    put((uint64_t)(uintptr_t)ctx->d_steer);
    put(ctx->setup_gen);
    kfmi::FindGraph& g = ctx->fg;
    const bool same = g.exec && g.nkey == nk && memcmp(g.key, key, sizeof(uint64_t) * nk) == 0;
    if (!same) {
        release_graph(ctx);
        hipGraph_t sub[4] = {nullptr, nullptr, nullptr, nullptr};
        kf_tracks* st = seeds;
        const int fit_flags = flags & (KF_PREC_MASK | KF_NO_MATERIAL | KF_INIT_MLP);
        e = capture(ctx, &sub[0], [&](hipStream_t cs) {
            hipError_t x = kfmi::launch_seed(ctx, hits, seed_hits, st, fit_flags, cs);
            if (x == hipSuccess) x = kfmi::launch_fit(ctx, st, hits, seed_layers, seed_hits, 3, fit_flags, cs);
            return x;
        });
        if (e == hipSuccess) e = capture(ctx, &sub[1], [&](hipStream_t cs) { return phase_bin(ctx, L, cs); });
        if (e == hipSuccess) e = capture(ctx, &sub[2], [&](hipStream_t cs) { return phase_order(ctx, L, cs); });
        if (e == hipSuccess) e = capture(ctx, &sub[3], [&](hipStream_t cs) { return phase_find(ctx, L, cs); });
        if (e == hipSuccess) e = hipGraphCreate(&g.graph, 0);
        // event 0 -> seed+fit -> event 1 -> binning -> event 2 -> order -> event 3 -> find -> event 4
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < kfmi::kPhaseEvents && e == hipSuccess; ++k) {
            e = hipGraphAddEventRecordNode(&g.ev_node[k], g.graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                           ctx->idle_ev[k]);
            prev = g.ev_node[k];
            if (e == hipSuccess && k < 4) {
                hipGraphNode_t child;
                e = hipGraphAddChildGraphNode(&child, g.graph, &prev, 1, sub[k]);
                prev = child;
            }
        }
        for (int k = 0; k < 4; ++k)
            if (sub[k]) (void)hipGraphDestroy(sub[k]);   // the child nodes hold copies
        if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            release_graph(ctx);
            return hip_fail(ctx, e, "kf_find_batched capture");
        }
        memcpy(g.key, key, sizeof(uint64_t) * nk);
        g.nkey = nk;
        g.timed = false;
    }
    hipEvent_t* ev = timing_set(ctx);
    if (ev || g.timed) {
        for (int k = 0; k < kfmi::kPhaseEvents && e == hipSuccess; ++k)
            e = hipGraphExecEventRecordNodeSetEvent(g.exec, g.ev_node[k], ev ? ev[k] : ctx->idle_ev[k]);
        if (e != hipSuccess) return hip_fail(ctx, e, "kf_find_batched timing");
        g.timed = ev != nullptr;
    }
    e = hipGraphLaunch(g.exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_find_batched launch");
    if (ev) ctx->timing_used++;
    return KF_OK;
}

int kf_set_timing(kf_ctx* ctx, int32_t n)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_set_timing: null context");
    if (n < 0 || n > 256) return fail(ctx, KF_EINVAL, "kf_set_timing: n must be in 0..256");
    constexpr int E = kfmi::kPhaseEvents;
    if (n > ctx->timing_cap) {
        hipEvent_t* ev = new hipEvent_t[E * n];
        int k = 0;
        for (; k < E * ctx->timing_cap; ++k) ev[k] = ctx->ev[k];
        for (; k < E * n; ++k) {
            hipError_t r = hipEventCreate(&ev[k]);
            if (r != hipSuccess) {
                for (int j = E * ctx->timing_cap; j < k; ++j) (void)hipEventDestroy(ev[j]);
                delete[] ev;
                return hip_fail(ctx, r, "kf_set_timing");
            }
        }
        // a captured pass may still point at the old sets: point it back at
        // the idle events before they go
        if (ctx->fg.exec && ctx->fg.timed) {
            for (int j = 0; j < E; ++j)
                (void)hipGraphExecEventRecordNodeSetEvent(ctx->fg.exec, ctx->fg.ev_node[j],
                                                          ctx->idle_ev[j]);
            ctx->fg.timed = false;
        }
        delete[] ctx->ev;
        ctx->ev = ev;
        ctx->timing_cap = n;
    }
    // the next n calls record into sets 0..n-1; later calls are not recorded
    ctx->timing_used = 0;
    ctx->timing_n = n;
    return KF_OK;
}

int kf_timings(kf_ctx* ctx, float ms[5])
{
    if (!ctx || !ms) return fail(ctx, KF_EINVAL, "kf_timings: null argument");
    constexpr int E = kfmi::kPhaseEvents;
    const int last = ctx->timing_used;
    if (ctx->timing_n == 0 || last <= 0) return fail(ctx, KF_EINVAL, "kf_timings: nothing recorded");
    hipError_t e = hipEventSynchronize(ctx->ev[E * (last - 1) + E - 1]);
    double acc[E - 1] = {};
    for (int c = 0; c < last && e == hipSuccess; ++c)
        for (int k = 0; k < E - 1 && e == hipSuccess; ++k) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ctx->ev[E * c + k], ctx->ev[E * c + k + 1]);
            acc[k] += t;
        }
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_timings");
    for (int k = 0; k < E - 1; ++k) ms[k] = float(acc[k] / last);
    ms[E - 1] = float(last);
    return KF_OK;
}

int kf_autotune(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
                int32_t* out_hits, kf_tracks* out, int flags, int32_t reps, float* table,
                void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_autotune: null context");
    if (reps < 1 || reps > 100) return fail(ctx, KF_EINVAL, "kf_autotune: reps must be in 1..100");
    hipStream_t s = (hipStream_t)stream;
    constexpr int NW = 4, NC = 2 * NW;
    static const int widths[NW] = {32, 64, 128, 256};
    const int w0 = ctx->find_width, lf0 = ctx->find_largest_first;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return hip_fail(ctx, e, "kf_autotune");
    }
    const int saved_n = ctx->timing_n, saved_used = ctx->timing_used;
    ctx->timing_n = ctx->timing_used = 0;       // tuning calls are not recorded
    float best_ms[NC];
    bool fits[NC];
    for (int c = 0; c < NC; ++c) {
        best_ms[c] = -1.0f;
        const int w = widths[c / 2];
        fits[c] = kfmi::seeds_per_wg(w, ctx->params.max_cands) >= 1 &&
                  !((flags & KF_INIT_MLP) && w < 64) &&
                  kfmi::find_shared_size(w, kfmi::seeds_per_wg(w, ctx->params.max_cands), ctx->n_layers,
                                         flags & KF_PREC_MASK) <= (size_t)ctx->max_lds;
    }
    // configurations are visited round-robin, reps rounds, each call timed
    // on its own after one untimed call per configuration, and the fastest
    // call counts: clock ramps and other drifts hit every configuration
    int r = KF_OK;
    for (int round = -1; round < reps && r == KF_OK; ++round)
        for (int c = 0; c < NC && r == KF_OK; ++c) {
            if (!fits[c]) continue;
            ctx->find_width = widths[c / 2];
            ctx->find_largest_first = c & 1;
            if (round >= 0 && (e = hipEventRecord(ev[0], s)) != hipSuccess) r = hip_fail(ctx, e, "kf_autotune");
            if (r == KF_OK)
                r = kf_find(ctx, hits, event_off, n_events, seeds, seed_event, seed_hits, out_hits,
                            out, nullptr, flags, stream);
            if (r != KF_OK || round < 0) continue;
            float ms = 0.0f;
            if ((e = hipEventRecord(ev[1], s)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
                r = hip_fail(ctx, e, "kf_autotune");
                continue;
            }
            if (best_ms[c] < 0.0f || ms < best_ms[c]) best_ms[c] = ms;
        }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    ctx->timing_n = saved_n;
    ctx->timing_used = saved_used;
    if (r != KF_OK) {
        ctx->find_width = w0;
        ctx->find_largest_first = lf0;
        return r;
    }
    int best = -1;
    for (int c = 0; c < NC; ++c) {
        if (table) table[c] = best_ms[c];
        if (best_ms[c] >= 0.0f && (best < 0 || best_ms[c] < best_ms[best])) best = c;
    }
    if (best < 0) {
        ctx->find_width = w0;
        ctx->find_largest_first = lf0;
        return fail(ctx, KF_EUNSUPPORTED, "kf_autotune: no configuration fits the device");
    }
    ctx->find_width = widths[best / 2];
    ctx->find_largest_first = best & 1;
    return KF_OK;
}


// ------------------------------------------------------------------ learned guess

int kf_mlp_load(kf_ctx* ctx, const float* w)
{
    if (!ctx || !w) return fail(ctx, KF_EINVAL, "kf_mlp_load: null argument");
    for (int p = 0; p < kfmi::kMlpParams; ++p)
        if (!std::isfinite(w[p])) return fail(ctx, KF_EINVAL, "kf_mlp_load: parameter %d is not finite", p);
    hipError_t e = hipSuccess;
    constexpr size_t nf = 3 * kfmi::kMlpParams + 193;
    constexpr size_t fbytes = (nf * sizeof(float) + 255) & ~size_t(255);
    if (!ctx->mlp_mem) {
        e = hipMalloc(&ctx->mlp_mem, fbytes + sizeof(uint16_t) * (64 * 16 + 2 * 64 * 64));
        if (e != hipSuccess) {
            ctx->mlp_mem = nullptr;
            return hip_fail(ctx, e, "kf_mlp_load");
        }
        float* f = (float*)ctx->mlp_mem;
        uint16_t* b = (uint16_t*)((char*)ctx->mlp_mem + fbytes);
        ctx->mlp.master = f;
        ctx->mlp.m = f + kfmi::kMlpParams;
        ctx->mlp.v = f + 2 * kfmi::kMlpParams;
        ctx->mlp.bias = f + 3 * kfmi::kMlpParams;
        ctx->mlp.w1 = b;
        ctx->mlp.w2 = b + 64 * 16;
        ctx->mlp.w2t = b + 64 * 16 + 64 * 64;
    }
    e = hipMemcpy(ctx->mlp.master, w, sizeof(float) * kfmi::kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(ctx->mlp.m, 0, sizeof(float) * 2 * kfmi::kMlpParams);
    if (e == hipSuccess) e = kfmi::launch_mlp_publish(ctx->mlp, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_mlp_load");
    ctx->mlp_loaded = true;
    ctx->mlp_step = 0;
    return KF_OK;
}

int kf_mlp_get(kf_ctx* ctx, float* w)
{
    if (!ctx || !w) return fail(ctx, KF_EINVAL, "kf_mlp_get: null argument");
    if (!ctx->mlp_loaded) return fail(ctx, KF_EINVAL, "kf_mlp_get: no learned model loaded");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(w, ctx->mlp.master, sizeof(float) * kfmi::kMlpParams, hipMemcpyDeviceToHost);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_mlp_get");
}

int kf_mlp_features(kf_ctx* ctx, const kf_tracks* t, const int32_t* target_layer, float* feats,
                    int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_mlp_features: null context");
    int r = check_tracks(ctx, t, "kf_mlp_features");
    if (r) return r;
    if (t->n > 0 && (!target_layer || !feats)) return fail(ctx, KF_EINVAL, "kf_mlp_features: null array");
    hipError_t e = kfmi::launch_mlp_features(ctx, t, target_layer, feats, flags & KF_PREC_MASK,
                                             (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_mlp_features");
}

int kf_mlp_targets(kf_ctx* ctx, const float* feats, const float* path_len, int64_t n, int64_t ld,
                   float* target, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_mlp_targets: null context");
    if (n < 0 || ld < n) return fail(ctx, KF_EINVAL, "kf_mlp_targets: need 0 <= n <= ld");
    if (n > 0 && (!feats || !path_len || !target))
        return fail(ctx, KF_EINVAL, "kf_mlp_targets: null array");
    hipError_t e = kfmi::launch_mlp_targets(feats, path_len, n, ld, target, (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_mlp_targets");
}

int kf_mlp_forward(kf_ctx* ctx, const float* feats, int64_t n, int64_t ld, float* out, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_mlp_forward: null context");
    if (!ctx->mlp_loaded) return fail(ctx, KF_EINVAL, "kf_mlp_forward: no learned model loaded");
    if (n < 0 || ld < n) return fail(ctx, KF_EINVAL, "kf_mlp_forward: need 0 <= n <= ld");
    if (n > 0 && (!feats || !out)) return fail(ctx, KF_EINVAL, "kf_mlp_forward: null array");
    hipError_t e = kfmi::launch_mlp_forward(ctx->mlp.dev(), feats, n, ld, out, (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_mlp_forward");
}

namespace {
int mlp_step_args(kf_ctx* ctx, const float* feats, const float* target, int64_t n, int64_t ld,
                  const int32_t* rows, int32_t batch, const char* what)
{
    if (!ctx->mlp_loaded) return fail(ctx, KF_EINVAL, "%s: no learned model loaded", what);
    if (n < 1 || ld < n) return fail(ctx, KF_EINVAL, "%s: need 1 <= n <= ld", what);
    if (batch < 1 || batch > (1 << 20)) return fail(ctx, KF_EINVAL, "%s: batch must be in 1..2^20", what);
    if (!feats || !target || !rows) return fail(ctx, KF_EINVAL, "%s: null array", what);
    return KF_OK;
}
}  // namespace

int kf_mlp_grad(kf_ctx* ctx, const float* feats, const float* target, int64_t n, int64_t ld,
                const int32_t* rows, int32_t batch, float* grad, float* loss, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_mlp_grad: null context");
    int r = mlp_step_args(ctx, feats, target, n, ld, rows, batch, "kf_mlp_grad");
    if (r) return r;
    if (!grad) return fail(ctx, KF_EINVAL, "kf_mlp_grad: null grad");
    void* scratch = ctx->mlp_ws.get(kfmi::mlp_partial_bytes(batch));
    if (!scratch) return fail(ctx, KF_ENOMEM, "kf_mlp_grad: scratch");
    kfmi::AdamStep ad{};
    hipError_t e = kfmi::launch_mlp_step(ctx->mlp, feats, target, n, ld, rows, batch, scratch, 0, ad,
                                         grad, loss, (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_mlp_grad");
}

int kf_mlp_train(kf_ctx* ctx, const float* feats, const float* target, int64_t n, int64_t ld,
                 const int32_t* rows, int32_t batch, int32_t n_steps, const kf_mlp_train_cfg* cfg,
                 float* loss, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_mlp_train: null context");
    int r = mlp_step_args(ctx, feats, target, n, ld, rows, batch, "kf_mlp_train");
    if (r) return r;
    if (n_steps < 0) return fail(ctx, KF_EINVAL, "kf_mlp_train: negative n_steps");
    kf_mlp_train_cfg c{1e-3, 0.9, 0.999, 1e-8};
    if (cfg) c = *cfg;
    if (!(c.lr > 0) || !(c.beta1 >= 0 && c.beta1 < 1) || !(c.beta2 >= 0 && c.beta2 < 1) || !(c.eps > 0))
        return fail(ctx, KF_EINVAL, "kf_mlp_train: bad optimiser settings");
    void* scratch = ctx->mlp_ws.get(kfmi::mlp_partial_bytes(batch));
    if (!scratch) return fail(ctx, KF_ENOMEM, "kf_mlp_train: scratch");
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < n_steps && e == hipSuccess; ++k) {
        const int64_t t = ++ctx->mlp_step;
        kfmi::AdamStep ad;
        ad.lr = float(c.lr);
        ad.beta1 = float(c.beta1);
        ad.beta2 = float(c.beta2);
        ad.eps = float(c.eps);
        ad.c1 = float(1.0 / (1.0 - std::pow(c.beta1, double(t))));
        ad.c2 = float(1.0 / (1.0 - std::pow(c.beta2, double(t))));
        e = kfmi::launch_mlp_step(ctx->mlp, feats, target, n, ld, rows + (int64_t)k * batch, batch,
                                  scratch, 1, ad, nullptr, loss ? loss + k : nullptr,
                                  (hipStream_t)stream);
    }
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_mlp_train");
}

}  // extern "C"
