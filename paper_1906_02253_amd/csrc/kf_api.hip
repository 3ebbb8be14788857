// C-ABI entry points of libkfmi.so: argument validation, context and
// workspace management, dispatch to the kernel launchers.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "kf_find.hpp"

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

}  // namespace kfmi

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
            L.nbin_phi > 4096 || L.nbin_2 > 4096 || !(L.x0 >= 0.0) ||
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
    }
    if (!(p.bz != 0.0) || !(p.chi2_cut > 0.0) || p.max_cands < 1 || p.max_cands > 8 ||
        p.max_newton < 1 || p.max_newton > 64 || !(p.newton_tol > 0.0) || !(p.mass >= 0.0) ||
        p.max_miss < 0 || p.mlp_max_iter < 1 || p.mlp_max_iter > 64)
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
    for (int k = 0; k < 4 * ctx->timing_cap; ++k) (void)hipEventDestroy(ctx->ev[k]);
    delete[] ctx->ev;
    ctx->ws.release();
    if (ctx->d_layers) (void)hipFree(ctx->d_layers);
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
    if (flags & KF_INIT_MLP) return fail(ctx, KF_EUNSUPPORTED, "kf_propagate: no learned model loaded");
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
    if (flags & KF_INIT_MLP) return fail(ctx, KF_EUNSUPPORTED, "kf_fit: no learned model loaded");
    hipError_t e = kfmi::launch_fit(ctx, t, hits, layer_seq, hit_idx, max_steps, flags,
                                    (hipStream_t)stream);
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_fit");
}

int kf_set_find_config(kf_ctx* ctx, int32_t width, int32_t largest_first)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_set_find_config: null context");
    if (width != 32 && width != 64 && width != 128 && width != 256)
        return fail(ctx, KF_EINVAL, "kf_set_find_config: width must be 32, 64, 128 or 256");
    if (width / ctx->params.max_cands < 1)
        return fail(ctx, KF_EINVAL, "kf_set_find_config: width below max_cands");
    ctx->find_width = width;
    ctx->find_largest_first = largest_first ? 1 : 0;
    return KF_OK;
}

int kf_find(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
            const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
            int32_t* out_hits, kf_tracks* out, uint64_t* counters, int flags, void* stream)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_find: null context");
    int r = check_tracks(ctx, seeds, "kf_find seeds");
    if (r) return r;
    r = check_tracks(ctx, out, "kf_find out");
    if (r) return r;
    r = check_hits(ctx, hits, "kf_find");
    if (r) return r;
    const int prec = flags & KF_PREC_MASK;
    if (prec == KF_PREC_FP64)
        return fail(ctx, KF_EUNSUPPORTED, "kf_find: float storage only (MIXED or FP32)");
    if (prec != KF_PREC_MIXED && prec != KF_PREC_FP32)
        return fail(ctx, KF_EINVAL, "kf_find: bad precision flag");
    if (flags & KF_INIT_MLP) return fail(ctx, KF_EUNSUPPORTED, "kf_find: no learned model loaded");
    if (out->n != seeds->n) return fail(ctx, KF_EINVAL, "kf_find: out->n must equal seeds->n");
    if (n_events < 1 || !event_off) return fail(ctx, KF_EINVAL, "kf_find: need n_events >= 1 and event_off");
    if (hits->n > 0x7fffffffLL) return fail(ctx, KF_EINVAL, "kf_find: at most 2^31-1 hits");
    if (seeds->n > 0x7fffffffLL) return fail(ctx, KF_EINVAL, "kf_find: at most 2^31-1 seeds");
    if (seeds->n > 0 && (!seed_event || !seed_hits || !out_hits))
        return fail(ctx, KF_EINVAL, "kf_find: null seed_event, seed_hits or out_hits");
    if (seeds->n == 0) return KF_OK;
    hipStream_t s = (hipStream_t)stream;
    const int W = ctx->find_width;
    const int MC = ctx->params.max_cands;
    const int S = W / MC;
    const int nl = ctx->n_layers;
    kfmi::FindPlan pl;
    int64_t per_event = 0;
    for (int l = 0; l < nl; ++l) {
        pl.bl.base[l] = (int32_t)per_event;
        per_event += (int64_t)ctx->layers[l].nbin_phi * ctx->layers[l].nbin_2;
    }
    if ((int64_t)n_events * per_event >= 0x7fffffffLL)
        return fail(ctx, KF_EINVAL, "kf_find: n_events x bins per event exceeds 2^31");
    pl.bl.per_event = (int32_t)per_event;
    const size_t lds = kfmi::find_shared_size(W, S, nl, prec);
    if (ctx->max_lds > 0 && lds > (size_t)ctx->max_lds)
        return fail(ctx, KF_EUNSUPPORTED, "kf_find: width %d needs %zu bytes of LDS, device allows %d",
                    W, lds, ctx->max_lds);
    int lw = 0;
    while ((1 << lw) < W) ++lw;
    const int pi = prec == KF_PREC_FP32 ? 1 : 0;
    int& occ = ctx->occ_cache[pi][lw];
    if (occ == 0) {
        hipError_t e = kfmi::find_max_blocks_per_cu(W, S, nl, prec, &occ);
        if (e != hipSuccess) return hip_fail(ctx, e, "kf_find occupancy");
        if (occ < 1) occ = 1;
    }
    const int64_t n_tiles = (seeds->n + S - 1) / S;
    int64_t grid = (int64_t)occ * (ctx->n_cu > 0 ? ctx->n_cu : 1);
    if (grid > n_tiles) grid = n_tiles;
    const size_t bytes = kfmi::plan_find(&pl, nullptr, hits->n, n_events, seeds->n, nl, (int)grid, S);
    void* base = ctx->ws.get(bytes);
    if (!base) return fail(ctx, KF_ENOMEM, "kf_find: workspace of %zu bytes", bytes);
    kfmi::plan_find(&pl, base, hits->n, n_events, seeds->n, nl, (int)grid, S);
    const bool tm = ctx->timing_used < ctx->timing_n;
    hipEvent_t* ev = tm ? ctx->ev + 4 * ctx->timing_used : nullptr;
    hipError_t e = hipSuccess;
    if (tm) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = kfmi::launch_bin(pl, hits, event_off, n_events, ctx->d_layers, nl, s);
    if (e == hipSuccess && tm) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess)
        e = kfmi::launch_seed_order(pl, seeds, seed_event, event_off, n_events,
                                    ctx->find_largest_first, s);
    if (e == hipSuccess) e = kfmi::launch_fill(pl.tile_counter, 64, 0, s);
    if (e == hipSuccess && tm) e = hipEventRecord(ev[2], s);
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_find setup");
    kfmi::FindArgs a;
    a.bh = (const kfmi::BinnedHit*)pl.binned;
    a.bin_off = pl.off;
    a.bl = pl.bl;
    a.n_hits = hits->n;
    a.hit_layer = hits->layer;
    a.n_seeds = seeds->n;
    a.sld = seeds->ld;
    a.spar = (const float*)seeds->par;
    a.scov = seeds->cov;
    a.schi2 = (const float*)seeds->chi2;
    a.sndf = seeds->ndf;
    a.sstatus = seeds->status;
    a.seed_event = seed_event;
    a.n_events = n_events;
    a.seed_hits = seed_hits;
    a.order = pl.order;
    a.out_hits = out_hits;
    a.old = out->ld;
    a.opar = (float*)out->par;
    a.ocov = out->cov;
    a.ochi2 = (float*)out->chi2;
    a.ondf = out->ndf;
    a.ostatus = out->status;
    a.bp = pl.bp;
    a.tile_counter = pl.tile_counter;
    a.counters = (unsigned long long*)counters;
    a.layers = ctx->d_layers;
    a.n_layers = nl;
    a.prm = ctx->params;
    a.material = (flags & KF_NO_MATERIAL) ? 0 : 1;
    a.n_tiles = (int)n_tiles;
    a.seeds_per_tile = S;
    e = kfmi::launch_find_kernel(a, W, (int)grid, prec, s);
    if (e == hipSuccess && tm) {
        e = hipEventRecord(ev[3], s);
        if (e == hipSuccess) ctx->timing_used++;
    }
    return e == hipSuccess ? KF_OK : hip_fail(ctx, e, "kf_find");
}

int kf_set_timing(kf_ctx* ctx, int32_t n)
{
    if (!ctx) return fail(nullptr, KF_EINVAL, "kf_set_timing: null context");
    if (n < 0 || n > 256) return fail(ctx, KF_EINVAL, "kf_set_timing: n must be in 0..256");
    if (n > ctx->timing_cap) {
        hipEvent_t* ev = new hipEvent_t[4 * n];
        int k = 0;
        for (; k < 4 * ctx->timing_cap; ++k) ev[k] = ctx->ev[k];
        for (; k < 4 * n; ++k) {
            hipError_t r = hipEventCreate(&ev[k]);
            if (r != hipSuccess) {
                for (int j = 4 * ctx->timing_cap; j < k; ++j) (void)hipEventDestroy(ev[j]);
                delete[] ev;
                return hip_fail(ctx, r, "kf_set_timing");
            }
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

int kf_timings(kf_ctx* ctx, float ms[4])
{
    if (!ctx || !ms) return fail(ctx, KF_EINVAL, "kf_timings: null argument");
    const int first = 0, last = ctx->timing_used;
    if (ctx->timing_n == 0 || last <= first) return fail(ctx, KF_EINVAL, "kf_timings: nothing recorded");
    hipError_t e = hipEventSynchronize(ctx->ev[4 * (last - 1) + 3]);
    double acc[3] = {0, 0, 0};
    for (int c = first; c < last && e == hipSuccess; ++c)
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ctx->ev[4 * c + k], ctx->ev[4 * c + k + 1]);
            acc[k] += t;
        }
    if (e != hipSuccess) return hip_fail(ctx, e, "kf_timings");
    for (int k = 0; k < 3; ++k) ms[k] = float(acc[k] / (last - first));
    ms[3] = float(last - first);
    return KF_OK;
}

}  // extern "C"
