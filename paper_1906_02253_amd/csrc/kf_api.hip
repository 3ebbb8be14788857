// C-ABI entry points of libkfmi.so: argument validation, context and
// workspace management, dispatch to the kernel launchers.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "kf_internal.hpp"

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
            L.nbin_phi > 4096 || L.nbin_2 > 4096 || !(L.x0 >= 0.0f) ||
            (L.kind == 0 && !(L.r_or_z > 0.0f)))
            return fail(nullptr, KF_EINVAL, "kf_create: invalid layer %d", i);
    }
    kf_params p;
    if (params) {
        p = *params;
    } else {
        p.bz = 3.8f;
        p.chi2_cut = 30.0f;
        p.max_cands = 6;
        p.max_newton = 10;
        p.newton_tol = 1e-4f;
        p.mass = 0.13957f;
        p.max_miss = 2;
        p.mlp_max_iter = 3;
    }
    if (!(p.bz != 0.0f) || !(p.chi2_cut > 0.0f) || p.max_cands < 1 || p.max_cands > 8 ||
        p.max_newton < 1 || p.max_newton > 64 || !(p.newton_tol > 0.0f) || !(p.mass >= 0.0f) ||
        p.max_miss < 0 || p.mlp_max_iter < 1 || p.mlp_max_iter > 64)
        return fail(nullptr, KF_EINVAL, "kf_create: invalid parameters");
    kf_ctx* ctx = new kf_ctx();
    ctx->n_layers = n_layers;
    memcpy(ctx->layers, layers, sizeof(kf_layer) * n_layers);
    ctx->params = p;
    hipError_t e = hipGetDevice(&ctx->device);
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

}  // extern "C"
