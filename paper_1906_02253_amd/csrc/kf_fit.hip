// Seed, propagate and fit kernels: one lane per track, structure-of-arrays
// state so that element k of consecutive tracks is one coalesced access.
//
// arXiv:1906.02253 Sec. 2 (vectorised KF track fitting over sets of small
// matrices), Sec. 3.1 (layer-to-layer propagation with per-layer material in
// a constant field), Sec. 3.2 (seeds provided externally).
#include "kf_internal.hpp"
#include "kf_math.hpp"
#include "kf_mlp.hpp"

namespace kfmi {

// par and cov are stored in T, the state precision (FP32 in the mixed and
// FP32 modes); in registers the state is held in U (the update precision) and
// the covariance in C (the covariance-arithmetic precision).
template <typename T, typename C, typename U>
__device__ inline void load_state(const T* par, const T* cov, int64_t ld, int64_t i, U p[6],
                                  C P[21])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = U(par[k * ld + i]);
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = C(cov[k * ld + i]);
}

template <typename T, typename C, typename U>
__device__ inline void store_state(T* par, T* cov, int64_t ld, int64_t i, const U p[6],
                                   const C P[21])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) par[k * ld + i] = T(p[k]);
#pragma unroll
    for (int k = 0; k < 21; ++k) cov[k * ld + i] = T(P[k]);
}

// Propagate (p, P) to layer L.  The surface solve, the helix and the
// transport Jacobian run in T on the state rounded to T; the state itself
// stays in U (transport adds the T increments in U) and the covariance in C.
// s_init < 0: straight-line start; otherwise the learned start with
// prm.mlp_max_iter evaluations before the fallback to the straight-line
// start (counted in *fallbacks).
// FIELD: the parametrised field (kf_params.field_z0 > 0); MAT: the r-z material
// map.  Both are compile-time variants so that the uniform-field, per-layer
// material instantiation keeps its register budget.
template <typename T, typename C, typename U, bool FIELD, bool MAT>
__device__ inline int propagate_to(U p[6], C P[21], const kf_layer& L, const kf_params& prm,
                                   bool material, const MatMap& mat, T s_init, T* s_out, int* evals,
                                   int* fallbacks)
{
    const T kb = T(kKappa) * T(prm.bz);
    T pt[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pt[k] = T(p[k]);
    T s;
    if constexpr (FIELD) {
        // parametrised field: Runge-Kutta transport to the barrel's radius or
        // the disk's z; the covariance is carried by the helix Jacobian in the
        // path's mean effective axial field
        const T sth = Tr<T>::sin_(pt[5]);
        T l;
        T q[6];
        int st;
        if (L.kind != 0) {
            st = solve_disk_field(pt, T(L.r_or_z), prm, &l, q, evals);
        } else {
            T bx, by, bz0;
            field_at(T(prm.bz), T(prm.field_z0), pt[0], pt[1], pt[2], &bx, &by, &bz0);
            const T kb0 = T(kKappa) * bz0;
            st = solve_barrel_field(pt, T(L.r_or_z), prm, kb0, s_init >= T(0) ? s_init / sth : T(-1),
                                    prm.mlp_max_iter, &l, q, evals, fallbacks);
        }
        if (st) return st;
        field_transport(p, P, q, l, prm, L.kind, T(L.r_or_z));
        if (material) {
            if constexpr (MAT)
                add_material(p, P, L, mat, T(prm.mass));
            else
                add_scatter(p, P, L.kind, T(L.x0), T(prm.mass));
        }
        if (s_out) *s_out = l * sth;
        bool fin = true;
#pragma unroll
        for (int k = 0; k < 6; ++k) fin &= isfinite(p[k]);
        return fin ? 0 : KF_ST_NAN;
    }
    if (L.kind == 0) {
        const T h = -kb * pt[3];
        T sph, cph;
        Tr<T>::sincos_(pt[4], &sph, &cph);
        const T r_l = T(L.r_or_z);
        T s_hi;
        if (!barrel_bracket(pt[0], pt[1], cph, sph, h, r_l, &s_hi)) return KF_ST_UNREACHABLE;
        int st = solve_barrel(pt, h, cph, sph, r_l, s_hi, prm, s_init, prm.mlp_max_iter, &s, evals,
                              fallbacks);
        if (st) return st;
    } else {
        T st_, ct_;
        Tr<T>::sincos_(pt[5], &st_, &ct_);
        if (ct_ == T(0)) return KF_ST_UNREACHABLE;
        s = (T(L.r_or_z) - pt[2]) * st_ / ct_;
        *evals += 1;
        if (s < T(0)) return KF_ST_UNREACHABLE;
    }
    transport(p, P, s, kb, L.kind, T(L.r_or_z));
    if (material) {
        if constexpr (MAT)
            add_material(p, P, L, mat, T(prm.mass));
        else
            add_scatter(p, P, L.kind, T(L.x0), T(prm.mass));
    }
    if (s_out) *s_out = s;
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) fin &= isfinite(p[k]);
    return fin ? 0 : KF_ST_NAN;
}

// ---------------------------------------------------------------- seed
template <typename T>
__global__ __launch_bounds__(256) void seed_kernel(int64_t n, int64_t ld, int64_t n_hits,
                                                   const float* __restrict__ hx,
                                                   const float* __restrict__ hy,
                                                   const float* __restrict__ hz,
                                                   const int32_t* __restrict__ seed_hits, double bz,
                                                   T* __restrict__ par, T* __restrict__ cov,
                                                   T* __restrict__ chi2, int32_t* __restrict__ ndf,
                                                   uint32_t* __restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t a = seed_hits[i], b = seed_hits[ld + i], c = seed_hits[2 * ld + i];
    if (a < 0 || b < 0 || c < 0 || a >= n_hits || b >= n_hits || c >= n_hits) {
        chi2[i] = T(0);
        ndf[i] = -5;
        status[i] = KF_ST_BADINPUT;
        return;
    }
    // computed in FP64 in every precision mode: the curvature is a small
    // cross product of differences (sagitta << chord for stiff tracks)
    using D = double;
    const D x1 = hx[a], y1 = hy[a], z1 = hz[a];
    const D ax = D(hx[b]) - x1, ay = D(hy[b]) - y1;
    const D bx = D(hx[c]) - x1, by = D(hy[c]) - y1;
    const D d12 = sqrt(ax * ax + ay * ay);
    const D d13 = sqrt(bx * bx + by * by);
    const D ex = D(hx[c]) - D(hx[b]), ey = D(hy[c]) - D(hy[b]);
    const D d23 = sqrt(ex * ex + ey * ey);
    // signed curvature of the circle through the three points
    const D h = D(2) * (ax * by - ay * bx) / (d12 * d23 * d13);
    D w = D(0.5) * h * d13;
    w = w > D(1) ? D(1) : (w < D(-1) ? D(-1) : w);
    const D w2 = w * w;
    const D s13 = fabs(w) < D(1e-4) ? d13 * (D(1) + w2 * (D(1.0 / 6.0) + w2 * D(3.0 / 40.0)))
                                     : d13 * asin(w) / w;
    T p[6];
    T P[21];
    p[0] = T(x1);
    p[1] = T(y1);
    p[2] = T(z1);
    p[3] = T(-h / (kKappa * D(bz)));
    p[4] = T(wrap_phi(atan2(by, bx) - D(0.5) * h * s13));
    p[5] = T(atan2(s13, D(hz[c]) - z1));
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = T(0);
    P[pk(0, 0)] = P[pk(1, 1)] = P[pk(2, 2)] = T(1);
    P[pk(3, 3)] = T(4);
    P[pk(4, 4)] = P[pk(5, 5)] = T(0.01);
    store_state<T, T, T>(par, cov, ld, i, p, P);
    chi2[i] = T(0);
    ndf[i] = -5;
    status[i] = 0;
}

// ---------------------------------------------------------------- propagate
// LEARN: every lane of the wave runs to the network call (uniform control
// flow around the matrix-core instructions).
template <typename T, typename C, typename U, bool LEARN, bool FIELD, bool MAT>
__global__ __launch_bounds__(256) void propagate_kernel(int64_t n, int64_t ld, T* __restrict__ par,
                                                        T* __restrict__ cov,
                                                        uint32_t* __restrict__ status,
                                                        const int32_t* __restrict__ target,
                                                        const kf_layer* __restrict__ layers,
                                                        int n_layers, kf_params prm, int material,
                                                        MatMap mat, float* __restrict__ path_len,
                                                        int32_t* __restrict__ iters, MlpDev mlp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!LEARN && i >= n) return;
    const bool inb = i < n;
    const int32_t l = inb ? target[i] : -1;
    uint32_t st = inb ? status[i] : 0u;
    if (l >= n_layers) st |= KF_ST_BADINPUT;
    const bool active = inb && l >= 0 && !(st & kFreezeMask);
    if (!LEARN && !active) {
        status[i] = st;
        if (path_len) path_len[i] = 0.0f;
        if (iters) iters[i] = 0;
        return;
    }
    U p[6];
    C P[21];
    kf_layer L;
    if (active) {
        load_state(par, cov, ld, i, p, P);
        L = layers[l];
    }
    T s_init = T(-1);
    if (LEARN) {
        float f[kMlpIn] = {0, 0, 0, 0, 0, 0, 0, 0};
        const bool want = active && L.kind == 0;
        if (want) {
            T pt[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) pt[k] = T(p[k]);
            mlp_features(pt, L, prm, f);
        }
        const uint64_t wmask = __ballot(want);
        const float y = wmask ? mlp_wave(mlp, f, wmask) : 0.0f;
        if (want) s_init = T(mlp_guess(f, y));
        if (!inb) return;
        if (!active) {
            status[i] = st;
            if (path_len) path_len[i] = 0.0f;
            if (iters) iters[i] = 0;
            return;
        }
    }
    T s = T(0);
    int ev = 0, fb = 0;
    int r = propagate_to<T, C, U, FIELD, MAT>(p, P, L, prm, material != 0, mat, s_init, &s, &ev, &fb);
    if (fb) st |= KF_ST_FALLBACK;
    if (r) {
        st |= (uint32_t)r;
    } else {
        store_state(par, cov, ld, i, p, P);
    }
    status[i] = st;
    if (path_len) path_len[i] = float(s);
    if (iters) iters[i] = ev;
}

// ---------------------------------------------------------------- fit
struct FitArgs {
    int64_t n, ld;
    void* par;
    void* cov;
    void* chi2;
    int32_t* ndf;
    uint32_t* status;
    const float *hx, *hy, *hz, *hsu, *hsv;
    const int32_t* layer_seq;
    const int32_t* hit_idx;
    int64_t n_hits;
    const kf_layer* layers;
    int n_layers;
    kf_params prm;
    int material;
    MatMap mat;                  // r-z material map (x0 == nullptr: none)
    MlpDev mlp;                  // learned guess (KF_INIT_MLP)
};

// Steps [k0, k1) of the fit.  init: start a fresh fit (chi2 = 0, ndf = -5).
// LEARN: every lane of the wave walks all steps (finished lanes idle), so
// that the network call at each step is in uniform control flow.
template <typename T, typename C, typename U, bool LEARN, bool FIELD, bool MAT>
__global__ __launch_bounds__(256) void fit_kernel(FitArgs a, int k0, int k1, int init)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!LEARN && i >= a.n) return;
    const bool inb = i < a.n;
    const int64_t ld = a.ld;
    T* par = (T*)a.par;
    T* cov = (T*)a.cov;
    T* chi2p = (T*)a.chi2;
    uint32_t st = (init || !inb) ? 0u : a.status[i];
    int32_t ndf = (init || !inb) ? -5 : a.ndf[i];
    U chi2 = (init || !inb) ? U(0) : U(chi2p[i]);
    bool alive = inb && !(st & kFreezeMask);
    if (!LEARN && !alive) return;
    const bool was_alive = alive;
    // the state stays in U between steps (rounded to T only when stored)
    U p[6];
    C P[21];
    if (alive) load_state(par, cov, ld, i, p, P);
    bool touched = false;
    for (int k = k0; k < k1; ++k) {
        if (!LEARN && !alive) break;
        int32_t l = -1;
        if (alive) {
            l = a.layer_seq ? a.layer_seq[(int64_t)k * ld + i] : k;
            if (l < 0) {
                alive = false;
            } else if (l >= a.n_layers) {
                st |= KF_ST_BADINPUT;
                alive = false;
            }
        }
        kf_layer L;
        if (alive) L = a.layers[l];
        T s_init = T(-1);
        if (LEARN) {
            float f[kMlpIn] = {0, 0, 0, 0, 0, 0, 0, 0};
            const bool want = alive && L.kind == 0;
            if (want) {
                T pt[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) pt[q] = T(p[q]);
                mlp_features(pt, L, a.prm, f);
            }
            const uint64_t wmask = __ballot(want);
            const float y = wmask ? mlp_wave(a.mlp, f, wmask) : 0.0f;
            if (want) s_init = T(mlp_guess(f, y));
        }
        if (!alive) continue;
        // the step's hit is read before the propagation, so that its two
        // dependent loads (index, then coordinates) overlap the state's loads
        // and the transport instead of following them
        const int32_t hi = a.hit_idx[(int64_t)k * ld + i];
        const bool has_hit = hi >= 0 && hi < a.n_hits;
        float hx = 0.f, hy = 0.f, hz = 0.f, hsu = 0.f, hsv = 0.f;
        if (has_hit) {
            hx = a.hx[hi];
            hy = a.hy[hi];
            hz = a.hz[hi];
            hsu = a.hsu[hi];
            hsv = a.hsv[hi];
        }
        int ev = 0, fb = 0;
        int r = propagate_to<T, C, U, FIELD, MAT>(p, P, L, a.prm, a.material != 0, a.mat, s_init,
                                                   (T*)nullptr, &ev, &fb);
        touched = true;
        if (fb) st |= KF_ST_FALLBACK;
        if (r) {
            st |= (uint32_t)r;
            alive = false;
            continue;
        }
        if (hi >= a.n_hits) {
            st |= KF_ST_BADINPUT;
            alive = false;
            continue;
        }
        if (has_hit) {
            HitFrame<U> f = hit_frame<U>(hx, hy, hz, hsu, hsv);
            U c2 = U(0);
            r = kf_update<U, C, U>(p, P, f, L.kind, &c2);
            if (r) {
                st |= (uint32_t)r;
                alive = false;
                continue;
            }
            // rounded to storage precision every step, so one launch per step
            // and one launch for all steps give identical results
            chi2 = U(T(chi2 + c2));
            ndf += 2;
        }
    }
    if (!was_alive) return;
    // on failure the registers hold the last good state (a failed solve or
    // update leaves them untouched)
    if (touched) store_state(par, cov, ld, i, p, P);
    chi2p[i] = T(chi2);
    a.ndf[i] = ndf;
    a.status[i] = st;
}

// ---------------------------------------------------------------- launchers
static inline dim3 grid_for(int64_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

hipError_t launch_seed(const kf_ctx* ctx, const kf_hits* h, const int32_t* seed_hits,
                       kf_tracks* out, int flags, hipStream_t s)
{
    if (out->n == 0) return hipSuccess;
    const int prec = flags & KF_PREC_MASK;
    dim3 g = grid_for(out->n, 256);
    if (prec == KF_PREC_FP64)
        seed_kernel<double><<<g, 256, 0, s>>>(out->n, out->ld, h->n, h->x, h->y, h->z, seed_hits,
                                              ctx->params.bz, (double*)out->par, (double*)out->cov,
                                              (double*)out->chi2, out->ndf, out->status);
    else
        seed_kernel<float><<<g, 256, 0, s>>>(out->n, out->ld, h->n, h->x, h->y, h->z, seed_hits,
                                             ctx->params.bz, (float*)out->par, (float*)out->cov,
                                             (float*)out->chi2, out->ndf, out->status);
    return hipGetLastError();
}

hipError_t launch_propagate(const kf_ctx* ctx, kf_tracks* t, const int32_t* target, float* path_len,
                            int32_t* iters, int flags, hipStream_t s)
{
    if (t->n == 0) return hipSuccess;
    const int prec = flags & KF_PREC_MASK;
    const int material = (flags & KF_NO_MATERIAL) ? 0 : 1;
    const bool learn = (flags & KF_INIT_MLP) != 0;
    const MlpDev m = ctx->mlp.dev();
    dim3 g = grid_for(t->n, 256);
    const bool field = ctx->params.field_z0 > 0.0, map = ctx->mat.x0 != nullptr;
#define KF_PROP1(TT, CC, UU, LL, FF, MM)                                                             \
    propagate_kernel<TT, CC, UU, LL, FF, MM><<<g, 256, 0, s>>>(t->n, t->ld, (TT*)t->par, (TT*)t->cov, \
                                                               t->status, target, ctx->d_layers,   \
                                                               ctx->n_layers, ctx->params,         \
                                                               material, ctx->mat, path_len, iters, \
                                                               m)
#define KF_PROP(TT, CC, UU, LL)                                                                      \
    do {                                                                                             \
        if (field) {                                                                                 \
            if (map) KF_PROP1(TT, CC, UU, LL, true, true);                                           \
            else KF_PROP1(TT, CC, UU, LL, true, false);                                              \
        } else {                                                                                     \
            if (map) KF_PROP1(TT, CC, UU, LL, false, true);                                          \
            else KF_PROP1(TT, CC, UU, LL, false, false);                                             \
        }                                                                                            \
    } while (0)
    if (prec == KF_PREC_FP64) {
        if (learn) KF_PROP(double, double, double, true);
        else KF_PROP(double, double, double, false);
    } else if (prec == KF_PREC_FP32) {
        if (learn) KF_PROP(float, float, float, true);
        else KF_PROP(float, float, float, false);
    } else {
        if (learn) KF_PROP(float, double, double, true);
        else KF_PROP(float, double, double, false);
    }
#undef KF_PROP
#undef KF_PROP1
    return hipGetLastError();
}

template <typename T, typename C, typename U, bool LEARN>
static void fit_launch(const FitArgs& a, dim3 g, int k0, int k1, int init, bool field, bool map,
                       hipStream_t s)
{
    if (field) {
        if (map) fit_kernel<T, C, U, LEARN, true, true><<<g, 256, 0, s>>>(a, k0, k1, init);
        else fit_kernel<T, C, U, LEARN, true, false><<<g, 256, 0, s>>>(a, k0, k1, init);
    } else {
        if (map) fit_kernel<T, C, U, LEARN, false, true><<<g, 256, 0, s>>>(a, k0, k1, init);
        else fit_kernel<T, C, U, LEARN, false, false><<<g, 256, 0, s>>>(a, k0, k1, init);
    }
}

hipError_t launch_fit(const kf_ctx* ctx, kf_tracks* t, const kf_hits* h, const int32_t* layer_seq,
                      const int32_t* hit_idx, int32_t max_steps, int flags, hipStream_t s)
{
    if (t->n == 0) return hipSuccess;
    FitArgs a;
    a.n = t->n;
    a.ld = t->ld;
    a.par = t->par;
    a.cov = t->cov;
    a.chi2 = t->chi2;
    a.ndf = t->ndf;
    a.status = t->status;
    a.hx = h->x;
    a.hy = h->y;
    a.hz = h->z;
    a.hsu = h->su;
    a.hsv = h->sv;
    a.layer_seq = layer_seq;
    a.hit_idx = hit_idx;
    a.n_hits = h->n;
    a.layers = ctx->d_layers;
    a.n_layers = ctx->n_layers;
    a.prm = ctx->params;
    a.material = (flags & KF_NO_MATERIAL) ? 0 : 1;
    a.mat = ctx->mat;
    a.mlp = ctx->mlp.dev();
    const bool learn = (flags & KF_INIT_MLP) != 0;
    const int prec = flags & KF_PREC_MASK;
    dim3 g = grid_for(t->n, 256);
    const bool per_layer = (flags & KF_PER_LAYER) != 0;
    const bool field = ctx->params.field_z0 > 0.0, map = ctx->mat.x0 != nullptr;
    const int nlaunch = per_layer ? max_steps : 1;
    for (int k = 0; k < nlaunch; ++k) {
        const int k0 = per_layer ? k : 0;
        const int k1 = per_layer ? k + 1 : max_steps;
        const int init = k == 0;
        if (prec == KF_PREC_FP64) {
            if (learn) fit_launch<double, double, double, true>(a, g, k0, k1, init, field, map, s);
            else fit_launch<double, double, double, false>(a, g, k0, k1, init, field, map, s);
        } else if (prec == KF_PREC_FP32) {
            if (learn) fit_launch<float, float, float, true>(a, g, k0, k1, init, field, map, s);
            else fit_launch<float, float, float, false>(a, g, k0, k1, init, field, map, s);
        } else {
            if (learn) fit_launch<float, double, double, true>(a, g, k0, k1, init, field, map, s);
            else fit_launch<float, double, double, false>(a, g, k0, k1, init, field, map, s);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kfmi
