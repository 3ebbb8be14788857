// Device-side Kalman-filter arithmetic for gfx950: helix transport, the
// propagate-to-surface solves, the transport Jacobian, scattering noise and
// the 2D-hit update.  One lane owns one track (or candidate); matrices live
// in registers.  T = state and transport precision (helix, Jacobian),
// C = covariance precision, U = update precision.
//
// Method references (arXiv:1906.02253): Sec. 1 (traditional Kalman filter),
// Sec. 2 (vectorised KF fit/find over many small matrices), Sec. 3.1
// (layer-to-layer propagation, per-layer material, constant field).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kf.h"
#include "kf_matmap.hpp"
#include "kf_steer.hpp"

// Device functions that a host-side operation counter can also instantiate.
#define KF_HD __host__ __device__

namespace kfmi {

constexpr double kKappa = 0.00299792458;   // GeV / (T cm)
constexpr double kPi = 3.14159265358979323846;
constexpr float kNextBarrelEps = 0.05f;    // cm
constexpr float kDiskAheadEps = 0.05f;     // cm
constexpr float kMaxFieldPath = 1000.0f;   // cm: longest 3D path the field's Runge-Kutta solves search

// packed upper-triangle index of a symmetric 6x6
__host__ __device__ constexpr int pk(int i, int j)
{
    return i <= j ? i * (11 - i) / 2 + j : j * (11 - j) / 2 + i;
}

template <typename T> struct Tr;
template <> struct Tr<float> {
    KF_HD static inline void sincos_(float x, float* s, float* c) { sincosf(x, s, c); }
    KF_HD static inline float sqrt_(float x) { return sqrtf(x); }
    KF_HD static inline float abs_(float x) { return fabsf(x); }
    KF_HD static inline float atan2_(float y, float x) { return atan2f(y, x); }
    KF_HD static inline float log_(float x) { return logf(x); }
    KF_HD static inline float fmod_(float x, float y) { return fmodf(x, y); }
    KF_HD static inline float asin_(float x) { return asinf(x); }
    KF_HD static inline float cos_(float x) { return cosf(x); }
    KF_HD static inline float sin_(float x) { return sinf(x); }
    KF_HD static inline float floor_(float x) { return floorf(x); }
    KF_HD static inline float min_(float a, float b) { return fminf(a, b); }
};
template <> struct Tr<double> {
    KF_HD static inline void sincos_(double x, double* s, double* c) { sincos(x, s, c); }
    KF_HD static inline double sqrt_(double x) { return sqrt(x); }
    KF_HD static inline double abs_(double x) { return fabs(x); }
    KF_HD static inline double atan2_(double y, double x) { return atan2(y, x); }
    KF_HD static inline double log_(double x) { return log(x); }
    KF_HD static inline double fmod_(double x, double y) { return fmod(x, y); }
    KF_HD static inline double asin_(double x) { return asin(x); }
    KF_HD static inline double cos_(double x) { return cos(x); }
    KF_HD static inline double sin_(double x) { return sin(x); }
    KF_HD static inline double floor_(double x) { return floor(x); }
    KF_HD static inline double min_(double a, double b) { return fmin(a, b); }
};

template <typename T>
KF_HD inline T wrap_phi(T a)
{
    const T pi = T(kPi), tpi = T(2.0 * kPi);
    if (a > pi) a -= tpi;
    if (a <= -pi) a += tpi;
    return a;
}

// sin(u)/u given sin(u)
template <typename T>
KF_HD inline T sinc_of(T u, T su)
{
    return Tr<T>::abs_(u) < T(1e-4) ? T(1) - u * u * T(1.0 / 6.0) : su / u;
}

// d/du [sin(u)/u]; Taylor series where the closed form cancels
template <typename T>
KF_HD inline T dsinc_of(T u, T su, T cu)
{
    if (Tr<T>::abs_(u) < T(0.5)) {
        T u2 = u * u;
        return u * (T(-1.0 / 3.0) +
                    u2 * (T(1.0 / 30.0) +
                          u2 * (T(-1.0 / 840.0) + u2 * (T(1.0 / 45360.0) + u2 * T(-1.0 / 3991680.0)))));
    }
    return (u * cu - su) / (u * u);
}

// Helix point at transverse arc length s (sinc form, exact as h -> 0).
template <typename T>
struct HelixPoint {
    T X, Y;          // transverse position
    T cph, sph;      // direction cos/sin of phi(s)
    T ca, sa;        // cos/sin(phi + h s / 2)
    T sc, su, cu;    // sinc(u), sin(u), cos(u), u = h s / 2
};

template <typename T>
KF_HD inline HelixPoint<T> helix_at(T x, T y, T phi, T h, T s)
{
    HelixPoint<T> q;
    T u = T(0.5) * h * s;
    Tr<T>::sincos_(u, &q.su, &q.cu);
    Tr<T>::sincos_(phi + u, &q.sa, &q.ca);
    q.sc = sinc_of(u, q.su);
    q.X = x + s * q.ca * q.sc;
    q.Y = y + s * q.sa * q.sc;
    q.cph = q.ca * q.cu - q.sa * q.su;
    q.sph = q.sa * q.cu + q.ca * q.su;
    return q;
}

// Straight-line (tangent) intersection with radius r_l: the plain initial guess.
template <typename T>
KF_HD inline T line_guess(T x, T y, T cphi, T sphi, T r_l)
{
    T pu = x * cphi + y * sphi;
    T disc = pu * pu - (x * x + y * y) + r_l * r_l;
    return disc > T(0) ? -pu + Tr<T>::sqrt_(disc) : -pu;
}

// Bracket of the outward crossing: [0, arc length to the point of largest
// radius].  Returns false when the circle never reaches r_l.
template <typename T>
KF_HD inline bool barrel_bracket(T x, T y, T cphi, T sphi, T h, T r_l, T* s_hi)
{
    if (h == T(0)) {
        *s_hi = T(1e30);
        return true;
    }
    T inv = T(1) / h;
    T cx = x - sphi * inv, cy = y + cphi * inv;
    T R = Tr<T>::abs_(inv);
    T dc = Tr<T>::sqrt_(cx * cx + cy * cy);
    if (dc + R < r_l) return false;
    T v0x = x - cx, v0y = y - cy;
    T v1x = R * cx / dc, v1y = R * cy / dc;
    T alpha = Tr<T>::atan2_(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y);
    // |alpha| <= pi, so the sweep in the direction of motion reduced to
    // [0, 2 pi) needs no remainder
    T sw = h > T(0) ? alpha : -alpha;
    if (sw < T(0)) sw += T(2.0 * kPi);
    *s_hi = sw * Tr<T>::abs_(inv);
    return true;
}

// Bracketed Newton on r(s) = r_l from s0 within [s_lo, s_hi]; converged when
// |r - r_l| < tol, then one more Newton step.  Returns 0 or KF_ST_NOCONV;
// *evals counts evaluations of r(s).
template <typename T>
KF_HD inline int newton_barrel(T x, T y, T phi, T h, T r_l, T s, T s_lo, T s_hi, int max_it,
                                    T tol, T* s_out, int* evals)
{
    if (s < s_lo) s = s_lo;
    if (s > s_hi) s = s_hi;
    for (int it = 1; it <= max_it; ++it) {
        HelixPoint<T> q = helix_at(x, y, phi, h, s);
        T r = Tr<T>::sqrt_(q.X * q.X + q.Y * q.Y);
        T res = r - r_l;
        T drds = (q.X * q.cph + q.Y * q.sph) / r;
        if (res < T(0)) {
            if (s > s_lo) s_lo = s;
        } else {
            if (s < s_hi) s_hi = s;
        }
        if (Tr<T>::abs_(res) < tol) {
            if (drds > T(0)) s -= res / drds;
            *s_out = s;
            *evals += it;
            return 0;
        }
        T sn = s - res / drds;
        if (!(drds > T(0)) || !(sn > s_lo && sn < s_hi)) sn = T(0.5) * (s_lo + s_hi);
        s = sn;
    }
    *s_out = s;
    *evals += max_it;
    return KF_ST_NOCONV;
}

// Transport of (p, P) by arc length s to a surface: new state, F P F^T.
// kind 0: barrel (path length from r(s) = r_l); 1: disk at z = zd.  The
// helix and the Jacobian are evaluated in T; the state p is held in S (S may
// be wider than T: the position and azimuth then advance by increments
// computed in T and added in S, so the predicted state carries no rounding
// to T before the update that consumes it); F P F^T is accumulated in C.
template <typename T, typename C, typename S>
KF_HD inline void transport(S p[6], C P[21], T s, T kb, int kind, T zd)
{
    const T x = T(p[0]), y = T(p[1]), z = T(p[2]), c = T(p[3]), phi = T(p[4]), th = T(p[5]);
    const T h = -kb * c;
    HelixPoint<T> q = helix_at(x, y, phi, h, s);
    T st, ct;
    Tr<T>::sincos_(th, &st, &ct);
    const T cot = ct / st;
    const T u = T(0.5) * h * s;
    const T dsc = dsinc_of(u, q.su, q.cu);

    // partial derivatives at fixed s
    const T D03 = -kb * (T(0.5) * s * s * (q.ca * dsc - q.sa * q.sc));
    const T D13 = -kb * (T(0.5) * s * s * (q.sa * dsc + q.ca * q.sc));
    const T D04 = -s * q.sa * q.sc;
    const T D14 = s * q.ca * q.sc;
    const T D43 = -kb * s;
    const T D25 = -s / (st * st);
    // derivative of the state with respect to s
    const T f0 = q.cph, f1 = q.sph, f2 = cot, f4 = h;
    // derivative of s with respect to the starting state
    T d0 = 0, d1 = 0, d2 = 0, d3 = 0, d4 = 0, d5 = 0;
    if (kind == 0) {
        T den = T(-1) / (q.X * f0 + q.Y * f1);
        d0 = q.X * den;
        d1 = q.Y * den;
        d3 = (q.X * D03 + q.Y * D13) * den;
        d4 = (q.X * D04 + q.Y * D14) * den;
    } else {
        d2 = -st / ct;
        d5 = (zd - z) / (ct * ct);
    }
    const C F[4][6] = {
        {T(1) + f0 * d0, f0 * d1, f0 * d2, D03 + f0 * d3, D04 + f0 * d4, f0 * d5},
        {f1 * d0, T(1) + f1 * d1, f1 * d2, D13 + f1 * d3, D14 + f1 * d4, f1 * d5},
        {f2 * d0, f2 * d1, T(1) + f2 * d2, f2 * d3, f2 * d4, D25 + f2 * d5},
        {f4 * d0, f4 * d1, f4 * d2, D43 + f4 * d3, T(1) + f4 * d4, f4 * d5},
    };
    // A = F P for the four general rows; rows 3 and 5 of F are unit rows
    C A[4][6];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            C acc = C(0);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc += F[r][k] * P[pk(k, j)];
            A[r][j] = acc;
        }
    // P' = A F^T (upper triangle).  Row of P' for F-row index: general rows use A,
    // unit rows 3 and 5 use P itself.
    C Pn[21];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            // pick row i of (F P): general or unit
            const int ri = i == 0 ? 0 : i == 1 ? 1 : i == 2 ? 2 : i == 4 ? 3 : -1;
            const int rj = j == 0 ? 0 : j == 1 ? 1 : j == 2 ? 2 : j == 4 ? 3 : -1;
            C v;
            if (rj < 0) {
                // column j of F^T is e_j: (F P)_{i j}
                v = ri >= 0 ? A[ri][j] : P[pk(i, j)];
            } else {
                C acc = C(0);
#pragma unroll
                for (int k = 0; k < 6; ++k) acc += (ri >= 0 ? A[ri][k] : P[pk(i, k)]) * F[rj][k];
                v = acc;
            }
            Pn[pk(i, j)] = v;
        }
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = Pn[k];
    p[0] = p[0] + S(s * q.ca * q.sc);
    p[1] = p[1] + S(s * q.sa * q.sc);
    p[2] = p[2] + S(s * cot);
    p[4] = wrap_phi(p[4] + S(h * s));
}

// Multiple-scattering process noise of a layer (PDG Highland width), added to
// the (c, phi, theta) block at the propagated state.  Evaluated in T on the
// state (held in S) rounded to T.
template <typename T, typename C, typename S>
KF_HD inline void add_scatter(const S ps[6], C P[21], int kind, T x0, T mass)
{
    if (!(x0 > T(0))) return;
    T p[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = T(ps[k]);
    T st, ct;
    Tr<T>::sincos_(p[5], &st, &ct);
    T cosa;
    if (kind == 0) {
        T sph, cph;
        Tr<T>::sincos_(p[4], &sph, &cph);
        T r = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
        cosa = st * (cph * p[0] + sph * p[1]) / r;
    } else {
        cosa = ct;
    }
    cosa = Tr<T>::abs_(cosa);
    if (cosa < T(1e-6)) cosa = T(1e-6);
    const T t = x0 / cosa;
    const T pm = T(1) / (Tr<T>::abs_(p[3]) * st);
    const T b2 = pm * pm / (pm * pm + mass * mass);
    const T beta = Tr<T>::sqrt_(b2);
    const T th0 = T(0.0136) / (beta * pm) * Tr<T>::sqrt_(t) * (T(1) + T(0.038) * Tr<T>::log_(t / b2));
    const T t2 = th0 * th0;
    const T cot = ct / st;
    P[pk(4, 4)] += C(t2 / (st * st));
    P[pk(5, 5)] += C(t2);
    P[pk(3, 5)] += C(-p[3] * cot * t2);
    P[pk(3, 3)] += C(p[3] * p[3] * cot * cot * t2);
}

// Mean ionisation loss in silicon [MeV cm^2/g]: the Bethe formula with the
// maximum energy transfer to an electron, no density effect (PDG, passage of
// particles through matter); Z/A = 0.49848, I = 173 eV.  p, m in GeV.
template <typename T>
KF_HD inline T bethe_si(T p, T m)
{
    const T me = T(0.51099895), K = T(0.307075), za = T(0.49848), I = T(173e-6);
    const T M = m * T(1e3), pm = p * T(1e3);
    const T E = Tr<T>::sqrt_(pm * pm + M * M);
    const T beta = pm / E, gam = E / M;
    const T b2 = beta * beta;
    const T bg2 = b2 * gam * gam;
    const T r = me / M;
    const T tmax = T(2) * me * bg2 / (T(1) + T(2) * gam * r + r * r);
    return K * za / b2 * (T(0.5) * Tr<T>::log_(T(2) * me * bg2 * tmax / (I * I)) - b2);
}

// Material effects at the crossing of layer L by the propagated state:
// without a map, the layer's scattering noise; with one, the cell at the
// crossing point gives the thickness for the noise and the areal density for
// the mean energy loss (|p| lowered at fixed direction, c' = c p/p', the
// covariance's c row and column scaled by dc'/dc = (p/p')^3 E'/E).
// The state is held in S; the lookup takes the crossing point in double, the
// noise and the loss are evaluated in T, and q/pT is scaled in S.
template <typename T, typename C, typename S>
KF_HD inline void add_material(S ps[6], C P[21], const kf_layer& L, const MatMap& m, T mass)
{
    if (!m.x0) {
        add_scatter(ps, P, L.kind, T(L.x0), mass);
        return;
    }
    const double r = sqrt((double)ps[0] * (double)ps[0] + (double)ps[1] * (double)ps[1]);
    int ir = (int)floor(r / (m.r_max / m.nr));
    int iz = (int)floor(((double)ps[2] - m.z_min) / ((m.z_max - m.z_min) / m.nz));
    ir = ir < 0 ? 0 : (ir >= m.nr ? m.nr - 1 : ir);
    iz = iz < 0 ? 0 : (iz >= m.nz ? m.nz - 1 : iz);
    const T x0 = T(m.x0[ir * m.nz + iz]), xi = T(m.xi[ir * m.nz + iz]);
    add_scatter(ps, P, L.kind, x0, mass);
    if (!(xi > T(0))) return;
    T p[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = T(ps[k]);
    T st, ct;
    Tr<T>::sincos_(p[5], &st, &ct);
    T cosa;
    if (L.kind == 0) {
        T sph, cph;
        Tr<T>::sincos_(p[4], &sph, &cph);
        const T rr = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
        cosa = st * (cph * p[0] + sph * p[1]) / rr;
    } else {
        cosa = ct;
    }
    cosa = Tr<T>::abs_(cosa);
    if (cosa < T(1e-6)) cosa = T(1e-6);
    const T pm = T(1) / (Tr<T>::abs_(p[3]) * st);
    const T E = Tr<T>::sqrt_(pm * pm + mass * mass);
    T dE = bethe_si(pm, mass) * xi / cosa * T(1e-3);
    const T cap = T(0.5) * (E - mass);
    if (dE > cap) dE = cap;
    const T E1 = E - dE;
    const T p1 = Tr<T>::sqrt_(E1 * E1 - mass * mass);
    const T ratio = pm / p1;
    const C J = C(ratio * ratio * ratio * (E1 / E));
    ps[3] *= S(ratio);
#pragma unroll
    for (int k = 0; k < 6; ++k) P[pk(3, k)] *= J;
    P[pk(3, 3)] *= J;
}

// Local frame of a hit: u along phi at the hit's azimuth, v along z (barrel)
// or r (disk).  H has two rows with entries only in the x, y, z columns.
template <typename U>
struct HitFrame {
    U c, s;          // cos/sin of the hit azimuth
    U hx, hy, hz;
    U vu, vv;        // sigma^2
};

template <typename U>
KF_HD inline HitFrame<U> hit_frame(float x, float y, float z, float su, float sv)
{
    HitFrame<U> f;
    f.hx = U(x);
    f.hy = U(y);
    f.hz = U(z);
    U rho = Tr<U>::sqrt_(f.hx * f.hx + f.hy * f.hy);
    f.c = f.hx / rho;
    f.s = f.hy / rho;
    f.vu = U(su) * U(su);
    f.vv = U(sv) * U(sv);
    return f;
}

// chi2 of a hit against a predicted position (x, y, z) and the position
// block of its covariance, without updating
template <typename U>
KF_HD inline U hit_chi2_pos(U x, U y, U z, U P00, U P01, U P02, U P11, U P12, U P22,
                            const HitFrame<U>& f, int kind)
{
    const U c = f.c, s = f.s;
    const U ru = -s * (f.hx - x) + c * (f.hy - y);
    // first three rows of P H^T (what S needs)
    const U b00 = -s * P00 + c * P01, b01 = -s * P01 + c * P11;
    U S00 = -s * b00 + c * b01 + f.vu;
    U rv, S01, S11;
    if (kind == 0) {
        rv = f.hz - z;
        S01 = -s * P02 + c * P12;
        S11 = P22 + f.vv;
    } else {
        rv = c * (f.hx - x) + s * (f.hy - y);
        const U b10 = c * P00 + s * P01, b11 = c * P01 + s * P11;
        S01 = -s * b10 + c * b11;
        S11 = c * b10 + s * b11 + f.vv;
    }
    const U det = S00 * S11 - S01 * S01;
    if (!(det > U(0)) || !(S00 > U(0))) return U(1e30);
    return (ru * ru * S11 - U(2) * ru * rv * S01 + rv * rv * S00) / det;
}

template <typename T, typename C, typename U>
KF_HD inline U hit_chi2(const T p[6], const C P[21], const HitFrame<U>& f, int kind)
{
    return hit_chi2_pos<U>(U(p[0]), U(p[1]), U(p[2]), U(P[pk(0, 0)]), U(P[pk(0, 1)]),
                           U(P[pk(0, 2)]), U(P[pk(1, 1)]), U(P[pk(1, 2)]), U(P[pk(2, 2)]), f, kind);
}

// Kalman update with a 2D hit.  Gain K = P H^T S^-1, state x + K r, covariance
// in Joseph form (I - K H) P (I - K H)^T + K V K^T, evaluated as
// M = P - K (H P), P+ = M - (M H^T) K^T + K V K^T.  Returns status bits.
template <typename T, typename C, typename U>
KF_HD inline int kf_update(T p[6], C P[21], const HitFrame<U>& f, int kind, U* chi2_out)
{
    const U c = f.c, s = f.s;
    U Pu[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) Pu[k] = U(P[k]);
    U ru = -s * (f.hx - U(p[0])) + c * (f.hy - U(p[1]));
    U rv = kind == 0 ? f.hz - U(p[2]) : c * (f.hx - U(p[0])) + s * (f.hy - U(p[1]));
    // B = P H^T (6x2)
    U B0[6], B1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        B0[i] = -s * Pu[pk(i, 0)] + c * Pu[pk(i, 1)];
        B1[i] = kind == 0 ? Pu[pk(i, 2)] : c * Pu[pk(i, 0)] + s * Pu[pk(i, 1)];
    }
    U S00 = -s * B0[0] + c * B0[1] + f.vu;
    U S01 = -s * B1[0] + c * B1[1];
    U S11 = (kind == 0 ? B1[2] : c * B1[0] + s * B1[1]) + f.vv;
    U det = S00 * S11 - S01 * S01;
    if (!(det > U(0)) || !(S00 > U(0))) return KF_ST_NONPD;
    U idet = U(1) / det;
    U I00 = S11 * idet, I01 = -S01 * idet, I11 = S00 * idet;
    *chi2_out = ru * (I00 * ru + I01 * rv) + rv * (I01 * ru + I11 * rv);
    U K0[6], K1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        K0[i] = B0[i] * I00 + B1[i] * I01;
        K1[i] = B0[i] * I01 + B1[i] * I11;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = T(U(p[i]) + K0[i] * ru + K1[i] * rv);
    p[4] = wrap_phi(p[4]);
    // M = P - K B^T: needed in full for columns 0..2 and in the upper triangle
    U Mc[6][3];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Mc[i][j] = Pu[pk(i, j)] - K0[i] * B0[j] - K1[i] * B1[j];
    // N = M H^T
    U N0[6], N1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        N0[i] = -s * Mc[i][0] + c * Mc[i][1];
        N1[i] = kind == 0 ? Mc[i][2] : c * Mc[i][0] + s * Mc[i][1];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            U m = j < 3 ? Mc[i][j] : Pu[pk(i, j)] - K0[i] * B0[j] - K1[i] * B1[j];
            U v = m - N0[i] * K0[j] - N1[i] * K1[j] + f.vu * K0[i] * K0[j] + f.vv * K1[i] * K1[j];
            P[pk(i, j)] = C(v);
        }
    bool fin = true;
#pragma unroll
    for (int i = 0; i < 6; ++i) fin &= isfinite(p[i]);
    return fin ? 0 : KF_ST_NAN;
}

// ---------------------------------------------------------------- parametrised field
// Solenoid-like, axially symmetric and divergence free: Bz = B0 / (1 +
// (z/Z0)^2) and Br = -(r/2) dBz/dz (paper Sec. 3.1 supports parametrised
// fields; the model is ours).
template <typename T>
KF_HD inline void field_at(T B0, T Z0, T x, T y, T z, T* bx, T* by, T* bz)
{
    const T u = z / Z0;
    const T g = T(1) / (T(1) + u * u);
    const T k = B0 * z / (Z0 * Z0) * g * g;    // -(1/2) dBz/dz
    *bx = k * x;
    *by = k * y;
    *bz = B0 * g;
}

// State after 3D path length l: fourth-order Runge-Kutta on (position,
// direction) with q/p = c sin(theta) conserved, n = ceil(|l| / step) equal
// steps (backwards for l < 0: the polish step of the radius solve can end a
// hair behind the start).  Output in the state parametrisation (x, y, z, c,
// phi, theta).  The position is accumulated as the displacement from the
// start, added to the start once at the end: summed onto |z| ~ 200 cm in
// FP32 the steps' rounding makes z(l) jump by ~2e-4 cm between neighbouring
// l, more than the solves' tolerance.
template <typename T>
KF_HD inline void rk_cart(const T p[6], T l, T B0, T Z0, T step, T y_out[3], T t_out[3])
{
    T st, ct, sp, cp;
    Tr<T>::sincos_(p[5], &st, &ct);
    Tr<T>::sincos_(p[4], &sp, &cp);
    const T kq = T(kKappa) * p[3] * st;
    const T x0 = p[0], x1 = p[1], x2 = p[2];
    T y0 = T(0), y1 = T(0), y2 = T(0), t0 = st * cp, t1 = st * sp, t2 = ct;
    const int n = (int)ceil(double(Tr<T>::abs_(l) / step));
    const T h = n > 0 ? l / T(n) : T(0);
    // compensated (Kahan) sums of the steps: in FP32 the rounding of a few
    // hundred like increments onto the position and the direction is biased
    // enough to move z(l) by 1e-3 cm, ten times the solves' tolerance
    T e[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    auto csum = [](T& sum, T& err, T inc) {
        const T v = inc - err;
        const T t = sum + v;
        err = (t - sum) - v;
        sum = t;
    };
    // derivative at the displacement (e0, e1, e2) from the start, direction u
    auto der = [&](T e0, T e1, T e2, T u0, T u1, T u2, T d[6]) {
        T bx, by, bz;
        field_at(B0, Z0, x0 + e0, x1 + e1, x2 + e2, &bx, &by, &bz);
        d[0] = u0;
        d[1] = u1;
        d[2] = u2;
        d[3] = kq * (u1 * bz - u2 * by);
        d[4] = kq * (u2 * bx - u0 * bz);
        d[5] = kq * (u0 * by - u1 * bx);
    };
    for (int i = 0; i < n; ++i) {
        T a[6], b[6], c[6], d[6];
        der(y0, y1, y2, t0, t1, t2, a);
        const T hh = T(0.5) * h;
        der(y0 + hh * a[0], y1 + hh * a[1], y2 + hh * a[2], t0 + hh * a[3], t1 + hh * a[4],
            t2 + hh * a[5], b);
        der(y0 + hh * b[0], y1 + hh * b[1], y2 + hh * b[2], t0 + hh * b[3], t1 + hh * b[4],
            t2 + hh * b[5], c);
        der(y0 + h * c[0], y1 + h * c[1], y2 + h * c[2], t0 + h * c[3], t1 + h * c[4],
            t2 + h * c[5], d);
        const T w = h / T(6);
        csum(y0, e[0], w * (a[0] + T(2) * b[0] + T(2) * c[0] + d[0]));
        csum(y1, e[1], w * (a[1] + T(2) * b[1] + T(2) * c[1] + d[1]));
        csum(y2, e[2], w * (a[2] + T(2) * b[2] + T(2) * c[2] + d[2]));
        csum(t0, e[3], w * (a[3] + T(2) * b[3] + T(2) * c[3] + d[3]));
        csum(t1, e[4], w * (a[4] + T(2) * b[4] + T(2) * c[4] + d[4]));
        csum(t2, e[5], w * (a[5] + T(2) * b[5] + T(2) * c[5] + d[5]));
    }
    y_out[0] = x0 + y0;
    y_out[1] = x1 + y1;
    y_out[2] = x2 + y2;
    t_out[0] = t0;
    t_out[1] = t1;
    t_out[2] = t2;
}

// The state parametrisation (x, y, z, c, phi, theta) of a position y and unit
// direction t reached from p (q/p = c sin(theta) conserved).
template <typename T>
KF_HD inline void rk_params(const T p[6], const T y[3], const T t[3], T out[6])
{
    const T tt = Tr<T>::sqrt_(t[0] * t[0] + t[1] * t[1]);
    out[0] = y[0];
    out[1] = y[1];
    out[2] = y[2];
    out[5] = Tr<T>::atan2_(tt, t[2]);
    out[4] = Tr<T>::atan2_(t[1], t[0]);
    out[3] = p[3] * Tr<T>::sin_(p[5]) / Tr<T>::sin_(out[5]);
}

template <typename T>
KF_HD inline void rk_path(const T p[6], T l, T B0, T Z0, T step, T out[6])
{
    T y[3], t[3];
    rk_cart(p, l, B0, Z0, step, y, t);
    rk_params(p, y, t, out);
}

// A Cartesian state (position y, unit direction t) of the track from p moved
// by a short path d: the solves' polish step after their last evaluation,
// first order in d (|d| below the solve's tolerance, so the neglected terms
// are below 1e-8 of it).
template <typename T>
KF_HD inline void rk_nudge(const T p[6], T B0, T Z0, T d, T y[3], T t[3])
{
    T bx, by, bz;
    field_at(B0, Z0, y[0], y[1], y[2], &bx, &by, &bz);
    const T kq = T(kKappa) * p[3] * Tr<T>::sin_(p[5]);
    const T d0 = kq * (t[1] * bz - t[2] * by), d1 = kq * (t[2] * bx - t[0] * bz),
            d2 = kq * (t[0] * by - t[1] * bx);
    y[0] += d * t[0];
    y[1] += d * t[1];
    y[2] += d * t[2];
    t[0] += d * d0;
    t[1] += d * d1;
    t[2] += d * d2;
}

// Propagation along the 3D path l in the parametrised field whose end state q
// (rk_path) is known: the covariance by the helix Jacobian (with ds/dp for the
// barrel or the disk at zd) over the transverse length l sin(theta0), in the
// path's mean effective axial field, then the state becomes q.  The effective
// field is what turns the transverse direction: Bz - cot(theta) B_T . t_T (the
// transverse field bends a track that also moves along z), averaged by
// Simpson's rule over the start, the chord's midpoint (with the mean
// direction) and the end.
template <typename T>
KF_HD inline T effective_bz(T B0, T Z0, T x, T y, T z, T phi, T theta)
{
    T bx, by, bz, sp, cp, st, ct;
    field_at(B0, Z0, x, y, z, &bx, &by, &bz);
    Tr<T>::sincos_(phi, &sp, &cp);
    Tr<T>::sincos_(theta, &st, &ct);
    return bz - ct / st * (bx * cp + by * sp);
}

template <typename T, typename C, typename S>
KF_HD inline void field_transport(S p[6], C P[21], const T q[6], T l, const kf_params& prm, int kind,
                                  T zd)
{
    T pc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pc[k] = T(p[k]);
    const T B0 = T(prm.bz), Z0 = T(prm.field_z0);
    const T half = T(0.5);
    const T b_a = effective_bz(B0, Z0, pc[0], pc[1], pc[2], pc[4], pc[5]);
    const T b_m = effective_bz(B0, Z0, half * (pc[0] + q[0]), half * (pc[1] + q[1]),
                               half * (pc[2] + q[2]), pc[4] + half * wrap_phi(q[4] - pc[4]),
                               half * (pc[5] + q[5]));
    const T b_b = effective_bz(B0, Z0, q[0], q[1], q[2], q[4], q[5]);
    const T kb = T(kKappa) * ((b_a + T(4) * b_m + b_b) / T(6));
    transport(pc, P, l * Tr<T>::sin_(pc[5]), kb, kind, zd);
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = S(q[k]);
    p[4] = wrap_phi(p[4]);
}

// Status bits that freeze a track (everything except the informational
// fallback bit of the learned guess).
constexpr uint32_t kFreezeMask = ~(uint32_t)KF_ST_FALLBACK;

// Surface orders for the dynamic navigation, built once per workgroup:
// barrel indices by radius (ascending, ties by index) and disk indices in
// layer order.
struct NavOrder {
    int8_t barrel[64];
    int8_t disk[64];
    int32_t nb, nd;
};

KF_HD inline void build_nav_order(const kf_layer* L, int nl, NavOrder* nv)
{
    nv->nb = nv->nd = 0;
    for (int l = 0; l < nl; ++l) {
        if (L[l].kind == 0) {
            // stable insertion by radius
            int k = nv->nb++;
            while (k > 0 && L[nv->barrel[k - 1]].r_or_z > L[l].r_or_z) {
                nv->barrel[k] = nv->barrel[k - 1];
                --k;
            }
            nv->barrel[k] = (int8_t)l;
        } else {
            nv->disk[nv->nd++] = (int8_t)l;
        }
    }
}

// The next barrel outward from the radius-ordered list: the first above
// rho + kNextBarrelEps (the same layer as next_barrel below), or -1.
template <typename T>
KF_HD inline int next_barrel(const T p[6], const kf_layer* L, const NavOrder& nv)
{
    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
    for (int k = 0; k < nv.nb; ++k) {
        const int l = nv.barrel[k];
        if (T(L[l].r_or_z) > rho + T(kNextBarrelEps)) return l;
    }
    return -1;
}

// The next barrel outward: smallest radius above rho + kNextBarrelEps, or -1.
template <typename T>
KF_HD inline int next_barrel(const T p[6], const kf_layer* L, int nl)
{
    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
    int bl = -1;
    T rbl = T(0);
    for (int l = 0; l < nl; ++l) {
        if (L[l].kind != 0) continue;
        const T r = T(L[l].r_or_z);
        if (r > rho + T(kNextBarrelEps) && (bl < 0 || r < rbl)) {
            bl = l;
            rbl = r;
        }
    }
    return bl;
}

// Propagate-to-radius solve.  Plain: bracketed Newton from the straight-line
// start s0.  With a learned guess s_guess >= 0 that differs from s0 by more
// than kLearnedGate newton tolerances (the network predicts a curved path the
// straight line misses), the solve starts at s_guess with learned_it
// evaluations; if those do not converge it counts a fallback and runs the
// plain solve.  Smaller predicted corrections keep the straight-line start,
// exact for straight tracks.
constexpr double kLearnedGate = 100.0;

template <typename T>
KF_HD inline int solve_barrel(const T p[6], T h, T cph, T sph, T r_l, T s_hi, const kf_params& prm,
                              T s_guess, int learned_it, T* s, int* evals, int* fallbacks)
{
    const T s0 = line_guess(p[0], p[1], cph, sph, r_l);
    if (s_guess >= T(0) && learned_it > 0 &&
        Tr<T>::abs_(s_guess - s0) > T(kLearnedGate * prm.newton_tol)) {
        if (!newton_barrel(p[0], p[1], p[4], h, r_l, s_guess, T(0), s_hi, learned_it,
                           T(prm.newton_tol), s, evals))
            return 0;
        ++*fallbacks;
    }
    return newton_barrel(p[0], p[1], p[4], h, r_l, s0, T(0), s_hi, prm.max_newton,
                         T(prm.newton_tol), s, evals);
}

// Propagate-to-radius in the parametrised field: bracketed Newton on the 3D
// path length l, r(l) from the Cartesian end state of rk_cart.  The bracket
// and reachability come from the helix in the start point's field (kb0 =
// kappa Bz(start)), the bracket cut at kMaxFieldPath (a barrel whose
// straight-line path exceeds it is unreachable); the start is the straight
// line, or l_guess >= 0 with learned_it evaluations before the fallback to the
// straight line (counted in *fallbacks).  On convergence the polish step is
// taken from the last evaluation's state (rk_nudge), and q_out gets the end
// state at the polished path *l_out.
template <typename T>
KF_HD inline int solve_barrel_field(const T p[6], T r_l, const kf_params& prm, T kb0, T l_guess,
                                    int learned_it, T* l_out, T q_out[6], int* evals, int* fallbacks)
{
    T sph, cph, sth, cth;
    Tr<T>::sincos_(p[4], &sph, &cph);
    Tr<T>::sincos_(p[5], &sth, &cth);
    const T h = -kb0 * p[3];
    T s_hi;
    if (!barrel_bracket(p[0], p[1], cph, sph, h, r_l, &s_hi)) return KF_ST_UNREACHABLE;
    const T l_line = line_guess(p[0], p[1], cph, sph, r_l) / sth;
    // the straight line is the shortest way to the radius
    if (l_line > T(kMaxFieldPath)) return KF_ST_UNREACHABLE;
    const T l_top = Tr<T>::min_(s_hi / sth, T(kMaxFieldPath));
    const T B0 = T(prm.bz), Z0 = T(prm.field_z0), step = T(prm.field_step);
    const T tol = T(prm.newton_tol);
    // bracketed Newton from l within [0, l_top] with at most max_it evaluations
    auto newton = [&](T l, int max_it) -> int {
        T lo = T(0), hi = l_top;
        if (l < lo) l = lo;
        if (l > hi) l = hi;
        for (int it = 1; it <= max_it; ++it) {
            T y[3], t[3];
            rk_cart(p, l, B0, Z0, step, y, t);
            const T r = Tr<T>::sqrt_(y[0] * y[0] + y[1] * y[1]);
            const T res = r - r_l;
            const T drdl = (y[0] * t[0] + y[1] * t[1]) / r;
            ++*evals;
            if (res < T(0)) {
                if (l > lo) lo = l;
            } else {
                if (l < hi) hi = l;
            }
            if (Tr<T>::abs_(res) < tol) {
                // the polish step, taken from this evaluation's state
                const T d = drdl > T(0) ? -res / drdl : T(0);
                rk_nudge(p, B0, Z0, d, y, t);
                rk_params(p, y, t, q_out);
                *l_out = l + d;
                return 0;
            }
            T ln = l - res / drdl;
            if (!(drdl > T(0)) || !(ln > lo && ln < hi)) ln = T(0.5) * (lo + hi);
            l = ln;
        }
        *l_out = l;
        return (int)KF_ST_NOCONV;
    };
    if (l_guess >= T(0) && learned_it > 0 &&
        Tr<T>::abs_(l_guess - l_line) * sth > T(kLearnedGate * prm.newton_tol)) {
        if (!newton(l_guess, learned_it)) return 0;
        ++*fallbacks;
    }
    return newton(l_line, prm.max_newton);
}

// Propagate-to-z in the parametrised field: bracketed Newton on the 3D path
// length l, z(l) from rk_cart with dz/dl = cos theta(l), the end state as in
// the radius solve.  Start: the straight
// line l0 = (z_d - z) / cos theta, exact in a uniform field; the plane must
// lie ahead (0 <= l0 <= kMaxFieldPath).  Bracket [0, min(2 l0,
// kMaxFieldPath)]: the radial field bends theta only slightly, and a track
// short of the plane after twice the straight path does not reach it
// (NOCONV).  Same stopping rule as the radius solve.
template <typename T>
KF_HD inline int solve_disk_field(const T p[6], T z_d, const kf_params& prm, T* l_out, T q_out[6],
                                  int* evals)
{
    T sth, cth;
    Tr<T>::sincos_(p[5], &sth, &cth);
    if (cth == T(0)) return KF_ST_UNREACHABLE;
    const T l0 = (z_d - p[2]) / cth;
    if (!(l0 >= T(0)) || l0 > T(kMaxFieldPath)) return KF_ST_UNREACHABLE;
    const T sgn = cth > T(0) ? T(1) : T(-1);
    const T B0 = T(prm.bz), Z0 = T(prm.field_z0), step = T(prm.field_step);
    const T tol = T(prm.newton_tol);
    T lo = T(0), hi = Tr<T>::min_(T(2) * l0, T(kMaxFieldPath)), l = l0;
    for (int it = 1; it <= prm.max_newton; ++it) {
        T y[3], t[3];
        rk_cart(p, l, B0, Z0, step, y, t);
        const T res = sgn * (y[2] - z_d);      // > 0: past the plane
        const T dzdl = sgn * t[2];
        ++*evals;
        if (res < T(0)) {
            if (l > lo) lo = l;
        } else {
            if (l < hi) hi = l;
        }
        if (Tr<T>::abs_(res) < tol) {
            // the polish step, taken from this evaluation's state
            const T d = dzdl > T(0) ? -res / dzdl : T(0);
            rk_nudge(p, B0, Z0, d, y, t);
            rk_params(p, y, t, q_out);
            *l_out = l + d;
            return 0;
        }
        T ln = l - res / dzdl;
        if (!(dzdl > T(0)) || !(ln > lo && ln < hi)) ln = T(0.5) * (lo + hi);
        l = ln;
    }
    *l_out = l;
    return (int)KF_ST_NOCONV;
}

// Next surface in the parametrised field: whichever comes first along the 3D
// path, the next barrel outward (next_barrel), reached by the Runge-Kutta
// radius solve and crossed inside |z| <= hi, or a disk ahead (|dz| >
// kDiskAheadEps in the direction of travel), reached by the Runge-Kutta z
// solve and crossed inside its radial extent; both within half a turn of the
// start point's curvature in the transverse plane.  Disks are taken in layer
// order; one whose straight-line path exceeds the best path found, or whose
// straight-line transverse path exceeds half a turn, by more than 1% + 1 cm
// is not solved (the solved path differs from the straight one by far less).  Returns the layer with the 3D path and the end state, or
// -1 (no surface left; a failed solve sets NOCONV).  l_guess >= 0: the
// learned start of the barrel solve (3D path), with learned_it evaluations
// before the fallback (counted in *fallbacks).
template <typename T>
KF_HD inline int navigate_field(const T p[6], const kf_layer* L, int nl, const kf_params& prm,
                                T* l_out, T q[6], uint32_t* st, int* newton_evals, int* disk_evals,
                                T l_guess = T(-1), int learned_it = 0, int* fallbacks = nullptr)
{
    const T B0 = T(prm.bz), Z0 = T(prm.field_z0), step = T(prm.field_step);
    T bx, by, bz0;
    field_at(B0, Z0, p[0], p[1], p[2], &bx, &by, &bz0);
    const T kb0 = T(kKappa) * bz0;
    const T hh = Tr<T>::abs_(kb0 * p[3]);
    const T s_max = hh > T(0) ? T(kPi) / hh : T(1e30);
    T sth, cth;
    Tr<T>::sincos_(p[5], &sth, &cth);
    T best = T(1e30);
    int best_l = -1;
    const int bl = next_barrel(p, L, nl);
    if (bl >= 0) {
        T l;
        int fb = 0;
        const int r = solve_barrel_field(p, T(L[bl].r_or_z), prm, kb0, l_guess, learned_it, &l, q,
                                         newton_evals, &fb);
        if (fallbacks) *fallbacks += fb;
        if (r == (int)KF_ST_NOCONV) {
            *st |= KF_ST_NOCONV;
            return -1;
        }
        if (r == 0) {
            if (Tr<T>::abs_(q[2]) <= T(L[bl].hi) && l * sth <= s_max) {
                best = l;
                best_l = bl;
            }
        }
    }
    for (int d = 0; d < nl; ++d) {
        if (L[d].kind != 1) continue;
        const T dz = T(L[d].r_or_z) - p[2];
        if (!(dz * cth > T(0)) || Tr<T>::abs_(dz) <= T(kDiskAheadEps)) continue;
        const T l_line = dz / cth;
        if (l_line > T(1.01) * best + T(1) || l_line * sth > T(1.01) * s_max + T(1)) continue;
        T ld;
        ++*disk_evals;
        T qd[6];
        const int r = solve_disk_field(p, T(L[d].r_or_z), prm, &ld, qd, newton_evals);
        if (r == (int)KF_ST_NOCONV) {
            *st |= KF_ST_NOCONV;
            return -1;
        }
        if (r) continue;
        const T rr = Tr<T>::sqrt_(qd[0] * qd[0] + qd[1] * qd[1]);
        if (ld * sth > s_max || rr < T(L[d].lo) || rr > T(L[d].hi)) continue;
        if (ld < best) {
            best = ld;
            best_l = d;
#pragma unroll
            for (int k = 0; k < 6; ++k) q[k] = qd[k];
        }
    }
    if (best_l >= 0) *l_out = best;
    return best_l;
}

// Steering in the parametrised field: as steer_next, each plan entry reached
// by its Runge-Kutta solve along the 3D path (as in navigate_field), half a
// turn taken at the start point's curvature; a disk whose straight-line
// transverse path exceeds half a turn by more than 1% + 1 cm is not solved.
// Returns the layer with the 3D path and the end state, or -1 when the plan
// is exhausted (a failed solve sets NOCONV and returns -1).
template <typename T>
KF_HD inline int steer_next_field(const T p[6], const kf_layer* L, const uint8_t* plan, int n_plan,
                                  int* pos, const kf_params& prm, T* l_out, T q[6], uint32_t* st,
                                  int* newton_evals, int* disk_evals)
{
    const T B0 = T(prm.bz), Z0 = T(prm.field_z0), step = T(prm.field_step);
    T bx, by, bz0;
    field_at(B0, Z0, p[0], p[1], p[2], &bx, &by, &bz0);
    const T kb0 = T(kKappa) * bz0;
    const T hh = Tr<T>::abs_(kb0 * p[3]);
    const T s_max = hh > T(0) ? T(kPi) / hh : T(1e30);
    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
    T sth, cth;
    Tr<T>::sincos_(p[5], &sth, &cth);
    for (int qi = *pos; qi < n_plan; ++qi) {
        const int l = plan[qi];
        const kf_layer& Ly = L[l];
        T ll;
        if (Ly.kind == 0) {
            const T r_l = T(Ly.r_or_z);
            if (!(r_l > rho + T(kNextBarrelEps))) continue;
            int fb = 0;
            const int r = solve_barrel_field(p, r_l, prm, kb0, T(-1), 0, &ll, q, newton_evals, &fb);
            if (r == (int)KF_ST_NOCONV) {
                *st |= KF_ST_NOCONV;
                *pos = qi + 1;
                return -1;
            }
            if (r) continue;
            if (Tr<T>::abs_(q[2]) > T(Ly.hi) || ll * sth > s_max) continue;
        } else {
            const T dz = T(Ly.r_or_z) - p[2];
            if (!(dz * cth > T(0)) || Tr<T>::abs_(dz) <= T(kDiskAheadEps)) continue;
            if (dz / cth * sth > T(1.01) * s_max + T(1)) continue;
            ++*disk_evals;
            const int r = solve_disk_field(p, T(Ly.r_or_z), prm, &ll, q, newton_evals);
            if (r == (int)KF_ST_NOCONV) {
                *st |= KF_ST_NOCONV;
                *pos = qi + 1;
                return -1;
            }
            if (r) continue;
            const T rr = Tr<T>::sqrt_(q[0] * q[0] + q[1] * q[1]);
            if (ll * sth > s_max || rr < T(Ly.lo) || rr > T(Ly.hi)) continue;
        }
        *l_out = ll;
        *pos = qi + 1;
        return l;
    }
    *pos = n_plan;
    return -1;
}

// Steering: from plan entry *pos on, the first layer the candidate reaches
// (a barrel outside rho + kNextBarrelEps crossed outward within half a turn
// inside |z| <= hi, or a disk ahead crossed within half a turn inside its
// radial extent); entries not reached are passed over.  Returns the layer,
// its path length and *pos past it, or -1 when the plan is exhausted (a
// failed barrel solve sets NOCONV and returns -1).
template <typename T>
KF_HD inline int steer_next(const T p[6], const kf_layer* L, const uint8_t* plan, int n_plan,
                            int* pos, const kf_params& prm, T kb, T* s_out, uint32_t* st,
                            int* newton_evals, int* disk_evals)
{
    const T hh = Tr<T>::abs_(kb * p[3]);
    const T s_max = hh > T(0) ? T(kPi) / hh : T(1e30);
    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
    T sth, cth, sph, cph;
    Tr<T>::sincos_(p[5], &sth, &cth);
    Tr<T>::sincos_(p[4], &sph, &cph);
    const T cot = cth / sth;
    const T h = -kb * p[3];
    for (int q = *pos; q < n_plan; ++q) {
        const int l = plan[q];
        const kf_layer& Ly = L[l];
        T s;
        if (Ly.kind == 0) {
            const T r_l = T(Ly.r_or_z);
            if (!(r_l > rho + T(kNextBarrelEps))) continue;
            T s_hi;
            if (!barrel_bracket(p[0], p[1], cph, sph, h, r_l, &s_hi)) continue;
            int fb = 0;
            if (solve_barrel(p, h, cph, sph, r_l, s_hi, prm, T(-1), 0, &s, newton_evals, &fb)) {
                *st |= KF_ST_NOCONV;
                *pos = q + 1;
                return -1;
            }
            const T zc = p[2] + s * cot;
            if (Tr<T>::abs_(zc) > T(Ly.hi) || s > s_max) continue;
        } else {
            const T dz = T(Ly.r_or_z) - p[2];
            if (!(dz * cot > T(0)) || Tr<T>::abs_(dz) <= T(kDiskAheadEps)) continue;
            s = dz / cot;
            if (s > s_max) continue;
            ++*disk_evals;
            const HelixPoint<T> hp = helix_at(p[0], p[1], p[4], h, s);
            const T r = Tr<T>::sqrt_(hp.X * hp.X + hp.Y * hp.Y);
            if (r < T(Ly.lo) || r > T(Ly.hi)) continue;
        }
        *s_out = s;
        *pos = q + 1;
        return l;
    }
    *pos = n_plan;
    return -1;
}

// Next surface: whichever comes first along the helix, the next barrel
// outward (smallest radius above the current one, reachable, crossing inside
// its z extent) or the first disk ahead whose crossing is inside its radial
// extent.  Returns the layer (or -1) and the path length.  s_guess >= 0: the
// learned start of the barrel solve (learned_it evaluations, then fallback).
template <typename T>
KF_HD inline int navigate(const T p[6], const kf_layer* L, const NavOrder& nv, const kf_params& prm, T kb,
                          T* s_out, uint32_t* st, int* newton_evals, int* disk_evals,
                          T s_guess = T(-1), int learned_it = 0, int* fallbacks = nullptr)
{
    // only surfaces reached within half a turn in the transverse plane
    const T hh = Tr<T>::abs_(kb * p[3]);
    const T s_max = hh > T(0) ? T(kPi) / hh : T(1e30);
    const int bl = next_barrel(p, L, nv);
    const T rbl = bl >= 0 ? T(L[bl].r_or_z) : T(0);
    T best_s = T(1e30);
    int best_l = -1;
    T sth, cth;
    Tr<T>::sincos_(p[5], &sth, &cth);
    if (bl >= 0) {
        const T h = -kb * p[3];
        T sph, cph;
        Tr<T>::sincos_(p[4], &sph, &cph);
        T s_hi;
        if (barrel_bracket(p[0], p[1], cph, sph, h, rbl, &s_hi)) {
            T s;
            int fb = 0;
            const int r = solve_barrel(p, h, cph, sph, rbl, s_hi, prm, s_guess, learned_it, &s,
                                       newton_evals, &fb);
            if (fallbacks) *fallbacks += fb;
            if (r) {
                *st |= KF_ST_NOCONV;
                return -1;
            }
            const T zc = p[2] + s * cth / sth;
            if (Tr<T>::abs_(zc) <= T(L[bl].hi) && s <= s_max) {
                best_s = s;
                best_l = bl;
            }
        }
    }
    const T cot = cth / sth;
    for (int k = 0; k < nv.nd; ++k) {
        const int l = nv.disk[k];
        const T dz = T(L[l].r_or_z) - p[2];
        if (!(dz * cot > T(0)) || Tr<T>::abs_(dz) <= T(kDiskAheadEps)) continue;
        const T s = dz / cot;
        if (!(s < best_s) || s > s_max) continue;
        ++*disk_evals;
        const HelixPoint<T> q = helix_at(p[0], p[1], p[4], -kb * p[3], s);
        const T r = Tr<T>::sqrt_(q.X * q.X + q.Y * q.Y);
        if (r < T(L[l].lo) || r > T(L[l].hi)) continue;
        best_s = s;
        best_l = l;
    }
    *s_out = best_s;
    return best_l;
}


// Hit-search window of a predicted state on a layer: the bounding box of the
// chi2 < cut ellipse (half-widths from the position covariance plus the
// layer's largest hit sigma) with a 1e-3 relative and 1e-4 absolute margin.
// Azimuth: |d| <= dphi, tested as cos d > 0 and |sin d| <= sin dphi (dphi
// below pi/2; wider windows take the whole circle).  Second coordinate: z
// (barrel) or r (disk) range for the bin enumeration, |residual| <= wv.
template <typename T>
struct Window {
    bool ok, all_phi;
    T dphi, cos_dphi, sin_dphi, wv, vlo, vhi;
};

template <typename T, typename C>
KF_HD inline Window<T> make_window(const T p[6], const C P[21], const kf_layer& L, T cut)
{
    Window<T> W;
    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
    const T pxx = T(P[pk(0, 0)]), pyy = T(P[pk(1, 1)]), pzz = T(P[pk(2, 2)]);
    const T wu = Tr<T>::sqrt_(cut * (pxx + pyy + T(L.win_su) * T(L.win_su)));
    const T tt = T(1.001) * wu / rho;
    T dphi = tt >= T(1) ? T(kPi) : Tr<T>::asin_(tt) + T(1e-4);
    if (dphi > T(0.5 * kPi)) dphi = T(kPi);
    W.dphi = dphi;
    W.all_phi = dphi >= T(kPi);
    W.cos_dphi = W.all_phi ? T(-1) : Tr<T>::cos_(dphi);
    W.sin_dphi = W.all_phi ? T(2) : Tr<T>::sin_(dphi);
    if (L.kind == 0) {
        W.wv = T(1.001) * Tr<T>::sqrt_(cut * (pzz + T(L.win_sv) * T(L.win_sv))) + T(1e-4);
        W.vlo = p[2] - W.wv;
        W.vhi = p[2] + W.wv;
    } else {
        W.wv = T(1.001) * Tr<T>::sqrt_(cut * (pxx + pyy + T(L.win_sv) * T(L.win_sv))) + T(1e-4);
        W.vlo = rho * W.cos_dphi - W.wv;
        W.vhi = rho + W.wv;
    }
    // a non-finite covariance gives no usable window: no hits tested
    W.ok = dphi >= T(0) && W.wv >= T(0) && W.wv < T(1e30) && rho > T(0);
    return W;
}

}  // namespace kfmi
