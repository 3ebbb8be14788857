// Host program: counts the floating-point operations of the device arithmetic
// (kf_math.hpp) by instantiating it with a counting number type.  Adds,
// subtracts, multiplies, divides and square roots count one operation each
// (a fused multiply-add is two); sin, cos, asin, atan2, log and fmod are
// counted separately as special-function calls.  Comparisons and
// conversions are free.  Prints JSON: operations per unit of work of the
// finding and fitting kernels, used to turn event counts into flops.
#include <cmath>
#include <cstdio>

#include "kf_math.hpp"

namespace {
long g_ops = 0, g_sfu = 0;

struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator float() const { return float(v); }
    explicit operator int() const { return int(v); }
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator==(Cnt a, Cnt b) { return a.v == b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
inline bool isfinite(Cnt a) { return std::isfinite(a.v); }
}  // namespace

namespace kfmi {
template <> struct Tr<Cnt> {
    static void sincos_(Cnt x, Cnt* s, Cnt* c)
    {
        g_sfu += 2;
        *s = Cnt(std::sin(x.v));
        *c = Cnt(std::cos(x.v));
    }
    static Cnt sqrt_(Cnt x) { ++g_ops; return Cnt(std::sqrt(x.v)); }
    static Cnt abs_(Cnt x) { return Cnt(std::fabs(x.v)); }
    static Cnt atan2_(Cnt y, Cnt x) { ++g_sfu; return Cnt(std::atan2(y.v, x.v)); }
    static Cnt log_(Cnt x) { ++g_sfu; return Cnt(std::log(x.v)); }
    static Cnt fmod_(Cnt x, Cnt y) { ++g_sfu; return Cnt(std::fmod(x.v, y.v)); }
    static Cnt asin_(Cnt x) { ++g_sfu; return Cnt(std::asin(x.v)); }
    static Cnt cos_(Cnt x) { ++g_sfu; return Cnt(std::cos(x.v)); }
    static Cnt sin_(Cnt x) { ++g_sfu; return Cnt(std::sin(x.v)); }
    static Cnt floor_(Cnt x) { return Cnt(std::floor(x.v)); }
    static Cnt min_(Cnt a, Cnt b) { return Cnt(std::fmin(a.v, b.v)); }
};
}  // namespace kfmi

using namespace kfmi;
using T = Cnt;

struct Tally {
    long ops, sfu;
};

template <typename F>
Tally count(F f)
{
    long o0 = g_ops, s0 = g_sfu;
    f();
    return {g_ops - o0, g_sfu - s0};
}

static void state(T p[6], T P[21], double r, double phi, double c, double th)
{
    p[0] = r * std::cos(phi);
    p[1] = r * std::sin(phi);
    p[2] = 3.0;
    p[3] = c;
    p[4] = phi + 0.05;
    p[5] = th;
    for (int k = 0; k < 21; ++k) P[k] = 0.0;
    const double d[6] = {1e-4, 1e-4, 1e-3, 1e-4, 1e-6, 1e-6};
    for (int i = 0; i < 6; ++i) P[pk(i, i)] = d[i];
    P[pk(0, 4)] = 1e-6;
}

int main()
{
    kf_params prm;
    prm.bz = 3.8;
    prm.chi2_cut = 30.0;
    prm.newton_tol = 1e-4;
    prm.mass = 0.13957;
    prm.max_cands = 6;
    prm.max_newton = 10;
    prm.max_miss = 2;
    prm.mlp_max_iter = 3;
    prm.field_z0 = 0.0;
    prm.field_step = 2.0;
    const T kb = T(kKappa * prm.bz);
    kf_layer barrel{0, 128, 32, 0, 50.0, -60.0, 60.0, 0.02, 0.01, 0.05};
    kf_layer disk{1, 128, 32, 0, 110.0, 20.0, 100.0, 0.02, 0.01, 0.05};

    // one evaluation of r(s) inside the bracketed Newton solve: difference of
    // solves allowed 2 and 1 evaluations on a start that does not converge early
    T p[6], P[21];
    state(p, P, 30.0, 0.3, 0.8, 1.2);
    const T h = -kb * p[3];
    T sph, cph, s_hi, s;
    Tr<T>::sincos_(p[4], &sph, &cph);
    int ev = 0;
    Tally t1 = count([&] { newton_barrel(p[0], p[1], p[4], h, T(50.0), T(0.0), T(0.0), T(200.0), 1,
                                         T(1e-12), &s, &ev); });
    Tally t2 = count([&] { newton_barrel(p[0], p[1], p[4], h, T(50.0), T(0.0), T(0.0), T(200.0), 2,
                                         T(1e-12), &s, &ev); });
    Tally newton_eval{t2.ops - t1.ops, t2.sfu - t1.sfu};
    // the fixed part of a barrel solve: bracket + straight-line start
    Tally barrel_setup = count([&] {
        T sp, cp;
        Tr<T>::sincos_(p[4], &sp, &cp);
        barrel_bracket(p[0], p[1], cp, sp, h, T(50.0), &s_hi);
        line_guess(p[0], p[1], cp, sp, T(50.0));
    });
    // one disk candidate tested by the navigation: helix point + radius
    Tally disk_eval = count([&] {
        HelixPoint<T> q = helix_at(p[0], p[1], p[4], h, T(40.0));
        Tr<T>::sqrt_(q.X * q.X + q.Y * q.Y);
    });
    // transport + scattering noise
    Tally tr_barrel = count([&] {
        T q[6], Q[21];
        for (int k = 0; k < 6; ++k) q[k] = p[k];
        for (int k = 0; k < 21; ++k) Q[k] = P[k];
        transport(q, Q, T(25.0), kb, 0, T(50.0));
        add_scatter(q, Q, 0, T(0.02), T(prm.mass));
    });
    Tally tr_disk = count([&] {
        T q[6], Q[21];
        for (int k = 0; k < 6; ++k) q[k] = p[k];
        for (int k = 0; k < 21; ++k) Q[k] = P[k];
        transport(q, Q, T(25.0), kb, 1, T(110.0));
        add_scatter(q, Q, 1, T(0.02), T(prm.mass));
    });
    // hit-search window and the per-hit tests (azimuth, second coordinate, chi2)
    Tally window = count([&] { make_window<T, T>(p, P, barrel, T(30.0)); });
    HitFrame<T> f;
    f.hx = 28.7;
    f.hy = 8.9;
    f.hz = 3.01;
    f.c = 0.955;
    f.s = 0.296;
    f.vu = 1e-4;
    f.vv = 2.5e-3;
    Tally hit_test = count([&] {
        T cd = f.c * p[0] + f.s * p[1];
        T sd = f.s * p[0] - f.c * p[1];
        T rv = f.hz - p[2];
        (void)cd;
        (void)sd;
        (void)rv;
        hit_chi2<T, T, T>(p, P, f, 0);
    });
    Tally update = count([&] {
        T q[6], Q[21];
        for (int k = 0; k < 6; ++k) q[k] = p[k];
        for (int k = 0; k < 21; ++k) Q[k] = P[k];
        T c2;
        kf_update<T, T, T>(q, Q, f, 0, &c2);
    });
    // navigation bookkeeping besides solves and disk tests: radius, cot theta,
    // the sincos of theta, the half-turn limit, the crossing z
    Tally nav_fixed = count([&] {
        Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
        Tr<T>::abs_(kb * p[3]);
        T(kPi) / h;
        T st, ct;
        Tr<T>::sincos_(p[5], &st, &ct);
        p[2] + T(25.0) * ct / st;
        ct / st;
    });
    // parametrised field: one fourth-order Runge-Kutta step, the fixed part
    // of a transport (state in and out), and one evaluation of the radius
    // solve besides its transport (a step longer than any path makes every
    // transport a single step)
    Tally rk_fixed = count([&] {
        T y[3], t[3];
        rk_cart(p, T(0.0), T(3.8), T(300.0), T(2.0), y, t);
    });
    Tally rk_one = count([&] {
        T y[3], t[3];
        rk_cart(p, T(1.5), T(3.8), T(300.0), T(2.0), y, t);
    });
    // a converged solve's end: the polish step and the state parametrisation
    Tally field_final = count([&] {
        T y[3] = {p[0], p[1], p[2]}, t[3] = {T(0.6), T(0.0), T(0.8)}, q[6];
        rk_nudge(p, T(3.8), T(300.0), T(1e-5), y, t);
        rk_params(p, y, t, q);
    });
    // the field transport's Jacobian field and the transport itself
    Tally field_transport_t = count([&] {
        T q[6] = {p[0] + T(1), p[1] + T(1), p[2] + T(1), p[3], p[4], p[5]};
        T x[6] = {p[0], p[1], p[2], p[3], p[4], p[5]};
        T Q[21];
        for (int k = 0; k < 21; ++k) Q[k] = P[k];
        kf_params fq = prm;
        fq.field_z0 = 300.0;
        field_transport(x, Q, q, T(1.5), fq, 0, T(50.0));
    });
    Tally rk_step{rk_one.ops - rk_fixed.ops, rk_one.sfu - rk_fixed.sfu};
    kf_params fp = prm;
    fp.field_z0 = 300.0;
    fp.field_step = 1e6;
    int fe = 0, ffb = 0;
    T lo;
    const T kb0 = T(kKappa * 3.8);
    fp.max_newton = 1;
    T qo[6];
    Tally f1 = count([&] { solve_barrel_field(p, T(50.0), fp, kb0, T(-1.0), 0, &lo, qo, &fe, &ffb); });
    fp.max_newton = 2;
    fp.newton_tol = 1e-300;
    Tally f2 = count([&] { solve_barrel_field(p, T(50.0), fp, kb0, T(-1.0), 0, &lo, qo, &fe, &ffb); });
    Tally field_eval{f2.ops - f1.ops - rk_one.ops, f2.sfu - f1.sfu - rk_one.sfu};
    Tally field_setup{f1.ops - (f2.ops - f1.ops), f1.sfu - (f2.sfu - f1.sfu)};
    Tally field_at_t = count([&] {
        T bx, by, bz;
        field_at(T(3.8), T(300.0), p[0], p[1], p[2], &bx, &by, &bz);
    });
    printf("{\n");
    auto pr = [](const char* k, Tally t, bool last = false) {
        printf("  \"%s\": {\"ops\": %ld, \"sfu\": %ld}%s\n", k, t.ops, t.sfu, last ? "" : ",");
    };
    pr("newton_eval", newton_eval);
    pr("barrel_setup", barrel_setup);
    pr("disk_eval", disk_eval);
    pr("transport_barrel", tr_barrel);
    pr("transport_disk", tr_disk);
    pr("window", window);
    pr("hit_test", hit_test);
    pr("update", update);
    pr("nav_fixed", nav_fixed);
    pr("rk_step", rk_step);
    pr("rk_fixed", rk_fixed);
    pr("field_eval", field_eval);
    pr("field_setup", field_setup);
    pr("field_final", field_final);
    pr("field_transport", field_transport_t);
    pr("field_at", field_at_t, true);
    printf("}\n");
    return 0;
}
