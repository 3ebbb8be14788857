/*
 * FP64 reference implementation of the KF track fit and combinatorial track
 * finding.  TEST INFRASTRUCTURE ONLY: the tests, smoke() and the CPU-baseline
 * leg of the benchmark use it; the product path never does.
 *
 * It is written for clarity, not speed: full 6x6 matrices, plain loops, one
 * candidate at a time.  The definitions it follows:
 *   - helix in a uniform field B along +z, state (x, y, z, c=q/pT, phi, theta),
 *     transverse arc length s, curvature h = dphi/ds = -kappa*B*c
 *     (kappa = 0.00299792458 GeV/(T cm));
 *   - propagation to the next layer (paper Sec. 3.1: layer-to-layer
 *     propagation following the geometry description): barrel radius by a
 *     bracketed Newton iteration, disk z in closed form;
 *   - transport Jacobian including the path-length derivative (implicit
 *     function theorem on the surface equation);
 *   - multiple scattering at every crossed layer (paper Sec. 3.1: material
 *     per layer) with the PDG Highland width.  Parity unpinned for the width's
 *     constants (13.6 MeV, 0.038) and the form of its logarithm: the only
 *     other statement of them is the event generator's, which the pins
 *     compare against; the structure around them (path-corrected thickness,
 *     beta p, the (c, phi, theta) block of the noise) is pinned by the
 *     toy Monte Carlo of the generator's kicks and by fit pulls;
 *   - Kalman update with a 2D hit measured in the hit's local frame,
 *     Joseph-form covariance (the traditional KF of the paper's Sec. 1);
 *   - layer-by-layer combinatorial finding (paper Sec. 2 and Sec. 4: hit
 *     search windows, chi2 selection, candidate scoring, bounded candidate
 *     count per seed);
 *   - optionally a parametrised (non-uniform) field (paper Sec. 3.1: constant
 *     or parametrised fields): an axially symmetric solenoid-like field,
 *     Bz = B0 / (1 + (z/Z0)^2) and Br = -(r/2) dBz/dz (divergence free),
 *     tracks integrated in 3D path length by fourth-order Runge-Kutta with
 *     equal steps of at most field_step; the propagate-to-radius solve is
 *     the same bracketed Newton iteration on the integrated radius, and the
 *     transport Jacobian is the helix one in the path's mean effective
 *     axial field (see transport_parts).  Disks are reached by the same
 *     Newton iteration on the integrated z.
 *     Both solves search at most MAX_FIELD_PATH (1000 cm) of 3D path.
 */
#include "kf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define KAPPA 0.00299792458
#define NEXT_BARREL_EPS 0.05      /* cm: a barrel is "ahead" if r > rho + eps */
#define DISK_AHEAD_EPS 0.05       /* cm: a disk is "ahead" if |dz| > eps in the travel direction */
#define MAX_FIELD_PATH 1000.0     /* cm: longest 3D path the field's Runge-Kutta solves search */
#define WIN_REL 1.001             /* window = chi2-ellipse bounding box, 1e-3 relative margin */
#define WIN_ABS 1e-4              /* plus an absolute margin (rad or cm) */
#define CLOSE_REL 1e-3            /* relative margin below which a decision counts as a tie */
#define NO_HIT 0x7fffffff
#define MAXL 64

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */

static int pidx(int i, int j)
{
    if (i > j) { int t = i; i = j; j = t; }
    return i * (11 - i) / 2 + j;
}

static void unpack(const double* Pk, double P[6][6])
{
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) P[i][j] = Pk[pidx(i, j)];
}

static void pack(double P[6][6], double* Pk)
{
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) Pk[pidx(i, j)] = 0.5 * (P[i][j] + P[j][i]);
}

static double wrap_pi(double a)
{
    /* to (-pi, pi] */
    while (a > PI) a -= 2.0 * PI;
    while (a <= -PI) a += 2.0 * PI;
    return a;
}

/* sin(u)/u */
static double sinc(double u)
{
    if (fabs(u) < 1e-4) return 1.0 - u * u / 6.0;
    return sin(u) / u;
}

/* d/du [sin(u)/u] = (u cos u - sin u) / u^2 */
static double dsinc(double u)
{
    if (fabs(u) < 0.05) {
        double u2 = u * u;
        return u * (-1.0 / 3.0 + u2 * (1.0 / 30.0 + u2 * (-1.0 / 840.0 + u2 / 45360.0)));
    }
    return (u * cos(u) - sin(u)) / (u * u);
}

/* C = A B for 6x6 */
static void mul66(double A[6][6], double B[6][6], double C[6][6])
{
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += A[i][k] * B[k][j];
            C[i][j] = acc;
        }
}

/* C = A B^T for 6x6 */
static void mul66t(double A[6][6], double B[6][6], double C[6][6])
{
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += A[i][k] * B[j][k];
            C[i][j] = acc;
        }
}

/* ------------------------------------------------------------------ */
/* helix                                                                */

void orc_helix(const double p[6], double s, double bz, double out[6])
{
    double h = -KAPPA * bz * p[3];
    double u = 0.5 * h * s;
    double a = p[4] + u;
    double sc = sinc(u);
    out[0] = p[0] + s * cos(a) * sc;
    out[1] = p[1] + s * sin(a) * sc;
    out[2] = p[2] + s * cos(p[5]) / sin(p[5]);
    out[3] = p[3];
    out[4] = wrap_pi(p[4] + h * s);
    out[5] = p[5];
}

/* ------------------------------------------------------------------ */
/* propagation to a barrel radius: bracketed Newton on r(s) = r_l        */
/*
 * Bracket [s_lo, s_hi] = [0, s_apex]: from a start inside the cylinder,
 * r(s) has exactly one outward crossing of r_l before the point of largest
 * radius (the apex) when the layer is reachable (|C| + R >= r_l, C the centre
 * of curvature, R the radius).  Newton steps that leave the bracket, or a
 * non-positive slope, are replaced by bisection.  Convergence: |r - r_l| <
 * tol, then one more Newton step.  Iterations count the evaluations of r(s).
 */
int orc_solve_barrel(const orc_cfg* cfg, const double p[6], double r_l, double s_init,
                     double* s_out, int* iters_out)
{
    double h = -KAPPA * cfg->bz * p[3];
    double cphi = cos(p[4]), sphi = sin(p[4]);
    double s_lo = 0.0, s_hi = 1e30;
    if (h != 0.0) {
        double cx = p[0] - sphi / h, cy = p[1] + cphi / h;
        double R = 1.0 / fabs(h);
        double dc = hypot(cx, cy);
        if (dc + R < r_l) {
            if (iters_out) *iters_out = 0;
            return ORC_ST_UNREACHABLE;
        }
        /* angle swept (in the direction of motion) from the current point to the apex */
        double v0x = p[0] - cx, v0y = p[1] - cy;
        double v1x = R * cx / dc, v1y = R * cy / dc;
        double alpha = atan2(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y);
        double sw = fmod((h > 0 ? alpha : -alpha), 2.0 * PI);
        if (sw < 0) sw += 2.0 * PI;
        s_hi = sw / fabs(h);
    }
    double s;
    if (s_init >= 0.0) {
        s = s_init;
    } else {
        /* straight-line intersection of the tangent with the cylinder */
        double pu = p[0] * cphi + p[1] * sphi;
        double disc = pu * pu - (p[0] * p[0] + p[1] * p[1]) + r_l * r_l;
        s = disc > 0.0 ? -pu + sqrt(disc) : -pu;
    }
    if (s < s_lo) s = s_lo;
    if (s > s_hi) s = s_hi;
    for (int it = 1; it <= cfg->max_newton; ++it) {
        double q[6];
        orc_helix(p, s, cfg->bz, q);
        double r = hypot(q[0], q[1]);
        double res = r - r_l;
        double drds = (q[0] * cos(q[4]) + q[1] * sin(q[4])) / r;
        if (res < 0.0) { if (s > s_lo) s_lo = s; }
        else { if (s < s_hi) s_hi = s; }
        if (fabs(res) < cfg->newton_tol) {
            if (drds > 0.0) s -= res / drds;
            *s_out = s;
            if (iters_out) *iters_out = it;
            return ORC_ST_OK;
        }
        double sn = s - res / drds;
        if (!(drds > 0.0) || !(sn > s_lo && sn < s_hi)) sn = 0.5 * (s_lo + s_hi);
        s = sn;
    }
    *s_out = s;
    if (iters_out) *iters_out = cfg->max_newton;
    return ORC_ST_NOCONV;
}

/* ------------------------------------------------------------------ */
/* parametrised field and Runge-Kutta transport                         */

void orc_field(const orc_cfg* cfg, const double x[3], double B[3])
{
    double u = x[2] / cfg->field_z0;
    double g = 1.0 / (1.0 + u * u);
    double bz = cfg->bz * g;
    /* dBz/dz = bz * (-2 z / Z0^2) * g; Br = -(r/2) dBz/dz */
    double dbz = -2.0 * cfg->bz * x[2] / (cfg->field_z0 * cfg->field_z0) * g * g;
    double br_over_r = -0.5 * dbz;
    B[0] = br_over_r * x[0];
    B[1] = br_over_r * x[1];
    B[2] = bz;
}

/* d/dl of (position, direction) for a charge with kq = kappa * q / p */
static void eom(const orc_cfg* cfg, double kq, const double y[6], double dy[6])
{
    double B[3];
    orc_field(cfg, y, B);
    dy[0] = y[3];
    dy[1] = y[4];
    dy[2] = y[5];
    dy[3] = kq * (y[4] * B[2] - y[5] * B[1]);
    dy[4] = kq * (y[5] * B[0] - y[3] * B[2]);
    dy[5] = kq * (y[3] * B[1] - y[4] * B[0]);
}

void orc_rk_path(const orc_cfg* cfg, const double p[6], double l, double out[6])
{
    double st = sin(p[5]);
    double y[6] = {p[0], p[1], p[2], st * cos(p[4]), st * sin(p[4]), cos(p[5])};
    double kq = KAPPA * p[3] * st;          /* q/p = c sin(theta) */
    int n = (int)ceil(fabs(l) / cfg->field_step);
    double h = n > 0 ? l / n : 0.0;
    for (int i = 0; i < n; ++i) {
        double k1[6], k2[6], k3[6], k4[6], t[6];
        eom(cfg, kq, y, k1);
        for (int j = 0; j < 6; ++j) t[j] = y[j] + 0.5 * h * k1[j];
        eom(cfg, kq, t, k2);
        for (int j = 0; j < 6; ++j) t[j] = y[j] + 0.5 * h * k2[j];
        eom(cfg, kq, t, k3);
        for (int j = 0; j < 6; ++j) t[j] = y[j] + h * k3[j];
        eom(cfg, kq, t, k4);
        for (int j = 0; j < 6; ++j) y[j] += h / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
    }
    double tt = hypot(y[3], y[4]);
    out[0] = y[0];
    out[1] = y[1];
    out[2] = y[2];
    out[5] = atan2(tt, y[5]);
    out[4] = atan2(y[4], y[3]);
    out[3] = p[3] * st / sin(out[5]);       /* q/p is conserved */
}

/* Propagate-to-radius in the parametrised field: bracketed Newton on the 3D
 * path length l with r(l) from the Runge-Kutta transport.  Start: the
 * straight-line intersection (l_init < 0) or l_init.  Bracket: the helix of
 * the start point's field (its apex), as in the uniform case, cut at
 * MAX_FIELD_PATH; a barrel whose straight-line path exceeds that is
 * unreachable. */
static int solve_barrel_field(const orc_cfg* cfg, const double p[6], double r_l, double l_init,
                              double* l_out, int* iters_out)
{
    double x0[3] = {p[0], p[1], p[2]}, B0[3];
    orc_field(cfg, x0, B0);
    orc_cfg loc = *cfg;
    loc.bz = B0[2];
    double st = sin(p[5]);
    double s_br, s_hi;
    /* reuse the uniform solve for the bracket: unreachable there is unreachable here */
    int it0 = 0;
    loc.max_newton = 1;
    int r0 = orc_solve_barrel(&loc, p, r_l, -1.0, &s_br, &it0);
    if (r0 == ORC_ST_UNREACHABLE) {
        if (iters_out) *iters_out = 0;
        return ORC_ST_UNREACHABLE;
    }
    double h = -KAPPA * loc.bz * p[3];
    s_hi = 1e30;
    if (h != 0.0) {
        double cphi = cos(p[4]), sphi = sin(p[4]);
        double cx = p[0] - sphi / h, cy = p[1] + cphi / h;
        double R = 1.0 / fabs(h), dc = hypot(cx, cy);
        double v0x = p[0] - cx, v0y = p[1] - cy;
        double v1x = R * cx / dc, v1y = R * cy / dc;
        double alpha = atan2(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y);
        double sw = fmod((h > 0 ? alpha : -alpha), 2.0 * PI);
        if (sw < 0) sw += 2.0 * PI;
        s_hi = sw / fabs(h);
    }
    double cphi = cos(p[4]), sphi = sin(p[4]);
    double pu = p[0] * cphi + p[1] * sphi;
    double disc = pu * pu - (p[0] * p[0] + p[1] * p[1]) + r_l * r_l;
    double l_line = (disc > 0.0 ? -pu + sqrt(disc) : -pu) / st;
    /* the straight line is the shortest way to the radius: beyond the
     * searched path the barrel is out of reach */
    if (l_line > MAX_FIELD_PATH) {
        if (iters_out) *iters_out = 0;
        return ORC_ST_UNREACHABLE;
    }
    double l_lo = 0.0, l_hi = fmin(s_hi / st, MAX_FIELD_PATH);
    double l = l_init >= 0.0 ? l_init : l_line;
    if (l < l_lo) l = l_lo;
    if (l > l_hi) l = l_hi;
    for (int it = 1; it <= cfg->max_newton; ++it) {
        double q[6];
        orc_rk_path(cfg, p, l, q);
        double r = hypot(q[0], q[1]);
        double res = r - r_l;
        double drdl = sin(q[5]) * (q[0] * cos(q[4]) + q[1] * sin(q[4])) / r;
        if (res < 0.0) { if (l > l_lo) l_lo = l; }
        else { if (l < l_hi) l_hi = l; }
        if (fabs(res) < cfg->newton_tol) {
            if (drdl > 0.0) l -= res / drdl;
            *l_out = l;
            if (iters_out) *iters_out = it;
            return ORC_ST_OK;
        }
        double ln = l - res / drdl;
        if (!(drdl > 0.0) || !(ln > l_lo && ln < l_hi)) ln = 0.5 * (l_lo + l_hi);
        l = ln;
    }
    *l_out = l;
    if (iters_out) *iters_out = cfg->max_newton;
    return ORC_ST_NOCONV;
}

/* Propagate-to-z in the parametrised field: bracketed Newton on the 3D path
 * length l with z(l) from the Runge-Kutta transport and dz/dl = cos theta(l).
 * Start: the straight line l0 = (z_d - z) / cos theta (exact in a uniform
 * field), or l_init >= 0.  The plane must lie ahead (0 <= l0 <=
 * MAX_FIELD_PATH).  Bracket [0, min(2 l0, MAX_FIELD_PATH)]: the field's
 * radial component bends theta only slightly, and a track that has not
 * reached the plane after twice the straight path does not reach it
 * (NOCONV).  Same stopping rule as the radius solve. */
static int solve_disk_field(const orc_cfg* cfg, const double p[6], double z_d, double l_init,
                            double* l_out, int* iters_out)
{
    double ct = cos(p[5]);
    double l0 = ct != 0.0 ? (z_d - p[2]) / ct : -1.0;
    if (!(l0 >= 0.0) || l0 > MAX_FIELD_PATH) {
        if (iters_out) *iters_out = 0;
        return ORC_ST_UNREACHABLE;
    }
    double sgn = ct > 0.0 ? 1.0 : -1.0;
    double l_lo = 0.0, l_hi = fmin(2.0 * l0, MAX_FIELD_PATH);
    double l = l_init >= 0.0 ? l_init : l0;
    if (l < l_lo) l = l_lo;
    if (l > l_hi) l = l_hi;
    for (int it = 1; it <= cfg->max_newton; ++it) {
        double q[6];
        orc_rk_path(cfg, p, l, q);
        double res = sgn * (q[2] - z_d);      /* > 0: past the plane */
        double drdl = sgn * cos(q[5]);
        if (res < 0.0) { if (l > l_lo) l_lo = l; }
        else { if (l < l_hi) l_hi = l; }
        if (fabs(res) < cfg->newton_tol) {
            if (drdl > 0.0) l -= res / drdl;
            *l_out = l;
            if (iters_out) *iters_out = it;
            return ORC_ST_OK;
        }
        double ln = l - res / drdl;
        if (!(drdl > 0.0) || !(ln > l_lo && ln < l_hi)) ln = 0.5 * (l_lo + l_hi);
        l = ln;
    }
    *l_out = l;
    if (iters_out) *iters_out = cfg->max_newton;
    return ORC_ST_NOCONV;
}

/* path length to a layer, no covariance */
static int path_to_layer(const orc_cfg* cfg, int layer, const double p[6], double* s, int* iters)
{
    const orc_layer* L = &cfg->layers[layer];
    if (cfg->field_z0 > 0.0) {
        /* parametrised field: s is the 3D path length here */
        if (L->kind != 0) return solve_disk_field(cfg, p, L->r_or_z, -1.0, s, iters);
        return solve_barrel_field(cfg, p, L->r_or_z, -1.0, s, iters);
    }
    if (L->kind == 0) return orc_solve_barrel(cfg, p, L->r_or_z, -1.0, s, iters);
    double ct = cos(p[5]);
    if (ct == 0.0) return ORC_ST_UNREACHABLE;
    *s = (L->r_or_z - p[2]) * sin(p[5]) / ct;
    if (iters) *iters = 1;
    return *s >= 0.0 ? ORC_ST_OK : ORC_ST_UNREACHABLE;
}

/* ------------------------------------------------------------------ */
/* transport Jacobian at path length s                                 */

static void jacobian_at_bz(double bz, const orc_layer* L, const double p[6], double s,
                           double F[6][6])
{
    double kb = KAPPA * bz;
    double h = -kb * p[3];
    double u = 0.5 * h * s;
    double a = p[4] + u;
    double sc = sinc(u), dsc = dsinc(u);
    double ca = cos(a), sa = sin(a);
    double st = sin(p[5]), ct = cos(p[5]);
    double q[6];
    orc_helix(p, s, bz, q);

    /* partial derivatives at fixed s */
    double D[6][6];
    memset(D, 0, sizeof(D));
    for (int i = 0; i < 6; ++i) D[i][i] = 1.0;
    D[0][4] = -s * sa * sc;
    D[1][4] = s * ca * sc;
    double dxdh = 0.5 * s * s * (ca * dsc - sa * sc);
    double dydh = 0.5 * s * s * (sa * dsc + ca * sc);
    D[0][3] = -kb * dxdh;
    D[1][3] = -kb * dydh;
    D[4][3] = -kb * s;
    D[2][5] = -s / (st * st);

    /* derivative of the helix with respect to s */
    double phis = p[4] + h * s;
    double fs[6] = {cos(phis), sin(phis), ct / st, 0.0, h, 0.0};

    /* derivative of the path length with respect to the starting state */
    double dsdp[6] = {0, 0, 0, 0, 0, 0};
    if (L->kind == 0) {
        double den = q[0] * fs[0] + q[1] * fs[1];
        for (int j = 0; j < 6; ++j) dsdp[j] = -(q[0] * D[0][j] + q[1] * D[1][j]) / den;
    } else {
        dsdp[2] = -st / ct;
        dsdp[5] = (L->r_or_z - p[2]) / (ct * ct);
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) F[i][j] = D[i][j] + fs[i] * dsdp[j];
}

static void jacobian_at(const orc_cfg* cfg, const orc_layer* L, const double p[6], double s,
                        double F[6][6])
{
    jacobian_at_bz(cfg->bz, L, p, s, F);
}

/* Field-dependent parts of a propagation over path s (transverse arc in the
 * uniform field, 3D length in the parametrised one): end state and Jacobian. */
static void transport_parts(const orc_cfg* cfg, const orc_layer* L, const double p[6], double s,
                            double q[6], double F[6][6])
{
    if (cfg->field_z0 > 0.0) {
        orc_rk_path(cfg, p, s, q);
        /* the helix Jacobian over the transverse path, in the path's mean
         * effective axial field: the transverse turning rate is
         * -kappa c (Bz - cot(theta) B_T . t_T), where the transverse field
         * bends a track that moves along z; averaged by Simpson's rule over
         * the start, the chord's midpoint (mean direction) and the end */
        double dphi = wrap_pi(q[4] - p[4]);
        double pts[3][5] = {{p[0], p[1], p[2], p[4], p[5]},
                            {0.5 * (p[0] + q[0]), 0.5 * (p[1] + q[1]), 0.5 * (p[2] + q[2]),
                             p[4] + 0.5 * dphi, 0.5 * (p[5] + q[5])},
                            {q[0], q[1], q[2], q[4], q[5]}};
        double beff[3];
        for (int k = 0; k < 3; ++k) {
            double B[3];
            orc_field(cfg, pts[k], B);
            double bt = B[0] * cos(pts[k][3]) + B[1] * sin(pts[k][3]);
            beff[k] = B[2] - cos(pts[k][4]) / sin(pts[k][4]) * bt;
        }
        jacobian_at_bz((beff[0] + 4.0 * beff[1] + beff[2]) / 6.0, L, p, s * sin(p[5]), F);
    } else {
        orc_helix(p, s, cfg->bz, q);
        jacobian_at(cfg, L, p, s, F);
    }
}

int orc_jacobian(const orc_cfg* cfg, int layer, const double p[6], double Fo[36])
{
    double s;
    int st = path_to_layer(cfg, layer, p, &s, NULL);
    if (st) return st;
    double F[6][6], q[6];
    transport_parts(cfg, &cfg->layers[layer], p, s, q, F);
    memcpy(Fo, F, sizeof(F));
    return 0;
}

/* ------------------------------------------------------------------ */
/* multiple-scattering process noise at a layer (PDG Highland formula)  */

/* |cos| of the angle between the track and the surface normal */
static double incidence(const orc_layer* L, const double q[6])
{
    double st = sin(q[5]), ct = cos(q[5]);
    double cosa;
    if (L->kind == 0) cosa = st * cos(q[4] - atan2(q[1], q[0]));
    else cosa = ct;
    cosa = fabs(cosa);
    if (cosa < 1e-6) cosa = 1e-6;
    return cosa;
}

static void add_scatter(const orc_cfg* cfg, const orc_layer* L, double x0, const double q[6],
                        double P[6][6])
{
    if (!(x0 > 0.0)) return;
    double st = sin(q[5]), ct = cos(q[5]);
    double t = x0 / incidence(L, q);
    double pmom = 1.0 / (fabs(q[3]) * st);
    double beta = pmom / sqrt(pmom * pmom + cfg->mass * cfg->mass);
    double th0 = 0.0136 / (beta * pmom) * sqrt(t) * (1.0 + 0.038 * log(t / (beta * beta)));
    double t2 = th0 * th0;
    double cot = ct / st;
    P[4][4] += t2 / (st * st);
    P[5][5] += t2;
    P[3][5] += -q[3] * cot * t2;
    P[5][3] += -q[3] * cot * t2;
    P[3][3] += q[3] * q[3] * cot * cot * t2;
}

/* Mean ionisation energy loss per unit areal density (PDG "Passage of
 * particles through matter": the Bethe formula with the maximum energy
 * transfer to an electron, without density-effect or shell corrections), for
 * silicon: Z/A = 0.49848, I = 173 eV.  Units MeV cm^2 / g. */
double orc_dedx(double p, double m)
{
    const double K = 0.307075, ZA = 0.49848, I = 173e-6, me = 0.51099895;  /* MeV */
    double M = m * 1e3;
    double pm = p * 1e3;
    double E = sqrt(pm * pm + M * M);
    double beta = pm / E, gamma = E / M;
    double bg2 = beta * beta * gamma * gamma;
    double tmax = 2.0 * me * bg2 / (1.0 + 2.0 * gamma * me / M + (me / M) * (me / M));
    return K * ZA / (beta * beta) * (0.5 * log(2.0 * me * bg2 * tmax / (I * I)) - beta * beta);
}

/* Material at a crossing: the map's cell at the crossing point, else the
 * layer's own thickness and no energy loss. */
static void material_at(const orc_cfg* cfg, const orc_layer* L, const double q[6], double* x0,
                        double* xi)
{
    if (!cfg->mat_x0) {
        *x0 = L->x0;
        *xi = 0.0;
        return;
    }
    double r = hypot(q[0], q[1]);
    int ir = (int)floor(r / (cfg->mat_rmax / cfg->mat_nr));
    int iz = (int)floor((q[2] - cfg->mat_zmin) / ((cfg->mat_zmax - cfg->mat_zmin) / cfg->mat_nz));
    if (ir < 0) ir = 0;
    if (ir >= cfg->mat_nr) ir = cfg->mat_nr - 1;
    if (iz < 0) iz = 0;
    if (iz >= cfg->mat_nz) iz = cfg->mat_nz - 1;
    *x0 = cfg->mat_x0[ir * cfg->mat_nz + iz];
    *xi = cfg->mat_xi[ir * cfg->mat_nz + iz];
}

/* Mean energy loss over the crossed thickness xi / cos(alpha): the momentum
 * magnitude drops to p' with E' = E - dE (the loss capped at half the
 * kinetic energy: a track that would stop keeps a finite state), direction
 * kept, so c' = c p / p'; the covariance follows the Jacobian
 * dc'/dc = (p/p')^3 E'/E of the loss at fixed dE. */
static void energy_loss(const orc_cfg* cfg, const orc_layer* L, double xi, double q[6],
                        double P[6][6])
{
    if (!(xi > 0.0)) return;
    double st = sin(q[5]);
    double p = 1.0 / (fabs(q[3]) * st);
    double m = cfg->mass;
    double E = sqrt(p * p + m * m);
    double dE = orc_dedx(p, m) * xi / incidence(L, q) * 1e-3;     /* GeV */
    if (dE > 0.5 * (E - m)) dE = 0.5 * (E - m);
    double E1 = E - dE;
    double p1 = sqrt(E1 * E1 - m * m);
    double J = (p / p1) * (p / p1) * (p / p1) * (E1 / E);
    q[3] *= p / p1;
    for (int k = 0; k < 6; ++k) {
        P[3][k] *= J;
        P[k][3] *= J;
    }
}

static void material_effects(const orc_cfg* cfg, const orc_layer* L, double q[6], double P[6][6])
{
    double x0, xi;
    material_at(cfg, L, q, &x0, &xi);
    add_scatter(cfg, L, x0, q, P);
    energy_loss(cfg, L, xi, q, P);
}

void orc_material(const orc_cfg* cfg, int layer, double q[6], double Pk[21])
{
    double P[6][6];
    unpack(Pk, P);
    material_effects(cfg, &cfg->layers[layer], q, P);
    pack(P, Pk);
}

int orc_propagate(const orc_cfg* cfg, int layer, const double p[6], const double Pk[21],
                  double p_out[6], double P_out[21], double* s_out, int* iters_out,
                  int add_noise)
{
    double s;
    int it = 0;
    int st = path_to_layer(cfg, layer, p, &s, &it);
    if (iters_out) *iters_out = it;
    if (st) return st;
    const orc_layer* L = &cfg->layers[layer];
    double q[6], F[6][6], P[6][6], T[6][6], Pn[6][6];
    transport_parts(cfg, L, p, s, q, F);
    unpack(Pk, P);
    mul66(F, P, T);
    mul66t(T, F, Pn);
    if (add_noise) material_effects(cfg, L, q, Pn);
    memcpy(p_out, q, sizeof(q));
    pack(Pn, P_out);
    if (s_out) *s_out = s;
    for (int i = 0; i < 6; ++i)
        if (!isfinite(q[i])) return ORC_ST_NAN;
    return ORC_ST_OK;
}

/* ------------------------------------------------------------------ */
/* measurement model and update                                        */

/* H (2x6) and residual r for a hit; local frame at the hit's azimuth:
 * u along phi, v along z (barrel) or along r (disk). */
static void measurement(const double p[6], const double hit[5], int kind, double H[2][6],
                        double r[2])
{
    double rho = hypot(hit[0], hit[1]);
    double c = hit[0] / rho, s = hit[1] / rho;
    memset(H, 0, sizeof(double) * 12);
    H[0][0] = -s;
    H[0][1] = c;
    r[0] = -s * (hit[0] - p[0]) + c * (hit[1] - p[1]);
    if (kind == 0) {
        H[1][2] = 1.0;
        r[1] = hit[2] - p[2];
    } else {
        H[1][0] = c;
        H[1][1] = s;
        r[1] = c * (hit[0] - p[0]) + s * (hit[1] - p[1]);
    }
}

/* S = H P H^T + V and its inverse; returns 0 when S is not positive definite */
static int innovation(double P[6][6], double H[2][6], const double hit[5], double S[2][2],
                      double Si[2][2])
{
    double HP[2][6];
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += H[a][k] * P[k][j];
            HP[a][j] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += HP[a][k] * H[b][k];
            S[a][b] = acc;
        }
    S[0][0] += hit[3] * hit[3];
    S[1][1] += hit[4] * hit[4];
    double det = S[0][0] * S[1][1] - S[0][1] * S[1][0];
    if (!(det > 0.0) || !(S[0][0] > 0.0)) return 0;
    Si[0][0] = S[1][1] / det;
    Si[1][1] = S[0][0] / det;
    Si[0][1] = -S[0][1] / det;
    Si[1][0] = -S[1][0] / det;
    return 1;
}

double orc_chi2(const double p[6], const double Pk[21], const double hit[5], int kind)
{
    double P[6][6], H[2][6], r[2], S[2][2], Si[2][2];
    unpack(Pk, P);
    measurement(p, hit, kind, H, r);
    if (!innovation(P, H, hit, S, Si)) return INFINITY;
    return r[0] * (Si[0][0] * r[0] + Si[0][1] * r[1]) + r[1] * (Si[1][0] * r[0] + Si[1][1] * r[1]);
}

int orc_update(const double p[6], const double Pk[21], const double hit[5], int kind,
               double p_out[6], double P_out[21], double* chi2_out)
{
    double P[6][6], H[2][6], r[2], S[2][2], Si[2][2];
    unpack(Pk, P);
    measurement(p, hit, kind, H, r);
    if (!innovation(P, H, hit, S, Si)) return ORC_ST_NONPD;
    double chi2 = r[0] * (Si[0][0] * r[0] + Si[0][1] * r[1]) +
                  r[1] * (Si[1][0] * r[0] + Si[1][1] * r[1]);
    /* gain K = P H^T S^-1 */
    double PHt[6][2], K[6][2];
    for (int i = 0; i < 6; ++i)
        for (int a = 0; a < 2; ++a) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k) acc += P[i][k] * H[a][k];
            PHt[i][a] = acc;
        }
    for (int i = 0; i < 6; ++i)
        for (int a = 0; a < 2; ++a) K[i][a] = PHt[i][0] * Si[0][a] + PHt[i][1] * Si[1][a];
    for (int i = 0; i < 6; ++i) p_out[i] = p[i] + K[i][0] * r[0] + K[i][1] * r[1];
    p_out[4] = wrap_pi(p_out[4]);
    /* Joseph form: (I - K H) P (I - K H)^T + K V K^T */
    double A[6][6], T[6][6], Pn[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j)
            A[i][j] = (i == j ? 1.0 : 0.0) - (K[i][0] * H[0][j] + K[i][1] * H[1][j]);
    mul66(A, P, T);
    mul66t(T, A, Pn);
    double v0 = hit[3] * hit[3], v1 = hit[4] * hit[4];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Pn[i][j] += K[i][0] * v0 * K[j][0] + K[i][1] * v1 * K[j][1];
    pack(Pn, P_out);
    if (chi2_out) *chi2_out = chi2;
    for (int i = 0; i < 6; ++i)
        if (!isfinite(p_out[i])) return ORC_ST_NAN;
    return ORC_ST_OK;
}

/* ------------------------------------------------------------------ */
/* seed from three hits                                                 */
/*
 * Signed curvature of the circle through the three transverse points
 * (Menger curvature, sign = sense of rotation 1 -> 2 -> 3), tangent
 * direction at hit 1 = chord 1->3 direction minus half the turning angle,
 * cot(theta) = dz / arc length between hits 1 and 3, position = hit 1.
 * Prior covariance: diag(1, 1, 1, 4, 0.01, 0.01) (cm^2, GeV^-2, rad^2).
 */
void orc_seed(const double h1[3], const double h2[3], const double h3[3], double bz,
              double p_out[6], double P_out[21])
{
    double ax = h2[0] - h1[0], ay = h2[1] - h1[1];
    double bx = h3[0] - h1[0], by = h3[1] - h1[1];
    double d12 = hypot(ax, ay);
    double d13 = hypot(bx, by);
    double d23 = hypot(h3[0] - h2[0], h3[1] - h2[1]);
    double cross = ax * by - ay * bx;
    double h = 2.0 * cross / (d12 * d23 * d13);
    double w = 0.5 * h * d13;
    if (w > 1.0) w = 1.0;
    if (w < -1.0) w = -1.0;
    double s13 = fabs(w) < 1e-8 ? d13 : d13 * asin(w) / w;
    double phi = atan2(by, bx) - 0.5 * h * s13;
    p_out[0] = h1[0];
    p_out[1] = h1[1];
    p_out[2] = h1[2];
    p_out[3] = -h / (KAPPA * bz);
    p_out[4] = wrap_pi(phi);
    p_out[5] = atan2(s13, h3[2] - h1[2]);
    double P[6][6];
    memset(P, 0, sizeof(P));
    P[0][0] = P[1][1] = P[2][2] = 1.0;
    P[3][3] = 4.0;
    P[4][4] = P[5][5] = 0.01;
    pack(P, P_out);
}

/* ------------------------------------------------------------------ */
/* fit                                                                 */

typedef struct {
    const orc_cfg* cfg;
    long lo, hi;
    int max_steps;
    const double *hx, *hy, *hz, *hsu, *hsv;
    const int *layer_seq, *hit_idx;
    double *par, *cov, *chi2;
    int *ndf, *status;
} fit_job;

static void fit_one(const fit_job* J, long t)
{
    const orc_cfg* cfg = J->cfg;
    double p[6], Pk[21], chi2 = 0.0;
    memcpy(p, J->par + 6 * t, sizeof(p));
    memcpy(Pk, J->cov + 21 * t, sizeof(Pk));
    int nh = 0, st = 0;
    for (int k = 0; k < J->max_steps; ++k) {
        int layer = J->layer_seq[(long)t * J->max_steps + k];
        if (layer < 0) break;
        double q[6], Q[21];
        st |= orc_propagate(cfg, layer, p, Pk, q, Q, NULL, NULL, cfg->use_material);
        if (st) break;
        memcpy(p, q, sizeof(p));
        memcpy(Pk, Q, sizeof(Pk));
        int hi = J->hit_idx[(long)t * J->max_steps + k];
        if (hi >= 0) {
            double hit[5] = {J->hx[hi], J->hy[hi], J->hz[hi], J->hsu[hi], J->hsv[hi]};
            double c2;
            st |= orc_update(p, Pk, hit, cfg->layers[layer].kind, q, Q, &c2);
            if (st) break;
            memcpy(p, q, sizeof(p));
            memcpy(Pk, Q, sizeof(Pk));
            chi2 += c2;
            nh++;
        }
    }
    memcpy(J->par + 6 * t, p, sizeof(p));
    memcpy(J->cov + 21 * t, Pk, sizeof(Pk));
    J->chi2[t] = chi2;
    J->ndf[t] = 2 * nh - 5;
    J->status[t] = st;
}

static void* fit_worker(void* arg)
{
    fit_job* J = (fit_job*)arg;
    for (long t = J->lo; t < J->hi; ++t) fit_one(J, t);
    return NULL;
}

void orc_fit(const orc_cfg* cfg, long n, int max_steps,
             const double* hx, const double* hy, const double* hz,
             const double* hsu, const double* hsv,
             const int* layer_seq, const int* hit_idx,
             double* par_io, double* cov_io, double* chi2_out, int* ndf_out,
             int* status_out, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    fit_job jobs[256];
    pthread_t th[256];
    for (int i = 0; i < n_threads; ++i) {
        fit_job J = {cfg, n * i / n_threads, n * (i + 1) / n_threads, max_steps,
                     hx, hy, hz, hsu, hsv, layer_seq, hit_idx,
                     par_io, cov_io, chi2_out, ndf_out, status_out};
        jobs[i] = J;
    }
    if (n_threads == 1) { fit_worker(&jobs[0]); return; }
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, fit_worker, &jobs[i]);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------ */
/* combinatorial finding                                                */

typedef struct {
    double p[6], P[21];
    double chi2;
    int nhits, misses, done, status;
    int pos;                 /* steering: next plan entry */
    int hits[MAXL];
    int visit[MAXL];         /* walk step at which each layer was last reached (-1: never) */
} cand_t;

typedef struct {
    int parent;      /* slot of the parent candidate */
    int hit;         /* original hit index, NO_HIT for the no-hit / frozen child */
    double chi2_hit;
    double chi2_tot;
    int nhits;
} child_t;

typedef struct {
    /* hits of one event */
    long n_hits;
    const double *hx, *hy, *hz, *hsu, *hsv;
    const int* hlayer;
    /* per-layer hit lists (all-hits scan) and bins (binned scan) */
    long* layer_off;     /* [n_layers+1] into layer_hits */
    long* layer_hits;
    long** bin_off;      /* per layer: [nbin_phi*nbin_2 + 1] into bin_hits[layer] */
    long** bin_hits;
} event_index;

static int hit_phi_bin(double phi, int nb)
{
    int b = (int)floor((phi + PI) * nb / (2.0 * PI));
    if (b < 0) b = 0;
    if (b > nb - 1) b = nb - 1;
    return b;
}

static int coord_bin(double v, double lo, double hi, int nb)
{
    double t = floor((v - lo) * nb / (hi - lo));
    if (!(t >= 0)) t = 0;
    if (t > nb - 1) t = nb - 1;
    return (int)t;
}

static double hit_coord2(const event_index* E, const orc_layer* L, long i)
{
    return L->kind == 0 ? E->hz[i] : hypot(E->hx[i], E->hy[i]);
}

static void build_index(const orc_cfg* cfg, event_index* E)
{
    int nl = cfg->n_layers;
    E->layer_off = (long*)calloc((size_t)(nl > 0 ? nl : 0) + 1, sizeof(long));
    E->layer_hits = (long*)malloc(sizeof(long) * (E->n_hits > 0 ? E->n_hits : 1));
    for (long i = 0; i < E->n_hits; ++i) E->layer_off[E->hlayer[i] + 1]++;
    for (int l = 0; l < nl; ++l) E->layer_off[l + 1] += E->layer_off[l];
    long* fill = (long*)calloc((size_t)(nl > 0 ? nl : 1), sizeof(long));
    for (long i = 0; i < E->n_hits; ++i) {
        int l = E->hlayer[i];
        E->layer_hits[E->layer_off[l] + fill[l]++] = i;
    }
    free(fill);
    E->bin_off = (long**)calloc((size_t)(nl > 0 ? nl : 1), sizeof(long*));
    E->bin_hits = (long**)calloc((size_t)(nl > 0 ? nl : 1), sizeof(long*));
    for (int l = 0; l < nl; ++l) {
        const orc_layer* L = &cfg->layers[l];
        int nb = L->nbin_phi * L->nbin_2;
        long n = E->layer_off[l + 1] - E->layer_off[l];
        long* off = (long*)calloc((size_t)(nb > 0 ? nb : 0) + 1, sizeof(long));
        long* hits = (long*)malloc(sizeof(long) * (n > 0 ? n : 1));
        int* bin_of = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
        for (long k = 0; k < n; ++k) {
            long i = E->layer_hits[E->layer_off[l] + k];
            int bp = hit_phi_bin(atan2(E->hy[i], E->hx[i]), L->nbin_phi);
            int bv = coord_bin(hit_coord2(E, L, i), L->lo, L->hi, L->nbin_2);
            bin_of[k] = bp * L->nbin_2 + bv;
            off[bin_of[k] + 1]++;
        }
        for (int b = 0; b < nb; ++b) off[b + 1] += off[b];
        long* f2 = (long*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(long));
        for (long k = 0; k < n; ++k) {
            int b = bin_of[k];
            hits[off[b] + f2[b]++] = E->layer_hits[E->layer_off[l] + k];
        }
        free(f2);
        free(bin_of);
        E->bin_off[l] = off;
        E->bin_hits[l] = hits;
    }
}

static void free_index(const orc_cfg* cfg, event_index* E)
{
    for (int l = 0; l < cfg->n_layers; ++l) {
        free(E->bin_off[l]);
        free(E->bin_hits[l]);
    }
    free(E->bin_off);
    free(E->bin_hits);
    free(E->layer_off);
    free(E->layer_hits);
}

/*
 * Next surface in the parametrised field: whichever comes first along the
 * 3D path, the next barrel outward (radius above rho + NEXT_BARREL_EPS),
 * reached by the Runge-Kutta radius solve and crossed inside |z| <= hi, or a
 * disk ahead (|dz| > DISK_AHEAD_EPS in the direction of travel), reached by
 * the Runge-Kutta z solve and crossed inside its radial extent; both within
 * half a turn of the start point's curvature in the transverse plane.  The
 * disks are taken in layer order; a disk whose straight-line path already
 * exceeds the best path found, or whose straight-line transverse path exceeds
 * half a turn, by more than 1% + 1 cm is not solved (the solved path differs
 * from the straight one by far less).
 */
static int navigate_field(const orc_cfg* cfg, const double p[6], int* stat, int* close)
{
    double rho = hypot(p[0], p[1]);
    int bl = -1;
    for (int l = 0; l < cfg->n_layers; ++l) {
        const orc_layer* L = &cfg->layers[l];
        if (L->kind != 0) continue;
        if (fabs(L->r_or_z - (rho + NEXT_BARREL_EPS)) < CLOSE_REL * NEXT_BARREL_EPS) *close = 1;
        if (L->r_or_z > rho + NEXT_BARREL_EPS && (bl < 0 || L->r_or_z < cfg->layers[bl].r_or_z))
            bl = l;
    }
    double x0[3] = {p[0], p[1], p[2]}, B0[3];
    orc_field(cfg, x0, B0);
    double hh = fabs(KAPPA * B0[2] * p[3]);
    double s_max = hh > 0.0 ? PI / hh : INFINITY;
    double h0 = -KAPPA * B0[2] * p[3];
    double st = sin(p[5]), ct = cos(p[5]);
    double best = INFINITY, l_b = INFINITY;
    int best_l = -1;
    if (bl >= 0) {
        const orc_layer* L = &cfg->layers[bl];
        if (h0 != 0.0) {
            /* reachability comes from the start point's helix: its farthest radius */
            double cx = p[0] - sin(p[4]) / h0, cy = p[1] + cos(p[4]) / h0;
            double rmax = hypot(cx, cy) + 1.0 / fabs(h0);
            if (fabs(rmax - L->r_or_z) < CLOSE_REL * L->r_or_z) *close = 1;
        }
        double l;
        int r = solve_barrel_field(cfg, p, L->r_or_z, -1.0, &l, NULL);
        if (r == ORC_ST_NOCONV) {
            *stat |= ORC_ST_NOCONV;
            return -1;
        }
        if (r == ORC_ST_OK) {
            double q[6];
            orc_rk_path(cfg, p, l, q);
            double s = l * st;
            if (fabs(fabs(q[2]) - L->hi) < CLOSE_REL * L->hi) *close = 1;
            if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
            if (fabs(q[2]) <= L->hi && s <= s_max) {
                best = l_b = l;
                best_l = bl;
            }
        }
    }
    for (int l = 0; l < cfg->n_layers; ++l) {
        const orc_layer* L = &cfg->layers[l];
        if (L->kind != 1) continue;
        double dz = L->r_or_z - p[2];
        if (fabs(fabs(dz) - DISK_AHEAD_EPS) < CLOSE_REL * DISK_AHEAD_EPS) *close = 1;
        if (!(dz * ct > 0.0) || fabs(dz) <= DISK_AHEAD_EPS) continue;
        double l_line = dz / ct;
        if (l_line > 1.01 * best + 1.0 || l_line * st > 1.01 * s_max + 1.0) continue;
        double ld;
        int r = solve_disk_field(cfg, p, L->r_or_z, -1.0, &ld, NULL);
        if (r == ORC_ST_NOCONV) {
            *stat |= ORC_ST_NOCONV;
            return -1;
        }
        if (r != ORC_ST_OK) continue;
        double q[6];
        orc_rk_path(cfg, p, ld, q);
        double rr = hypot(q[0], q[1]);
        double s = ld * st;
        if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
        if (fabs(rr - L->lo) < CLOSE_REL * L->lo || fabs(rr - L->hi) < CLOSE_REL * L->hi) *close = 1;
        if (s > s_max || rr < L->lo || rr > L->hi) continue;
        if (isfinite(l_b) && fabs(ld - l_b) < CLOSE_REL * (ld > l_b ? ld : l_b)) *close = 1;
        if (ld < best) {
            best = ld;
            best_l = l;
        }
    }
    return best_l;
}

/*
 * Next surface (dynamic navigation): the candidate moves to whichever is
 * reached first along the helix, the next barrel outward (smallest radius
 * above the current one, reachable, crossing inside its z extent) or the
 * first disk ahead in z whose crossing lies inside its radial extent.
 * Returns the layer or -1 (no surface left); *stat gets NOCONV if the
 * barrel solve failed.  *close is set when a decision had a relative
 * margin below 1e-3.
 */
static int navigate(const orc_cfg* cfg, const double p[6], int* stat, int* close)
{
    if (cfg->field_z0 > 0.0) return navigate_field(cfg, p, stat, close);
    double rho = hypot(p[0], p[1]);
    /* only surfaces reached within half a turn in the transverse plane */
    double hh = fabs(KAPPA * cfg->bz * p[3]);
    double s_max = hh > 0.0 ? PI / hh : INFINITY;
    double best_s = INFINITY;
    int best_l = -1;
    int bl = -1;
    for (int l = 0; l < cfg->n_layers; ++l) {
        const orc_layer* L = &cfg->layers[l];
        if (L->kind != 0) continue;
        if (fabs(L->r_or_z - (rho + NEXT_BARREL_EPS)) < CLOSE_REL * NEXT_BARREL_EPS) *close = 1;
        if (L->r_or_z > rho + NEXT_BARREL_EPS && (bl < 0 || L->r_or_z < cfg->layers[bl].r_or_z))
            bl = l;
    }
    double s_b = INFINITY;
    if (bl >= 0) {
        const orc_layer* L = &cfg->layers[bl];
        double h = -KAPPA * cfg->bz * p[3];
        if (h != 0.0) {
            double cx = p[0] - sin(p[4]) / h, cy = p[1] + cos(p[4]) / h;
            double rmax = hypot(cx, cy) + 1.0 / fabs(h);
            if (fabs(rmax - L->r_or_z) < CLOSE_REL * L->r_or_z) *close = 1;
        }
        double s;
        int st = orc_solve_barrel(cfg, p, L->r_or_z, -1.0, &s, NULL);
        if (st == ORC_ST_NOCONV) {
            *stat |= ORC_ST_NOCONV;
            return -1;
        }
        if (st == ORC_ST_OK) {
            double zc = p[2] + s * cos(p[5]) / sin(p[5]);
            if (fabs(fabs(zc) - L->hi) < CLOSE_REL * L->hi) *close = 1;
            if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
            if (fabs(zc) <= L->hi && s <= s_max) {
                best_s = s_b = s;
                best_l = bl;
            }
        }
    }
    double cot = cos(p[5]) / sin(p[5]);
    for (int l = 0; l < cfg->n_layers; ++l) {
        const orc_layer* L = &cfg->layers[l];
        if (L->kind != 1) continue;
        double dz = L->r_or_z - p[2];
        if (fabs(fabs(dz) - DISK_AHEAD_EPS) < CLOSE_REL * DISK_AHEAD_EPS) *close = 1;
        if (!(dz * cot > 0.0) || fabs(dz) <= DISK_AHEAD_EPS) continue;
        double s = dz / cot;
        if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
        if (s > s_max) continue;
        double q[6];
        orc_helix(p, s, cfg->bz, q);
        double r = hypot(q[0], q[1]);
        if (fabs(r - L->lo) < CLOSE_REL * L->lo || fabs(r - L->hi) < CLOSE_REL * L->hi) *close = 1;
        if (r < L->lo || r > L->hi) continue;
        if (isfinite(s_b) && fabs(s - s_b) < CLOSE_REL * (s > s_b ? s : s_b)) *close = 1;
        if (s < best_s) {
            best_s = s;
            best_l = l;
        }
    }
    return best_l;
}

/*
 * Steering (Sec. 3.1: a tracking region's list of layers to traverse).  From
 * plan entry *pos on, the first layer the candidate actually reaches: a
 * barrel outside rho + NEXT_BARREL_EPS whose outward crossing lies within
 * half a turn and inside |z| <= hi, or a disk ahead (|dz| > DISK_AHEAD_EPS)
 * crossed within half a turn inside its radial extent.  Entries not reached
 * are passed over.  Returns the layer (and sets *pos past it) or -1 when the
 * plan is exhausted; a failed barrel solve sets NOCONV and returns -1.
 */
/*
 * Steering in the parametrised field: the same rule along the 3D path, each
 * plan entry reached by its Runge-Kutta solve (radius or z) as in
 * navigate_field, half a turn taken at the start point's curvature; a disk
 * whose straight-line transverse path exceeds half a turn by more than 1% +
 * 1 cm is not solved.
 */
static int steer_field(const orc_cfg* cfg, const orc_region* R, int* pos, const double p[6],
                       int* stat, int* close)
{
    double rho = hypot(p[0], p[1]);
    double x0[3] = {p[0], p[1], p[2]}, B0[3];
    orc_field(cfg, x0, B0);
    double h0 = -KAPPA * B0[2] * p[3];
    double s_max = h0 != 0.0 ? PI / fabs(h0) : INFINITY;
    double st = sin(p[5]), ct = cos(p[5]);
    for (; *pos < R->n; ++*pos) {
        int l = R->layers[*pos];
        const orc_layer* L = &cfg->layers[l];
        double q[6];
        if (L->kind == 0) {
            if (fabs(L->r_or_z - (rho + NEXT_BARREL_EPS)) < CLOSE_REL * NEXT_BARREL_EPS) *close = 1;
            if (!(L->r_or_z > rho + NEXT_BARREL_EPS)) continue;
            if (h0 != 0.0) {
                double cx = p[0] - sin(p[4]) / h0, cy = p[1] + cos(p[4]) / h0;
                double rmax = hypot(cx, cy) + 1.0 / fabs(h0);
                if (fabs(rmax - L->r_or_z) < CLOSE_REL * L->r_or_z) *close = 1;
            }
            double ll;
            int r = solve_barrel_field(cfg, p, L->r_or_z, -1.0, &ll, NULL);
            if (r == ORC_ST_NOCONV) {
                *stat |= ORC_ST_NOCONV;
                return -1;
            }
            if (r != ORC_ST_OK) continue;
            orc_rk_path(cfg, p, ll, q);
            double s = ll * st;
            if (fabs(fabs(q[2]) - L->hi) < CLOSE_REL * L->hi) *close = 1;
            if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
            if (fabs(q[2]) > L->hi || s > s_max) continue;
        } else {
            double dz = L->r_or_z - p[2];
            if (fabs(fabs(dz) - DISK_AHEAD_EPS) < CLOSE_REL * DISK_AHEAD_EPS) *close = 1;
            if (!(dz * ct > 0.0) || fabs(dz) <= DISK_AHEAD_EPS) continue;
            if (dz / ct * st > 1.01 * s_max + 1.0) continue;
            double ld;
            int r = solve_disk_field(cfg, p, L->r_or_z, -1.0, &ld, NULL);
            if (r == ORC_ST_NOCONV) {
                *stat |= ORC_ST_NOCONV;
                return -1;
            }
            if (r != ORC_ST_OK) continue;
            orc_rk_path(cfg, p, ld, q);
            double rr = hypot(q[0], q[1]);
            double s = ld * st;
            if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
            if (fabs(rr - L->lo) < CLOSE_REL * L->lo || fabs(rr - L->hi) < CLOSE_REL * L->hi) *close = 1;
            if (s > s_max || rr < L->lo || rr > L->hi) continue;
        }
        ++*pos;
        return l;
    }
    return -1;
}

static int steer(const orc_cfg* cfg, const orc_region* R, int* pos, const double p[6], int* stat,
                 int* close)
{
    if (cfg->field_z0 > 0.0) return steer_field(cfg, R, pos, p, stat, close);
    double rho = hypot(p[0], p[1]);
    double hh = fabs(KAPPA * cfg->bz * p[3]);
    double s_max = hh > 0.0 ? PI / hh : INFINITY;
    double cot = cos(p[5]) / sin(p[5]);
    for (; *pos < R->n; ++*pos) {
        int l = R->layers[*pos];
        const orc_layer* L = &cfg->layers[l];
        if (L->kind == 0) {
            if (fabs(L->r_or_z - (rho + NEXT_BARREL_EPS)) < CLOSE_REL * NEXT_BARREL_EPS) *close = 1;
            if (!(L->r_or_z > rho + NEXT_BARREL_EPS)) continue;
            double h = -KAPPA * cfg->bz * p[3];
            if (h != 0.0) {
                double cx = p[0] - sin(p[4]) / h, cy = p[1] + cos(p[4]) / h;
                double rmax = hypot(cx, cy) + 1.0 / fabs(h);
                if (fabs(rmax - L->r_or_z) < CLOSE_REL * L->r_or_z) *close = 1;
            }
            double s;
            int st = orc_solve_barrel(cfg, p, L->r_or_z, -1.0, &s, NULL);
            if (st == ORC_ST_NOCONV) {
                *stat |= ORC_ST_NOCONV;
                return -1;
            }
            if (st != ORC_ST_OK) continue;
            double zc = p[2] + s * cot;
            if (fabs(fabs(zc) - L->hi) < CLOSE_REL * L->hi) *close = 1;
            if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
            if (fabs(zc) > L->hi || s > s_max) continue;
        } else {
            double dz = L->r_or_z - p[2];
            if (fabs(fabs(dz) - DISK_AHEAD_EPS) < CLOSE_REL * DISK_AHEAD_EPS) *close = 1;
            if (!(dz * cot > 0.0) || fabs(dz) <= DISK_AHEAD_EPS) continue;
            double s = dz / cot;
            if (fabs(s - s_max) < CLOSE_REL * s_max) *close = 1;
            if (s > s_max) continue;
            double q[6];
            orc_helix(p, s, cfg->bz, q);
            double r = hypot(q[0], q[1]);
            if (fabs(r - L->lo) < CLOSE_REL * L->lo || fabs(r - L->hi) < CLOSE_REL * L->hi) *close = 1;
            if (r < L->lo || r > L->hi) continue;
        }
        ++*pos;
        return l;
    }
    return -1;
}

/* The region of a seed state (first containing its eta), or -1; *close when
 * eta lies within 1e-3 of a region edge. */
static int seed_region(const orc_cfg* cfg, const double p[6], int* close)
{
    double eta = -log(tan(0.5 * p[5]));
    for (int g = 0; g < cfg->n_regions; ++g) {
        const orc_region* R = &cfg->regions[g];
        if (fabs(eta - R->eta_lo) < 1e-3 || fabs(eta - R->eta_hi) < 1e-3) *close = 1;
    }
    for (int g = 0; g < cfg->n_regions; ++g)
        if (eta >= cfg->regions[g].eta_lo && eta < cfg->regions[g].eta_hi) return g;
    return -1;
}

/* hits inside the window of a predicted state; returns count, writes (chi2, idx)
 * of the accepted ones.  *close set when a tested hit's chi2 is within 1e-3
 * relative of the cut. */
typedef struct {
    double chi2;
    long idx;
} hitsel_t;

static int cmp_hitsel(const void* a, const void* b)
{
    const hitsel_t* x = (const hitsel_t*)a;
    const hitsel_t* y = (const hitsel_t*)b;
    if (x->chi2 < y->chi2) return -1;
    if (x->chi2 > y->chi2) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

typedef struct {
    double sin_dphi;   /* sine of the azimuthal half-width (unused when dphi >= pi) */
    double dphi;       /* azimuthal half-width; pi means the whole circle */
    double wv;         /* half-width along z (barrel) / r (disk) */
    double vlo, vhi;   /* bin-enumeration range along the second coordinate */
    int ok;            /* 0: no finite window (no hit is tested) */
} window_t;

static void make_window(const orc_cfg* cfg, const orc_layer* L, const double q[6],
                        const double Pk[21], window_t* W)
{
    double cut = cfg->chi2_cut;
    double pxx = Pk[pidx(0, 0)], pyy = Pk[pidx(1, 1)], pzz = Pk[pidx(2, 2)];
    double rho = hypot(q[0], q[1]);
    double wu = sqrt(cut * (pxx + pyy + L->win_su * L->win_su));
    double t = WIN_REL * wu / rho;
    double dphi = t >= 1.0 ? PI : asin(t) + WIN_ABS;
    if (dphi > 0.5 * PI) dphi = PI;
    W->dphi = dphi;
    W->sin_dphi = dphi >= PI ? 2.0 : sin(dphi);
    if (L->kind == 0) {
        W->wv = WIN_REL * sqrt(cut * (pzz + L->win_sv * L->win_sv)) + WIN_ABS;
        W->vlo = q[2] - W->wv;
        W->vhi = q[2] + W->wv;
    } else {
        W->wv = WIN_REL * sqrt(cut * (pxx + pyy + L->win_sv * L->win_sv)) + WIN_ABS;
        W->vlo = rho * (dphi >= PI ? -1.0 : cos(dphi)) - W->wv;
        W->vhi = rho + W->wv;
    }
    W->ok = dphi >= 0.0 && W->wv >= 0.0 && W->wv < 1e30 && rho > 0.0;
}

/* test one hit: window predicate and chi2 cut */
static int test_hit(const orc_cfg* cfg, const orc_layer* L, const event_index* E, long i,
                    const double q[6], const double Pk[21], const window_t* W, double* chi2,
                    int* close)
{
    double rho = hypot(q[0], q[1]);
    double rh = hypot(E->hx[i], E->hy[i]);
    if (W->dphi < PI) {
        /* |azimuth difference| <= dphi (< pi/2): same half-plane and |sin| bounded */
        double cd = (E->hx[i] * q[0] + E->hy[i] * q[1]) / (rh * rho);
        double sd = (E->hy[i] * q[0] - E->hx[i] * q[1]) / (rh * rho);
        if (!(cd > 0.0) || fabs(sd) > W->sin_dphi) return 0;
    }
    double hit[5] = {E->hx[i], E->hy[i], E->hz[i], E->hsu[i], E->hsv[i]};
    double H[2][6], r[2];
    measurement(q, hit, L->kind, H, r);
    if (fabs(r[1]) > W->wv) return 0;
    double c2 = orc_chi2(q, Pk, hit, L->kind);
    if (fabs(c2 - cfg->chi2_cut) < CLOSE_REL * cfg->chi2_cut) *close = 1;
    if (!(c2 < cfg->chi2_cut)) return 0;
    *chi2 = c2;
    return 1;
}

static int scan_hits(const orc_cfg* cfg, int layer, const event_index* E, int binned,
                     const double q[6], const double Pk[21], hitsel_t** buf, int* cap,
                     int* close)
{
    const orc_layer* L = &cfg->layers[layer];
    window_t W;
    make_window(cfg, L, q, Pk, &W);
    int n = 0;
    if (!W.ok) return 0;
#define ACCEPT(I)                                                           \
    do {                                                                    \
        double c2_;                                                         \
        if (test_hit(cfg, L, E, (I), q, Pk, &W, &c2_, close)) {              \
            if (n == *cap) {                                                \
                *cap *= 2;                                                  \
                *buf = (hitsel_t*)realloc(*buf, sizeof(hitsel_t) * *cap);   \
            }                                                               \
            (*buf)[n].chi2 = c2_;                                           \
            (*buf)[n].idx = (I);                                            \
            n++;                                                            \
        }                                                                   \
    } while (0)
    if (!binned) {
        for (long k = E->layer_off[layer]; k < E->layer_off[layer + 1]; ++k) ACCEPT(E->layer_hits[k]);
    } else {
        int np = L->nbin_phi;
        double phi = atan2(q[1], q[0]);
        long b_lo, b_hi;
        if (W.dphi >= PI) {
            b_lo = 0;
            b_hi = np - 1;
        } else {
            b_lo = (long)floor((phi - W.dphi + PI) * np / (2.0 * PI));
            b_hi = (long)floor((phi + W.dphi + PI) * np / (2.0 * PI));
            if (b_hi - b_lo + 1 >= np) {
                b_lo = 0;
                b_hi = np - 1;
            }
        }
        int v_lo = coord_bin(W.vlo, L->lo, L->hi, L->nbin_2);
        int v_hi = coord_bin(W.vhi, L->lo, L->hi, L->nbin_2);
        for (long bb = b_lo; bb <= b_hi; ++bb) {
            int bp = (int)(((bb % np) + np) % np);
            for (int bv = v_lo; bv <= v_hi; ++bv) {
                int b = bp * L->nbin_2 + bv;
                for (long k = E->bin_off[layer][b]; k < E->bin_off[layer][b + 1]; ++k)
                    ACCEPT(E->bin_hits[layer][k]);
            }
        }
    }
#undef ACCEPT
    qsort(*buf, n, sizeof(hitsel_t), cmp_hitsel);
    return n;
}

static int cmp_child(const child_t* a, const child_t* b)
{
    if (a->nhits != b->nhits) return a->nhits > b->nhits ? -1 : 1;
    if (a->chi2_tot != b->chi2_tot) return a->chi2_tot < b->chi2_tot ? -1 : 1;
    if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
    return (a->hit > b->hit) - (a->hit < b->hit);
}

static int cmp_child_q(const void* a, const void* b)
{
    return cmp_child((const child_t*)a, (const child_t*)b);
}

static int near_tie(double a, double b)
{
    double m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
    if (m < 1.0) m = 1.0;
    return fabs(a - b) <= CLOSE_REL * m;
}

typedef struct {
    const orc_cfg* cfg;
    const event_index* E;
    long lo, hi;
    const int* seed_hits;
    int binned;
    int* out_hits;
    double *out_par, *out_cov, *out_chi2;
    int *out_ndf, *out_status, *out_tie, *out_visit;
    long counters[2];
} find_job;

static void find_seed(find_job* J, long sd)
{
    const orc_cfg* cfg = J->cfg;
    const event_index* E = J->E;
    int nl = cfg->n_layers;
    int mc = cfg->max_cands;
    int cap_c = mc > 0 ? mc : 1;
    cand_t* cands = (cand_t*)malloc(sizeof(cand_t) * cap_c);
    cand_t* next = (cand_t*)malloc(sizeof(cand_t) * cap_c);
    int cap_ch = 64, cap_h = 64;
    child_t* ch = (child_t*)malloc(sizeof(child_t) * cap_ch);
    hitsel_t* hs = (hitsel_t*)malloc(sizeof(hitsel_t) * cap_h);
    double (*pred_p)[6] = malloc(sizeof(double) * 6 * cap_c);
    double (*pred_P)[21] = malloc(sizeof(double) * 21 * cap_c);
    int* pred_layer = (int*)malloc(sizeof(int) * cap_c);
    int tie = -1;

    /* seed: 3-hit circle, then the KF over the three seed hits */
    const int* sh = J->seed_hits + 3 * sd;
    cand_t* c0 = &cands[0];
    memset(c0, 0, sizeof(cand_t));
    for (int l = 0; l < nl; ++l) c0->hits[l] = -1;
    for (int l = 0; l < nl; ++l) c0->visit[l] = -1;
    double a[3] = {E->hx[sh[0]], E->hy[sh[0]], E->hz[sh[0]]};
    double b[3] = {E->hx[sh[1]], E->hy[sh[1]], E->hz[sh[1]]};
    double c[3] = {E->hx[sh[2]], E->hy[sh[2]], E->hz[sh[2]]};
    orc_seed(a, b, c, cfg->bz, c0->p, c0->P);
    for (int k = 0; k < 3 && !c0->status; ++k) {
        long hi = sh[k];
        int layer = E->hlayer[hi];
        double q[6], Q[21], c2;
        c0->status |= orc_propagate(cfg, layer, c0->p, c0->P, q, Q, NULL, NULL, cfg->use_material);
        if (c0->status) break;
        double hit[5] = {E->hx[hi], E->hy[hi], E->hz[hi], E->hsu[hi], E->hsv[hi]};
        c0->status |= orc_update(q, Q, hit, cfg->layers[layer].kind, c0->p, c0->P, &c2);
        c0->chi2 += c2;
        c0->nhits++;
        c0->hits[layer] = (int)hi;
    }
    c0->done = c0->status != 0;
    /* steering: the seed's region, and the plan entry after its last seed layer */
    const orc_region* R = NULL;
    c0->pos = 0;
    if (cfg->n_regions > 0 && !c0->done) {
        int close0 = 0;
        int g = seed_region(cfg, c0->p, &close0);
        if (close0) tie = 0;
        int start = -1;
        if (g >= 0) {
            R = &cfg->regions[g];
            for (int k = 0; k < 3; ++k)
                for (int q = 0; q < R->n; ++q)
                    if (R->layers[q] == E->hlayer[sh[k]] && q + 1 > start) start = q + 1;
        }
        if (start < 0) {
            c0->status |= ORC_ST_UNREACHABLE;
            c0->done = 1;
        } else {
            c0->pos = start;
        }
    }
    int nc = 1;

    for (int step = 0; step < nl; ++step) {
        int any = 0;
        for (int k = 0; k < nc; ++k) any |= !cands[k].done;
        if (!any) break;
        int close = 0, nch = 0;
        for (int k = 0; k < nc; ++k) {
            cand_t* cd = &cands[k];
            if (nch + cap_c + 2 > cap_ch) {
                cap_ch = 2 * (nch + cap_c + 2);
                ch = (child_t*)realloc(ch, sizeof(child_t) * cap_ch);
            }
            pred_layer[k] = -1;
            if (!cd->done) {
                int st = 0;
                int layer = R ? steer(cfg, R, &cd->pos, cd->p, &st, &close)
                              : navigate(cfg, cd->p, &st, &close);
                if (layer < 0) {
                    cd->done = 1;
                    cd->status |= st;
                } else {
                    J->counters[0]++;
                    st = orc_propagate(cfg, layer, cd->p, cd->P, pred_p[k], pred_P[k], NULL, NULL,
                                       cfg->use_material);
                    if (st) {
                        cd->done = 1;
                        cd->status |= st;
                    } else {
                        pred_layer[k] = layer;
                    }
                }
            }
            if (pred_layer[k] < 0) {
                child_t x = {k, NO_HIT, 0.0, cd->chi2, cd->nhits};
                ch[nch++] = x;
                continue;
            }
            int nh = scan_hits(cfg, pred_layer[k], E, J->binned, pred_p[k], pred_P[k], &hs, &cap_h,
                               &close);
            int keep = nh < mc ? nh : mc;
            if (nh > mc && near_tie(hs[mc - 1].chi2, hs[mc].chi2)) close = 1;
            if (nch + keep + 1 > cap_ch) {
                cap_ch = 2 * (nch + keep + 1);
                ch = (child_t*)realloc(ch, sizeof(child_t) * cap_ch);
            }
            for (int j = 0; j < keep; ++j) {
                child_t x = {k, (int)hs[j].idx, hs[j].chi2, cd->chi2 + hs[j].chi2, cd->nhits + 1};
                ch[nch++] = x;
            }
            child_t x = {k, NO_HIT, 0.0, cd->chi2, cd->nhits};
            ch[nch++] = x;
        }
        qsort(ch, nch, sizeof(child_t), cmp_child_q);
        int nk = nch < mc ? nch : mc;
        /* only the kept/dropped boundary changes which candidates survive */
        if (nch > nk && ch[nk - 1].nhits == ch[nk].nhits &&
            near_tie(ch[nk - 1].chi2_tot, ch[nk].chi2_tot))
            close = 1;
        if (close && tie < 0) tie = step;
        for (int j = 0; j < nk; ++j) {
            const child_t* x = &ch[j];
            const cand_t* par = &cands[x->parent];
            cand_t* nx = &next[j];
            *nx = *par;
            int layer = pred_layer[x->parent];
            if (layer < 0) continue;              /* frozen: carried unchanged */
            nx->visit[layer] = step;
            if (x->hit != NO_HIT) {
                double hit[5] = {E->hx[x->hit], E->hy[x->hit], E->hz[x->hit], E->hsu[x->hit],
                                 E->hsv[x->hit]};
                double c2;
                int st = orc_update(pred_p[x->parent], pred_P[x->parent], hit,
                                    cfg->layers[layer].kind, nx->p, nx->P, &c2);
                J->counters[1]++;
                nx->status |= st;
                if (st) nx->done = 1;
                nx->chi2 = x->chi2_tot;
                nx->nhits = x->nhits;
                nx->misses = 0;
                nx->hits[layer] = x->hit;
            } else {
                memcpy(nx->p, pred_p[x->parent], sizeof(nx->p));
                memcpy(nx->P, pred_P[x->parent], sizeof(nx->P));
                nx->misses = par->misses + 1;
                if (nx->misses > cfg->max_miss) nx->done = 1;
            }
        }
        cand_t* t = cands;
        cands = next;
        next = t;
        nc = nk;
    }
    /* the final choice between the two best candidates */
    if (nc > 1 && cands[0].nhits == cands[1].nhits && near_tie(cands[0].chi2, cands[1].chi2) &&
        tie < 0)
        tie = nl;
    const cand_t* best = &cands[0];
    for (int l = 0; l < nl; ++l) J->out_hits[sd * nl + l] = best->hits[l];
    if (J->out_visit)
        for (int l = 0; l < nl; ++l) J->out_visit[sd * nl + l] = best->visit[l];
    memcpy(J->out_par + 6 * sd, best->p, sizeof(best->p));
    memcpy(J->out_cov + 21 * sd, best->P, sizeof(best->P));
    J->out_chi2[sd] = best->chi2;
    J->out_ndf[sd] = 2 * best->nhits - 5;
    J->out_status[sd] = best->status;
    J->out_tie[sd] = tie;
    free(cands);
    free(next);
    free(ch);
    free(hs);
    free(pred_p);
    free(pred_P);
    free(pred_layer);
}

static void* find_worker(void* arg)
{
    find_job* J = (find_job*)arg;
    for (long s = J->lo; s < J->hi; ++s) find_seed(J, s);
    return NULL;
}

void orc_find(const orc_cfg* cfg, long n_hits,
              const double* hx, const double* hy, const double* hz,
              const double* hsu, const double* hsv, const int* hlayer,
              long n_seeds, const int* seed_hits, int binned,
              int* out_hits, double* out_par, double* out_cov, double* out_chi2,
              int* out_ndf, int* out_status, int* out_tie_step, int* out_visit, long* counters,
              int n_threads)
{
    event_index E;
    memset(&E, 0, sizeof(E));
    E.n_hits = n_hits;
    E.hx = hx; E.hy = hy; E.hz = hz; E.hsu = hsu; E.hsv = hsv; E.hlayer = hlayer;
    build_index(cfg, &E);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    find_job* jobs = (find_job*)calloc(n_threads, sizeof(find_job));
    pthread_t th[256];
    for (int i = 0; i < n_threads; ++i) {
        find_job J = {cfg, &E, n_seeds * i / n_threads, n_seeds * (i + 1) / n_threads,
                      seed_hits, binned, out_hits, out_par, out_cov, out_chi2, out_ndf,
                      out_status, out_tie_step, out_visit, {0, 0}};
        jobs[i] = J;
    }
    if (n_threads == 1) find_worker(&jobs[0]);
    else {
        for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, find_worker, &jobs[i]);
        for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    }
    counters[0] = counters[1] = 0;
    for (int i = 0; i < n_threads; ++i) {
        counters[0] += jobs[i].counters[0];
        counters[1] += jobs[i].counters[1];
    }
    free(jobs);
    free_index(cfg, &E);
}

/* ------------------------------------------------------------------ */
/* Seed cleaning (paper Sec. 3.2: before finding, seeds that probably come
 * from the same particle are removed, judged by shared hits and by the
 * seeds' pT, eta and phi; the paper leaves the rule open).  Reading taken:
 *   two seeds of the same event are duplicates if they share a hit, or if
 *   |d eta| < deta, |d phi| (modulo 2 pi) < dphi and |d c| < dc all hold;
 *   seed i is better than seed j if (float) chi2_i < (float) chi2_j, equal
 *   chi2 going to the lower index;
 *   a seed is removed iff some better seed is its duplicate (whether or not
 *   that seed is itself removed: the order-free form, so every seed is
 *   decided independently of the others' fate).
 * Only seeds with status 0 take part; the others are kept (keep = 1) and
 * neither remove nor are removed.  tie[j] = 1 marks a seed in a pair whose
 * decision lies within the bands stated below of a threshold or of a chi2
 * equality. */
static double seed_eta(double th) { return -log(tan(0.5 * th)); }

void orc_clean_seeds(long n, const double* par, const double* chi2, const int* status,
                     const int* event, const int* hits, double deta, double dphi, double dc,
                     int* keep, int* tie)
{
    /* group seed indices by event (counting sort; events are small ints) */
    int ev_max = -1;
    for (long i = 0; i < n; ++i) if (event[i] > ev_max) ev_max = event[i];
    long* cnt = (long*)calloc((size_t)ev_max + 2, sizeof(long));
    long* idx = (long*)malloc((size_t)(n > 0 ? n : 1) * sizeof(long));
    for (long i = 0; i < n; ++i) cnt[event[i] + 1]++;
    for (int e = 0; e <= ev_max; ++e) cnt[e + 1] += cnt[e];
    long* fill = (long*)calloc((size_t)ev_max + 1, sizeof(long));
    for (long i = 0; i < n; ++i) idx[cnt[event[i]] + fill[event[i]]++] = i;
    for (long i = 0; i < n; ++i) {
        keep[i] = 1;
        tie[i] = 0;
    }
    for (int e = 0; e <= ev_max; ++e) {
        for (long a = cnt[e]; a < cnt[e + 1]; ++a) {
            long j = idx[a];
            if (status[j] != 0) continue;
            float fj = (float)chi2[j];
            for (long b = cnt[e]; b < cnt[e + 1]; ++b) {
                long i = idx[b];
                if (i == j || status[i] != 0) continue;
                int share = 0;
                for (int u = 0; u < 3; ++u)
                    for (int v = 0; v < 3; ++v)
                        if (hits[3 * i + u] >= 0 && hits[3 * i + u] == hits[3 * j + v]) share = 1;
                double de = fabs(seed_eta(par[6 * i + 5]) - seed_eta(par[6 * j + 5]));
                double dp = fabs(wrap_pi(par[6 * i + 4] - par[6 * j + 4]));
                double dq = fabs(par[6 * i + 3] - par[6 * j + 3]);
                int close = de < deta && dp < dphi && dq < dc;
                int dup = share || close;
                float fi = (float)chi2[i];
                int better = fi < fj || (fi == fj && i < j);
                if (dup && better) keep[j] = 0;
                /* near-threshold decisions: within 1e-3 of a threshold, the band
                 * for q/pT also 1e-3 of |q/pT| and the one for chi2 2e-3 of
                 * max(chi2, 1) (ten times the parity bars of a seed fit's
                 * parameters and twice that of its chi2, so that a fit of the
                 * same seed within those bars cannot flip an unmarked decision) */
                if (!share) {
                    const double t = 1e-3;
                    double bq = t * dc;
                    double cm = fmax(fabs(par[6 * i + 3]), fabs(par[6 * j + 3]));
                    if (t * cm > bq) bq = t * cm;
                    int all_in = de < deta * (1 + t) && dp < dphi * (1 + t) && dq < dc + bq;
                    int any_edge = fabs(de - deta) <= t * deta || fabs(dp - dphi) <= t * dphi ||
                                   fabs(dq - dc) <= bq;
                    if (all_in && any_edge) tie[i] = tie[j] = 1;
                }
                if (dup && fabs((double)fi - (double)fj) <= 2e-3 * fmax(1.0, fmax(fabs(fi), fabs(fj))))
                    tie[i] = tie[j] = 1;
            }
        }
    }
    free(cnt);
    free(fill);
    free(idx);
}

/* ------------------------------------------------------------------ */
/* Duplicate removal of found tracks (the paper's Sec. 4 names removing
 * duplicate tracks from several seeds of one particle as the cleaning of the
 * final collection; it gives no rule).  Reading taken: two found tracks of
 * one event are duplicates if the hits they share number at least
 * frac * min(n_i, n_j), n = hits in a track's list; track i is better than
 * track j by (more hits, lower chi2 compared in float, lower index); a track
 * is removed iff a better duplicate exists.  Tracks with status != 0 take no
 * part.  hits [n][nl] (-1 none). */
void orc_dedup(long n, int nl, const int* hits, const double* chi2, const int* status,
               const int* event, double frac, int* keep)
{
    /* hit -> tracks using it, so that only pairs sharing a hit are counted */
    long hmax = -1;
    for (long i = 0; i < n * nl; ++i) if (hits[i] > hmax) hmax = hits[i];
    long* off = (long*)calloc((size_t)(hmax + 2), sizeof(long));
    for (long i = 0; i < n * nl; ++i) if (hits[i] >= 0) off[hits[i] + 1]++;
    for (long h = 0; h <= hmax; ++h) off[h + 1] += off[h];
    long* fill = (long*)calloc((size_t)(hmax + 1 > 0 ? hmax + 1 : 1), sizeof(long));
    long* users = (long*)malloc((size_t)(off[hmax + 1] > 0 ? off[hmax + 1] : 1) * sizeof(long));
    int* nh = (int*)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
    for (long i = 0; i < n; ++i)
        for (int l = 0; l < nl; ++l) {
            int h = hits[i * nl + l];
            if (h < 0) continue;
            nh[i]++;
            users[off[h] + fill[h]++] = i;
        }
    long* part = (long*)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    int* cnt = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (long j = 0; j < n; ++j) {
        keep[j] = 1;
        if (status[j] != 0) continue;
        /* shared-hit counts with every track meeting j in some hit */
        long np = 0;
        for (int l = 0; l < nl; ++l) {
            int h = hits[j * nl + l];
            if (h < 0) continue;
            for (long u = off[h]; u < off[h + 1]; ++u) {
                long i = users[u];
                if (i == j) continue;
                long q = 0;
                while (q < np && part[q] != i) ++q;
                if (q == np) {
                    part[np] = i;
                    cnt[np++] = 0;
                }
                cnt[q]++;
            }
        }
        for (long q = 0; q < np; ++q) {
            long i = part[q];
            if (status[i] != 0 || event[i] != event[j]) continue;
            int mn = nh[i] < nh[j] ? nh[i] : nh[j];
            if (mn == 0 || !(cnt[q] >= frac * mn)) continue;
            float fi = (float)chi2[i], fj = (float)chi2[j];
            int better = nh[i] > nh[j] || (nh[i] == nh[j] && (fi < fj || (fi == fj && i < j)));
            if (better) {
                keep[j] = 0;
                break;
            }
        }
    }
    free(off);
    free(fill);
    free(users);
    free(nh);
    free(part);
    free(cnt);
}
