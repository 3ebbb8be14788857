/*
 * FP64 reference implementation of the Kalman-filter track fit and
 * combinatorial track finding (test infrastructure only: it is used by the
 * tests, by smoke() and by the CPU-baseline leg of the benchmark, never by
 * the product path).
 *
 * Method (the paper's parallelised KF tracking, Sec. 2, built on the
 * traditional Kalman filter it cites in Sec. 1):
 *   - state p = (x, y, z, c = q/pT, phi, theta) at a point on the track,
 *     6x6 covariance, units cm / GeV / T / rad;
 *   - helix transport in a uniform field along +z, propagate to the next
 *     detector layer (barrel radius by Newton iteration, disk z in closed
 *     form), transport Jacobian including the derivative of the path
 *     length, multiple-scattering process noise from the layer material
 *     (geometry section: material constants per layer);
 *   - 2D hit measurement in the hit's local frame, chi2, gain, Joseph-form
 *     covariance update;
 *   - layer-by-layer combinatorial finding with a chi2 cut, a bounded
 *     number of candidates per seed and a score (the paper's list of items
 *     under optimisation: hit-search windows, candidate scoring).
 * Every number is double.  Covariances cross this interface packed as the
 * upper triangle, idx(i<=j) = i*(11-i)/2 + j, 21 entries.
 */
#ifndef KF_ORACLE_H
#define KF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_ST_OK = 0,
    ORC_ST_UNREACHABLE = 1,
    ORC_ST_NOCONV = 2,
    ORC_ST_NONPD = 8,
    ORC_ST_NAN = 16,
    ORC_ST_DONE = 32
};

typedef struct {
    int kind;          /* 0 barrel, 1 disk */
    double r_or_z;     /* barrel radius or disk z */
    double lo, hi;     /* barrel z extent / disk r extent */
    double x0;         /* thickness in radiation lengths */
    int nbin_phi, nbin_2;
    double win_su, win_sv;
} orc_layer;

/* A tracking region and its layer plan (Sec. 3.1 steering): seeds with eta
 * in [eta_lo, eta_hi) follow `layers` in this order. */
typedef struct {
    double eta_lo, eta_hi;
    int n;
    int layers[64];
} orc_region;

typedef struct {
    int n_layers;
    const orc_layer* layers;
    double bz;          /* Tesla */
    double chi2_cut;    /* hit acceptance */
    int max_cands;      /* candidates kept per seed */
    int max_newton;     /* Newton iteration limit */
    double newton_tol;  /* cm */
    double mass;        /* GeV, for beta in the scattering formula */
    int max_miss;       /* consecutive missed layers allowed */
    int use_material;   /* add process noise */
    double field_z0;    /* > 0: parametrised field (see orc_field), Bz = bz / (1 + (z/field_z0)^2) */
    double field_step;  /* largest integration step in the parametrised field [cm] */
    /* optional r-z material map (mat_x0 NULL: the layers' own x0, no energy
     * loss): cell (ir, iz) with ir = floor(r / (mat_rmax / mat_nr)) and
     * iz = floor((z - mat_zmin) / ((mat_zmax - mat_zmin) / mat_nz)), clamped;
     * x0 = radiation-length fraction, xi = areal density [g/cm^2] for the
     * ionisation loss, both at normal incidence, arrays [mat_nr][mat_nz] */
    int mat_nr, mat_nz;
    double mat_rmax, mat_zmin, mat_zmax;
    const double* mat_x0;
    const double* mat_xi;
    /* optional steering (n_regions 0: dynamic navigation) */
    int n_regions;
    const orc_region* regions;
} orc_cfg;

/* helix transport by transverse arc length s */
void orc_helix(const double p[6], double s, double bz, double out[6]);
/* parametrised field at x[3] (cm): B[3] in T (Bx, By, Bz) */
void orc_field(const orc_cfg* cfg, const double x[3], double B[3]);
/* state after 3D path length l through the parametrised field (RK4) */
void orc_rk_path(const orc_cfg* cfg, const double p[6], double l, double out[6]);

/* propagate state+cov to layer `layer`; returns status bits.
 * s_out / iters_out may be NULL. add_noise: add scattering noise of the layer. */
int orc_propagate(const orc_cfg* cfg, int layer, const double p[6], const double Pk[21],
                  double p_out[6], double P_out[21], double* s_out, int* iters_out,
                  int add_noise);

/* Newton solve only (for iteration statistics); s_init < 0 means the
 * straight-line start.  Returns status; writes s and iteration count. */
int orc_solve_barrel(const orc_cfg* cfg, const double p[6], double r_l, double s_init,
                     double* s_out, int* iters_out);

/* transport Jacobian F (row-major 6x6) of the propagation to `layer` */
int orc_jacobian(const orc_cfg* cfg, int layer, const double p[6], double F[36]);

/* one KF update with hit (x,y,z,su,sv) on a layer of kind `kind` */
int orc_update(const double p[6], const double Pk[21], const double hit[5], int kind,
               double p_out[6], double P_out[21], double* chi2_out);

/* chi2 of a hit against a predicted state (no update) */
double orc_chi2(const double p[6], const double Pk[21], const double hit[5], int kind);

/* seed state and prior from three hits (x,y,z each) */
void orc_seed(const double h1[3], const double h2[3], const double h3[3], double bz,
              double p_out[6], double P_out[21]);

/* Track fit.  n tracks; steps described by layer_seq / hit_idx, row-major
 * [n][max_steps] (layer -1 ends the track, hit -1 = no hit at that layer).
 * par_io [n][6] / cov_io [n][21]: in = starting state, out = fitted. */
void orc_fit(const orc_cfg* cfg, long n, int max_steps,
             const double* hx, const double* hy, const double* hz,
             const double* hsu, const double* hsv,
             const int* layer_seq, const int* hit_idx,
             double* par_io, double* cov_io, double* chi2_out, int* ndf_out,
             int* status_out, int n_threads);

/* Combinatorial finding in one event.
 *   hits: n_hits arrays + layer id.
 *   seeds: seed_hits [n_seeds][3] (indices into the event's hits).
 *   binned: 1 = phi/(z|r) binned window search, 0 = test every hit of the layer.
 *   outputs per seed: out_hits [n_seeds][n_layers] (-1 none), par/cov/chi2/ndf/status
 *   of the best candidate, tie_step (first step with a decision closer than
 *   1e-3 relative to its threshold, -1 if none).
 *   counters[0] = propagations (KF steps), counters[1] = updates. */
void orc_find(const orc_cfg* cfg, long n_hits,
              const double* hx, const double* hy, const double* hz,
              const double* hsu, const double* hsv, const int* hlayer,
              long n_seeds, const int* seed_hits, int binned,
              int* out_hits, double* out_par, double* out_cov, double* out_chi2,
              int* out_ndf, int* out_status, int* out_tie_step, int* out_visit,
              long* counters, int n_threads);

/* Mean ionisation loss (Bethe, no density effect) in silicon [MeV cm^2/g]
 * of a particle of momentum p and mass m [GeV]. */
double orc_dedx(double p, double m);

/* Material effects at a crossing of `layer` by state q (in place): the
 * scattering noise and the mean energy loss, as in propagation. */
void orc_material(const orc_cfg* cfg, int layer, double q[6], double Pk[21]);

/* Seed cleaning within each event (see kf_oracle.c).  par [n][6], chi2 [n],
 * status [n] (only 0 takes part), event [n], hits [n][3] (-1 none).
 * keep [n] = 1 kept, 0 removed; tie [n] = 1 near a threshold. */
void orc_clean_seeds(long n, const double* par, const double* chi2, const int* status,
                     const int* event, const int* hits, double deta, double dphi, double dc,
                     int* keep, int* tie);

/* Duplicate removal of found tracks (see kf_oracle.c): keep [n] = 1 kept. */
void orc_dedup(long n, int nl, const int* hits, const double* chi2, const int* status,
               const int* event, double frac, int* keep);

#ifdef __cplusplus
}
#endif
#endif
