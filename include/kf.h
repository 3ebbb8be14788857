/*
 * kf.h - C ABI of libkfmi.so, the MI355X (gfx950) Kalman-filter track fit and
 * combinatorial track finding library.
 *
 * Method: the parallelised Kalman-filter tracking of arXiv:1906.02253
 * (Sec. 2: vectorised KF fit and KF-based finding over many small matrices at
 * once; Sec. 3.1: geometry as a vector of per-layer descriptions, layer-to-
 * layer propagation, material per layer, constant field; Sec. 3.2: hits and
 * seeds provided by the caller, found tracks handed back; Sec. 4: chi2-based
 * hit selection inside search windows, candidate scoring).
 *
 * Conventions shared by every entry point
 *   Units: cm, GeV, Tesla, radians.  Field along +z.
 *   State p = (x, y, z, c = q/pT, phi, theta) at a point on the track.
 *   Covariance: symmetric 6x6 stored as the packed upper triangle,
 *   index(i <= j) = i*(11-i)/2 + j, 21 entries.
 *   Track arrays are structure-of-arrays with leading dimension ld (elements):
 *   element k of track i is at [k*ld + i]; ld is a multiple of 64 and >= n.
 *   All array pointers are DEVICE pointers unless marked "host".  The caller
 *   owns every array; the library never frees caller memory.  A context owns
 *   its device workspace (allocated on first use of a given size, reused).
 *   Calls are asynchronous on `stream` (a hipStream_t passed as void*, NULL =
 *   the null stream); the caller synchronises before reading results.
 *   Return value: KF_OK, or a negative kf_status for invalid arguments or a
 *   HIP error (see kf_last_error).  Numerical trouble is never an error: it is
 *   reported per track in `status` bits and the track is frozen from there on
 *   (KF_ST_FALLBACK excepted, which only informs).
 *   A context must not be used from two host threads at once.
 */
#ifndef KFMI_KF_H
#define KFMI_KF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kf_ctx kf_ctx;

enum kf_status {
    KF_OK = 0,
    KF_EINVAL = -1,        /* bad argument */
    KF_EHIP = -2,          /* HIP runtime error (launch, copy, allocation) */
    KF_ENOMEM = -3,        /* workspace allocation failed */
    KF_EUNSUPPORTED = -4   /* valid but not supported by this library */
};

/* per-track status bits */
enum {
    KF_ST_OK = 0,
    KF_ST_UNREACHABLE = 1, /* target surface not reachable (looper / behind) */
    KF_ST_NOCONV = 2,      /* propagate-to-radius did not converge */
    KF_ST_FALLBACK = 4,    /* informational, does not freeze the track: the learned
                              initial guess did not converge within mlp_max_iter
                              evaluations and the straight-line start was used */
    KF_ST_NONPD = 8,       /* innovation matrix not positive definite */
    KF_ST_NAN = 16,        /* non-finite state */
    KF_ST_BADINPUT = 32,   /* out-of-range layer or hit index in the caller's arrays */
    KF_ST_DUPLICATE = 64,  /* seed removed by seed cleaning (kf_clean_seeds, KF_CLEAN_SEEDS) */
    KF_ST_DUPTRACK = 128   /* found track removed as a duplicate (kf_remove_duplicates,
                              KF_REMOVE_DUPLICATES) */
};

/* flags */
enum {
    KF_PREC_MIXED = 0,     /* FP32 storage of state and covariance; surface solves, helix,
                              transport Jacobian, navigation and search windows FP32; F P F^T,
                              the process noise and the update (S, S^-1, gain, Joseph) FP64,
                              with the state held in FP64 between its FP32 loads and stores */
    KF_PREC_FP32 = 1,      /* everything FP32 (Joseph form kept) */
    KF_PREC_FP64 = 2,      /* everything FP64 */
    KF_PREC_MASK = 3,
    KF_INIT_MLP = 4,       /* start propagate-to-radius from the learned path-length guess
                              (needs kf_mlp_load; kf_find needs a width >= 64) */
    KF_NO_MATERIAL = 8,    /* ignore the layers' material (no process noise) */
    KF_PER_LAYER = 16,     /* kf_fit: one launch per step, state through HBM between steps */
    KF_CLEAN_SEEDS = 32,   /* kf_find, kf_find_batched: seed cleaning (kf_clean_seeds) after
                              the seed order, before the finding kernel */
    KF_REMOVE_DUPLICATES = 64  /* kf_find, kf_find_batched: duplicate removal of the found
                                  tracks (kf_remove_duplicates) after the finding kernel */
};

/* One detector layer (paper Sec. 3.1, the per-layer geometry record). */
typedef struct {
    int32_t kind;          /* 0 = barrel cylinder, 1 = disk */
    int32_t nbin_phi;      /* hit bins in phi over [-pi, pi) */
    int32_t nbin_2;        /* hit bins in z (barrel) / r (disk) over [lo, hi];
                              nbin_phi * nbin_2 <= 16384 */
    int32_t reserved;      /* 0 */
    double r_or_z;         /* barrel radius / disk z */
    double lo, hi;         /* barrel: z extent [lo, hi]; disk: radial extent */
    double x0;             /* material thickness in radiation lengths */
    double win_su, win_sv; /* largest hit sigma (u, v) on the layer, sizes the search window */
} kf_layer;

typedef struct {
    double bz;             /* field [T] */
    double chi2_cut;       /* hit acceptance chi2 (2 dof) */
    double newton_tol;     /* |r - r_layer| convergence threshold [cm] */
    double mass;           /* particle mass for the scattering width [GeV] */
    int32_t max_cands;     /* candidates kept per seed, 1..8 */
    int32_t max_newton;    /* propagate-to-radius iteration limit */
    int32_t max_miss;      /* consecutive missed layers allowed */
    int32_t mlp_max_iter;  /* iterations allowed from the learned guess before fallback */
    double field_z0;       /* 0: uniform field bz along z.  > 0: parametrised solenoid-like
                              field Bz = bz / (1 + (z/field_z0)^2), Br = -(r/2) dBz/dz, tracks
                              integrated by fourth-order Runge-Kutta (kf_propagate, kf_fit,
                              kf_find; barrels by a Newton iteration on the integrated radius,
                              disks on the integrated z, each over at most 1000 cm of path (a
                              surface further along the track is UNREACHABLE); the covariance by
                              the helix Jacobian in the path's mean effective axial field
                              Bz - cot(theta) B_T.t_T; in finding, steering and the learned start
                              work as in the uniform field, their surfaces reached by these solves
                              along the 3D path) */
    double field_step;     /* largest Runge-Kutta step [cm] in the parametrised field (> 0) */
    double clean_deta;     /* seed cleaning: |d eta| below which two seeds may be duplicates,
                              0 .. 0.09375 (the width of a seed cell in eta) */
    double clean_dphi;     /* seed cleaning: |d phi| [rad], 0 .. 2 pi / 64 (a seed cell in phi) */
    double clean_dc;       /* seed cleaning: |d (q/pT)| [1/GeV], >= 0 */
    double dup_frac;       /* duplicate removal: shared fraction of the shorter track's hits,
                              0 < dup_frac <= 1 */
} kf_params;

/* Track states, SoA with leading dimension ld.  par [6][ld], cov [21][ld]
 * and chi2 [ld] are float (double with KF_PREC_FP64).  ndf = 2*hits - 5. */
typedef struct {
    int64_t n, ld;
    void* par;
    void* cov;
    void* chi2;
    int32_t* ndf;
    uint32_t* status;
} kf_tracks;

/* Hits, SoA float32 (paper Sec. 3.2: provided externally). */
typedef struct {
    int64_t n;
    const float *x, *y, *z;   /* global position */
    const float *su, *sv;     /* sigma along r*phi and along z (barrel) / r (disk) */
    const int32_t* layer;     /* layer index of each hit */
} kf_hits;

/* r-z material map (paper Sec. 3.1: scattering and energy loss from
 * two-dimensional material arrays indexed in r-z).  Cell (ir, iz) with
 * ir = floor(r / (r_max / nr)) and iz = floor((z - z_min) / ((z_max - z_min) /
 * nz)), clamped to the grid, holds the radiation-length fraction x0 and the
 * areal density xi [g/cm^2] of the surface crossing it, both at normal
 * incidence.  Host arrays [nr][nz] float, copied. */
typedef struct {
    int32_t nr, nz;        /* 1 <= nr, nz; nr * nz <= 2^22 */
    double r_max;          /* > 0 [cm] */
    double z_min, z_max;   /* z_min < z_max [cm] */
    const float* x0;       /* [nr][nz] >= 0 */
    const float* xi;       /* [nr][nz] >= 0 */
} kf_material;

/* Create a context.  layers: host array of n_layers (<= 64) records, copied.
 * params: host, copied; NULL = defaults (3.8 T uniform, chi2 30, 6
 * candidates, 10 Newton iterations, 1e-4 cm, pion mass, 2 misses, 3 learned
 * iterations, Runge-Kutta step 2 cm, seed cleaning 0.01 / 0.01 rad / 0.05
 * 1/GeV, duplicate fraction 0.5). */
int kf_create(kf_ctx** ctx, const kf_layer* layers, int32_t n_layers, const kf_params* params);
void kf_destroy(kf_ctx* ctx);
/* Text of the last error on this context (valid until the next call). */
const char* kf_last_error(const kf_ctx* ctx);
/* Library-wide last error for failures without a context (kf_create). */
const char* kf_last_error_global(void);

/* Tracking regions with layer plans (paper Sec. 3.1: regions in eta with
 * steering parameters that list the layers finding traverses; the finder
 * follows them without knowing the detector's structure). */
#define KF_MAX_REGIONS 8
typedef struct {
    double eta_lo, eta_hi;   /* seeds with eta = -ln tan(theta/2) in [eta_lo, eta_hi) */
    int32_t n_layers;        /* plan length, 1..64 */
    int32_t layers[64];      /* layer indices in traversal order, each at most once */
} kf_region;

/* Sets (n_regions >= 1) or removes (regions NULL or n_regions 0) steering
 * for kf_find / kf_find_batched.  With steering a seed takes the first
 * region containing its eta (none: KF_ST_UNREACHABLE, not searched); its
 * search starts after the last plan entry that is one of its seed hits'
 * layers (none: KF_ST_UNREACHABLE); at each step a candidate takes, from its
 * plan position on, the first layer it actually reaches - a barrel outside
 * rho + 0.05 cm crossed outward within half a turn inside |z| <= hi, or a
 * disk ahead (|dz| > 0.05 cm) crossed within half a turn inside its radial
 * extent - passing over entries it does not reach.  Without steering the
 * next surface is found dynamically (the first reached of the next barrel
 * outward and the next disk ahead).  Steering excludes KF_INIT_MLP; in the
 * parametrised field the plan's surfaces are reached by the Runge-Kutta radius
 * and z solves along the 3D path (half a turn at the start point's curvature).
 * Synchronous; do not call while work that uses the context is in flight. */
int kf_set_steering(kf_ctx* ctx, const kf_region* regions, int32_t n_regions);

/* Sets (map != NULL) or removes (NULL) the context's r-z material map.  With
 * a map, the material at each layer crossing (unless KF_NO_MATERIAL) comes
 * from the map's cell at the crossing point instead of the layer's x0: the
 * Highland scattering noise of x0 / cos(alpha), then the mean ionisation
 * loss (Bethe formula with the maximum energy transfer, no density effect,
 * silicon Z/A = 0.49848 and I = 173 eV, the context's mass) over
 * xi / cos(alpha): |p| drops to p' with E' = E - dE (dE capped at half the
 * kinetic energy), the direction is kept, c' = c p / p', and the covariance
 * row and column of c are scaled by dc'/dc = (p/p')^3 E'/E.  Synchronous;
 * do not call while work that uses the context is in flight. */
int kf_set_material(kf_ctx* ctx, const kf_material* map);

/* Seed states from three hits per track (paper Sec. 3.2: seeds): circle
 * through the transverse positions, tangent at hit 1, dip from the arc, prior
 * covariance diag(1, 1, 1, 4, 0.01, 0.01).  seed_hits [3][ld] int32 hit
 * indices.  Writes par, cov; chi2 = 0, ndf = -5, status = 0. */
int kf_seed(kf_ctx* ctx, const kf_hits* hits, const int32_t* seed_hits, kf_tracks* out,
            int flags, void* stream);

/* Propagate every track to its target layer (target_layer [ld] int32, -1 =
 * leave unchanged): helix transport, transport Jacobian with the path-length
 * derivative, F P F^T plus the layer's scattering noise (unless
 * KF_NO_MATERIAL).  Optional outputs (NULL to skip): path_len [ld] float
 * transverse arc length, iters [ld] int32 evaluations of r(s). */
int kf_propagate(kf_ctx* ctx, kf_tracks* t, const int32_t* target_layer, float* path_len,
                 int32_t* iters, int flags, void* stream);

/* Kalman fit (paper Sec. 2: KF track fitting).  In: t holds the starting
 * state (e.g. from kf_seed).  Steps: layer_seq [max_steps][ld] (NULL = step k
 * targets layer k; -1 ends the track) and hit_idx [max_steps][ld] (-1 = no
 * hit at that step).  For each step: propagate, add the layer's noise,
 * update with the hit.  Out: fitted state at the last step, chi2, ndf, status. */
int kf_fit(kf_ctx* ctx, kf_tracks* t, const kf_hits* hits, const int32_t* layer_seq,
           const int32_t* hit_idx, int32_t max_steps, int flags, void* stream);

/* Seed cleaning (paper Sec. 3.2: before finding, seeds that probably stem
 * from the same particle are removed using hit identity and the seeds' pT,
 * eta and phi).  Two seeds of one event are duplicates if they share a hit,
 * or if |d eta| < clean_deta, |d phi| < clean_dphi (modulo 2 pi) and
 * |d c| < clean_dc all hold (eta = -ln tan(theta/2), differences in double
 * precision from the stored floats).  A seed is better than another if its
 * chi2 (float) is lower, equal chi2 going to the lower index.  A seed is
 * removed iff some better seed is its duplicate, whether or not that seed is
 * removed itself (every seed is decided independently).
 *   hits        only hits->n is used (seed hit indices outside [0, n) match nothing)
 *   seeds       in: par, chi2, status after the seed fit (KF_PREC_MIXED or
 *               KF_PREC_FP32 storage); out: status gets KF_ST_DUPLICATE set on
 *               removed seeds and cleared on kept ones.  Seeds with any other
 *               freezing bit, or with seed_event outside [0, n_events), take no
 *               part: they are neither removed nor remove others.
 *   seed_event  [n_seeds] int32, seed_hits [3][seeds->ld] int32 global hit
 *               indices (an index belongs to one event, as in kf_find)
 * kf_find skips seeds with KF_ST_DUPLICATE like any frozen seed (their output
 * is the seed state with the seed's own hits).  The result is the same on
 * every call with the same inputs. */
int kf_clean_seeds(kf_ctx* ctx, const kf_hits* hits, int32_t n_events, kf_tracks* seeds,
                   const int32_t* seed_event, const int32_t* seed_hits, int flags, void* stream);

/* Duplicate removal of found tracks (paper Sec. 4: several seeds of one
 * particle give the same track; removing them is the cleaning of the final
 * collection).  Two tracks of one event are duplicates if the hits they
 * share number at least dup_frac * min(n_i, n_j), n = hits in a track's
 * list.  A track is better than another by (more hits, lower chi2 as float,
 * lower index); a track is removed iff a better duplicate exists (each track
 * decided independently).
 *   hits         only hits->n is used (hit indices outside [0, n) are ignored)
 *   tracks       in: chi2, status (KF_PREC_MIXED or KF_PREC_FP32 storage);
 *                out: KF_ST_DUPTRACK set on removed tracks, cleared on kept
 *                ones.  Tracks with any other freezing bit take no part.
 *   track_hits   [tracks->n][n_layers] int32, the hit of each track on each
 *                layer, -1 = none (kf_find's out_hits); a hit index may appear
 *                only in its own layer's column
 *   track_event  [tracks->n] int32 event of each track
 * The result is the same on every call with the same inputs. */
int kf_remove_duplicates(kf_ctx* ctx, const kf_hits* hits, kf_tracks* tracks,
                         const int32_t* track_hits, const int32_t* track_event, int flags,
                         void* stream);

/* Combinatorial track finding over one or many events (paper Sec. 2: KF-based
 * track finding; Sec. 3.1: layer-to-layer propagation following the geometry;
 * Sec. 3.2: seeds grouped close in eta-phi and processed in parallel; Sec. 4:
 * hit-search windows, chi2 selection, candidate scoring).
 *   hits        all events' hits concatenated (float32 SoA + layer id)
 *   event_off   [n_events+1] int32: event e owns hits [event_off[e], event_off[e+1])
 *   seeds       n_seeds states after the seed fit (kf_seed, then kf_fit over the
 *               three seed hits), KF_PREC_MIXED or KF_PREC_FP32 storage
 *   seed_event  [n_seeds] int32 event of each seed
 *   seed_hits   [3][seeds->ld] int32 the seed's hits (copied to the hit list)
 *   out_hits    [n_seeds][n_layers] int32: hit of the best candidate on each
 *               layer (global hit index), -1 = none
 *   out         n_seeds tracks, out->n == seeds->n: best candidate's state at its
 *               last surface, chi2, ndf = 2*hits - 5, status
 *   counters    optional [8] uint64, incremented by (propagations, updates,
 *               chi2 tests, Newton evaluations, disk-crossing tests, learned
 *               guesses evaluated, learned guesses that fell back, candidates
 *               kept from the children of propagated parents)
 * Per layer a candidate is propagated to its next surface (the first reached
 * of the next barrel outward and the next disk ahead; in the parametrised
 * field along the 3D path, by the Runge-Kutta radius and z solves), every hit in the chi2
 * window's bins passing chi2 < chi2_cut becomes a child (best max_cands per
 * parent), plus one no-hit child; per seed the best max_cands children by
 * (most hits, lowest chi2, parent rank, hit index) survive.  A candidate stops
 * after max_miss + 1 consecutive missed layers or when no surface is left.
 * With KF_CLEAN_SEEDS the seeds are cleaned first (kf_clean_seeds; it writes
 * the seeds' status); with KF_REMOVE_DUPLICATES the found tracks are
 * deduplicated last (kf_remove_duplicates on out, out_hits and seed_event).
 * Device scratch comes from the context workspace (grown on demand). */
int kf_find(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
            const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
            int32_t* out_hits, kf_tracks* out, uint64_t* counters, int flags, void* stream);

/* kf_find for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same pass and results as kf_find, with its scratch taken from a
 * static device array of 64 MiB that the library holds on every device it
 * runs on until the process ends (its address looked up once per device by
 * kf_create), instead of the context's workspace.  No allocation, no
 * freeing, no phase timing.  A call whose scratch would exceed 64 MiB
 * (about 88 B per hit, 140 B per seed, the back-pointers of the resident
 * workgroups and 0.4 MB of bins per event at 24 layers of 128 x 32 bins)
 * returns KF_EINVAL with the sizes in kf_last_error.  Every call on one
 * device shares that device's array and leaves its contents behind (each
 * call clears what it needs): calls that overlap on one device - two
 * streams, two contexts or two host threads - race and must not be issued. */
int kf_find_noalloc(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                    const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
                    int32_t* out_hits, kf_tracks* out, uint64_t* counters, int flags, void* stream);

/* The whole finding pass over a batch of events as one captured HIP graph
 * (paper Sec. 3.2: seeds processed in parallel; events of uneven size in one
 * persistent launch): kf_seed of every seed from its three hits, kf_fit over
 * those hits (layers seed_layers [3][seeds->ld] int32), then kf_find as above.
 * seeds is caller-owned scratch for the seed states (n = number of seeds);
 * the other arguments are those of kf_find.  The first call with a given set
 * of pointers, sizes, flags and finding configuration captures the pass into
 * a graph held by the context; later calls with the same set replay it, so
 * the caller must keep those arrays alive and in place between calls (any
 * change captures again).  The graph holds kernels and event records only.
 * Results are identical to kf_seed + kf_fit + kf_find. */
int kf_find_batched(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                    const int32_t* seed_hits, const int32_t* seed_layers, const int32_t* seed_event,
                    kf_tracks* seeds, int32_t* out_hits, kf_tracks* out, uint64_t* counters,
                    int flags, void* stream);

/* Workgroup width of the finding kernel (32, 64, 128 or 256 lanes; a lane per
 * candidate slot, floor(64 / max_cands) seeds per wave) and tile order (0:
 * seeds sorted by event, eta, phi; 1: events largest first (up to 16,384
 * events; more keep their order), then eta, phi).  Either order is cut into
 * eight ranges, one tile queue each, and within a range the seeds go by a
 * cost class of pT and |eta|, costliest first; the costliest (pT < 0.6 GeV,
 * |eta| < 0.5) come in tiles of half the seeds.  Default 64, 0.  Results do
 * not depend on either; speed does. */
int kf_set_find_config(kf_ctx* ctx, int32_t width, int32_t largest_first);
/* The configuration in use (host outputs). */
int kf_get_find_config(kf_ctx* ctx, int32_t* width, int32_t* largest_first);

/* Autotuner: times kf_find on the caller's sample (arguments as kf_find, no
 * counters) for every width in {32, 64, 128, 256} that fits the device's LDS
 * and both tile orders: one untimed call per configuration, then reps rounds
 * over all configurations with every call timed on its own; the fastest call
 * of a configuration is its time, and the fastest configuration is kept in
 * the context (kf_get_find_config reads it).  table: optional host float [8],
 * ms at [2*w + order] for widths 32, 64, 128, 256 (-1 = not run).
 * Synchronises on `stream` after every timed call.
 * out_hits and out hold the results of the last configuration tried. */
int kf_autotune(kf_ctx* ctx, const kf_hits* hits, const int32_t* event_off, int32_t n_events,
                const kf_tracks* seeds, const int32_t* seed_event, const int32_t* seed_hits,
                int32_t* out_hits, kf_tracks* out, int flags, int32_t reps, float* table,
                void* stream);

/* Kernel timing.  kf_set_timing(ctx, n) with 1 <= n <= 256 makes the next n
 * kf_find or kf_find_batched calls record HIP events on their stream at the
 * boundaries of their phases (seed + seed fit, hit binning, seed ordering,
 * finding kernel), one event set per call, with no host synchronisation;
 * n = 0 turns it off.  kf_timings synchronises on the last recorded event and
 * writes the mean milliseconds over the recorded calls: ms[0] seeding and
 * seed fit (0 for kf_find), ms[1] binning, ms[2] seed ordering, ms[3] finding
 * kernel, and ms[4] = number of calls recorded.  Returns KF_EINVAL if none was. */
int kf_set_timing(kf_ctx* ctx, int32_t n);
int kf_timings(kf_ctx* ctx, float ms[5]);


/* ---- Learned initial guess of propagate-to-radius (not in the paper; the
 * solve it starts stays exact).  Network 8 -> 64 (tanh) -> 64 (tanh) -> 1,
 * evaluated on the matrix cores in bf16 with FP32 accumulation; trained on the
 * device with FP32 master weights and Adam.  Parameters, flat FP32, 4801:
 * W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3 (W row-major [out][in]).
 * Inputs (8): rho/100, sin and cos of (phi - atan2(y, x)), h * (target radius,
 * or 100 cm for a disk) with h = -0.00299792458 Bz c (Bz at the start point),
 * target radius or disk z
 * over 100, the straight-line path length s_line to the target over 100, cot
 * theta, z/100.  Output: (transverse path length - s_line) / (h s_line^2); in
 * the parametrised field the transverse path length is the 3D one times sin
 * theta at the start.  With KF_INIT_MLP a barrel solve whose predicted correction
 * exceeds 100 newton_tol starts from s_line + h s_line^2 * output with
 * mlp_max_iter evaluations of r(s), and if those do not converge runs the
 * plain solve (fallback); smaller corrections keep the straight-line start. */

#define KF_MLP_NPARAM 4801
#define KF_MLP_NIN 8

typedef struct {
    double lr;             /* Adam step size (default 1e-3) */
    double beta1, beta2;   /* moment decays (0.9, 0.999) */
    double eps;            /* 1e-8 */
} kf_mlp_train_cfg;

/* Loads the FP32 parameters w (host [4801]) as the master copy, resets the
 * Adam moments and step count, and publishes the bf16 copies.  Synchronous;
 * must not overlap calls that use the network. */
int kf_mlp_load(kf_ctx* ctx, const float* w);
/* Reads the FP32 master parameters into w (host [4801]); synchronises the device. */
int kf_mlp_get(kf_ctx* ctx, float* w);
/* Network inputs for propagating each track of t to target_layer [ld] int32
 * (-1: zeros).  feats [8][t->ld] float32, device. */
int kf_mlp_features(kf_ctx* ctx, const kf_tracks* t, const int32_t* target_layer, float* feats,
                    int flags, void* stream);
/* Training targets: for n propagations with inputs feats [8][ld] (from
 * kf_mlp_features) and transverse path lengths path_len [ld] [cm] (from the
 * plain kf_propagate), target [ld] = the network output that makes the guess
 * equal the path, (path_len - s_line) / (h s_line^2) in the inputs' units
 * (s_line = 100 feats[5], h s_line^2 = 100 feats[3] feats[5]^2 / feats[4]);
 * 0 where |feats[3] feats[5]^2 / feats[4]| <= 1e-9 (no curvature term).
 * Device float arrays; rows beyond n untouched. */
int kf_mlp_targets(kf_ctx* ctx, const float* feats, const float* path_len, int64_t n, int64_t ld,
                   float* target, void* stream);
/* Network outputs out [n] for inputs feats [8][ld] (device). */
int kf_mlp_forward(kf_ctx* ctx, const float* feats, int64_t n, int64_t ld, float* out, void* stream);
/* Mean-squared-error loss and its gradient over the batch rows rows [batch]
 * (int32 indices into the n columns of feats [8][ld] and target [ld]; rows
 * outside [0, n) are skipped but still count in the mean).  grad: device
 * float [4801]; loss: device float [1] or NULL.  Parameters unchanged. */
int kf_mlp_grad(kf_ctx* ctx, const float* feats, const float* target, int64_t n, int64_t ld,
                const int32_t* rows, int32_t batch, float* grad, float* loss, void* stream);
/* n_steps Adam steps; step k uses the rows rows[k*batch .. (k+1)*batch) (the
 * caller draws the shuffling).  cfg: host, NULL = defaults.  loss: optional
 * device float [n_steps], the batch loss before each step. */
int kf_mlp_train(kf_ctx* ctx, const float* feats, const float* target, int64_t n, int64_t ld,
                 const int32_t* rows, int32_t batch, int32_t n_steps, const kf_mlp_train_cfg* cfg,
                 float* loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif
