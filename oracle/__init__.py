"""FP64 CPU oracle for the KF fit and combinatorial finding.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; the product path (the HIP
library and its binding) never imports it and shares no code with it.

The arithmetic lives in ``kf_oracle.c`` (plain C, double precision); this
module builds it with gcc and marshals numpy arrays through ctypes.  The
MLP oracle (double-precision forward/backward/Adam) is in ``mlp.py``.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ST_OK, ST_UNREACHABLE, ST_NOCONV, ST_NONPD, ST_NAN, ST_DONE = 0, 1, 2, 8, 16, 32


def build(force=True):
    """Compile the oracle with gcc (strict IEEE double, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


class _Layer(C.Structure):
    _fields_ = [("kind", C.c_int), ("r_or_z", C.c_double), ("lo", C.c_double),
                ("hi", C.c_double), ("x0", C.c_double), ("nbin_phi", C.c_int),
                ("nbin_2", C.c_int), ("win_su", C.c_double), ("win_sv", C.c_double)]


class _Region(C.Structure):
    _fields_ = [("eta_lo", C.c_double), ("eta_hi", C.c_double), ("n", C.c_int),
                ("layers", C.c_int * 64)]


class _Cfg(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("layers", C.POINTER(_Layer)), ("bz", C.c_double),
                ("chi2_cut", C.c_double), ("max_cands", C.c_int), ("max_newton", C.c_int),
                ("newton_tol", C.c_double), ("mass", C.c_double), ("max_miss", C.c_int),
                ("use_material", C.c_int), ("field_z0", C.c_double), ("field_step", C.c_double),
                ("mat_nr", C.c_int), ("mat_nz", C.c_int), ("mat_rmax", C.c_double),
                ("mat_zmin", C.c_double), ("mat_zmax", C.c_double),
                ("mat_x0", C.POINTER(C.c_double)), ("mat_xi", C.POINTER(C.c_double)),
                ("n_regions", C.c_int), ("regions", C.POINTER(_Region))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        cfgp = C.POINTER(_Cfg)
        L.orc_helix.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_field.argtypes = [cfgp, dp, dp]
        L.orc_rk_path.argtypes = [cfgp, dp, C.c_double, dp]
        L.orc_propagate.argtypes = [cfgp, C.c_int, dp, dp, dp, dp, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int), C.c_int]
        L.orc_propagate.restype = C.c_int
        L.orc_solve_barrel.argtypes = [cfgp, dp, C.c_double, C.c_double,
                                       C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.orc_solve_barrel.restype = C.c_int
        L.orc_jacobian.argtypes = [cfgp, C.c_int, dp, dp]
        L.orc_jacobian.restype = C.c_int
        L.orc_update.argtypes = [dp, dp, dp, C.c_int, dp, dp, C.POINTER(C.c_double)]
        L.orc_update.restype = C.c_int
        L.orc_chi2.argtypes = [dp, dp, dp, C.c_int]
        L.orc_chi2.restype = C.c_double
        L.orc_seed.argtypes = [dp, dp, dp, C.c_double, dp, dp]
        L.orc_fit.argtypes = [cfgp, C.c_long, C.c_int, dp, dp, dp, dp, dp, ip, ip, dp, dp, dp,
                              ip, ip, C.c_int]
        L.orc_find.argtypes = [cfgp, C.c_long, dp, dp, dp, dp, dp, ip, C.c_long, ip, C.c_int,
                               ip, dp, dp, dp, ip, ip, ip, ip, lp, C.c_int]
        L.orc_dedup.argtypes = [C.c_long, C.c_int, ip, dp, ip, ip, C.c_double, ip]
        L.orc_dedx.argtypes = [C.c_double, C.c_double]
        L.orc_dedx.restype = C.c_double
        L.orc_material.argtypes = [cfgp, C.c_int, dp, dp]
        L.orc_clean_seeds.argtypes = [C.c_long, dp, dp, ip, ip, ip, C.c_double, C.c_double,
                                      C.c_double, ip, ip]
        _lib = L
    return _lib


class Config:
    """Geometry + filter parameters, held alive for the C side."""

    def __init__(self, geom, bz=3.8, chi2_cut=30.0, max_cands=6, max_newton=10,
                 newton_tol=1e-4, mass=0.13957, max_miss=2, material=None, field_z0=0.0,
                 field_step=2.0, material_map=None, steering=None):
        self.geom = geom
        arr = (_Layer * len(geom))()
        for i, L in enumerate(geom):
            arr[i] = _Layer(int(L["kind"]), L["r_or_z"], L["lo"], L["hi"], L["x0"],
                            int(L["nbin_phi"]), int(L["nbin_2"]), L["win_su"], L["win_sv"])
        self._arr = arr
        if material is None:
            material = any(L["x0"] > 0 for L in geom) or material_map is not None
        self.c = _Cfg(len(geom), arr, bz, chi2_cut, max_cands, max_newton, newton_tol, mass,
                      max_miss, int(bool(material)), field_z0, field_step)
        if steering:
            # [dict(eta_lo, eta_hi, layers=[...]), ...]: tracking regions and plans
            self._reg = (_Region * len(steering))()
            for g, R in enumerate(steering):
                self._reg[g].eta_lo, self._reg[g].eta_hi = R["eta_lo"], R["eta_hi"]
                self._reg[g].n = len(R["layers"])
                for q, l in enumerate(R["layers"]):
                    self._reg[g].layers[q] = int(l)
            self.c.n_regions = len(steering)
            self.c.regions = self._reg
        if material_map is not None:
            # dict(r_max, z_min, z_max, x0 [nr, nz], xi [nr, nz])
            m = material_map
            self._mx0 = np.ascontiguousarray(m["x0"], np.float64)
            self._mxi = np.ascontiguousarray(m["xi"], np.float64)
            self.c.mat_nr, self.c.mat_nz = self._mx0.shape
            self.c.mat_rmax, self.c.mat_zmin, self.c.mat_zmax = m["r_max"], m["z_min"], m["z_max"]
            dpp = C.POINTER(C.c_double)
            self.c.mat_x0 = self._mx0.ctypes.data_as(dpp)
            self.c.mat_xi = self._mxi.ctypes.data_as(dpp)
        self.ref = C.byref(self.c)


# packed upper-triangle index of a symmetric 6x6
PIDX = np.array([[min(i, j) * (11 - min(i, j)) // 2 + max(i, j) for j in range(6)]
                 for i in range(6)])


def unpack(Pk):
    Pk = np.asarray(Pk)
    return Pk[..., PIDX]


def pack(P):
    P = np.asarray(P)
    out = np.zeros(P.shape[:-2] + (21,))
    for i in range(6):
        for j in range(i, 6):
            out[..., PIDX[i, j]] = P[..., i, j]
    return out


def helix(p, s, bz=3.8):
    out = np.zeros(6)
    lib().orc_helix(np.ascontiguousarray(p, np.float64), float(s), bz, out)
    return out


def propagate(cfg, layer, p, Pk, noise=True):
    po, Po = np.zeros(6), np.zeros(21)
    s, it = C.c_double(0), C.c_int(0)
    st = lib().orc_propagate(cfg.ref, int(layer), np.ascontiguousarray(p, np.float64),
                             np.ascontiguousarray(Pk, np.float64), po, Po, C.byref(s),
                             C.byref(it), int(noise))
    return st, po, Po, s.value, it.value


def solve_barrel(cfg, p, r_l, s_init=-1.0):
    s, it = C.c_double(0), C.c_int(0)
    st = lib().orc_solve_barrel(cfg.ref, np.ascontiguousarray(p, np.float64), float(r_l),
                                float(s_init), C.byref(s), C.byref(it))
    return st, s.value, it.value


def jacobian(cfg, layer, p):
    F = np.zeros(36)
    st = lib().orc_jacobian(cfg.ref, int(layer), np.ascontiguousarray(p, np.float64), F)
    return st, F.reshape(6, 6)


def update(p, Pk, hit, kind):
    po, Po = np.zeros(6), np.zeros(21)
    c2 = C.c_double(0)
    st = lib().orc_update(np.ascontiguousarray(p, np.float64), np.ascontiguousarray(Pk, np.float64),
                          np.ascontiguousarray(hit, np.float64), int(kind), po, Po, C.byref(c2))
    return st, po, Po, c2.value


def chi2(p, Pk, hit, kind):
    return lib().orc_chi2(np.ascontiguousarray(p, np.float64), np.ascontiguousarray(Pk, np.float64),
                          np.ascontiguousarray(hit, np.float64), int(kind))


def seed(h1, h2, h3, bz=3.8):
    p, P = np.zeros(6), np.zeros(21)
    f = lambda h: np.ascontiguousarray(h, np.float64)
    lib().orc_seed(f(h1), f(h2), f(h3), bz, p, P)
    return p, P


def seeds_for_event(ev, bz=3.8):
    """Seed states (3-hit circle + prior) for every track with >= 3 hits."""
    n = ev.n_tracks
    par = np.zeros((n, 6))
    cov = np.zeros((n, 21))
    for t in range(n):
        sh = ev.seq_hit[t, :3]
        if (sh < 0).any():
            continue
        hs = [np.array([ev.x[i], ev.y[i], ev.z[i]], np.float64) for i in sh]
        par[t], cov[t] = seed(*hs, bz=bz)
    return par, cov


def fit(cfg, hits, layer_seq, hit_idx, par0, cov0, n_threads=1):
    """Fit n tracks.  hits: dict with x, y, z, su, sv arrays."""
    L = lib()
    n, ms = layer_seq.shape
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    par = f64(par0).copy()
    cov = f64(cov0).copy()
    chi2o = np.zeros(n)
    ndf = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    L.orc_fit(cfg.ref, n, ms, f64(hits["x"]), f64(hits["y"]), f64(hits["z"]), f64(hits["su"]),
              f64(hits["sv"]), np.ascontiguousarray(layer_seq, np.int32),
              np.ascontiguousarray(hit_idx, np.int32), par, cov, chi2o, ndf, st, int(n_threads))
    return dict(par=par, cov=cov, chi2=chi2o, ndf=ndf, status=st)


def find(cfg, ev, seed_hits, binned=True, n_threads=1):
    """Combinatorial finding on one event; seed_hits [n_seeds, 3] event-local
    indices.  Per seed: the best candidate's hit list, state, chi2, ndf and
    status; tie = the walk step of the first decision taken within 1e-3 of its
    threshold (nl: only the final choice was close; -1: none); visit [n_seeds,
    n_layers] = the walk step at which the best candidate last reached each
    layer (-1: never; the seed's own layers precede the walk)."""
    L = lib()
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    seed_hits = np.ascontiguousarray(seed_hits, np.int32)
    ns = seed_hits.shape[0]
    nl = len(cfg.geom)
    out_hits = np.zeros((ns, nl), np.int32)
    par = np.zeros((ns, 6))
    cov = np.zeros((ns, 21))
    c2 = np.zeros(ns)
    ndf = np.zeros(ns, np.int32)
    st = np.zeros(ns, np.int32)
    tie = np.zeros(ns, np.int32)
    visit = np.zeros((ns, nl), np.int32)
    cnt = np.zeros(2, np.int64)
    L.orc_find(cfg.ref, ev.n_hits, f64(ev.x), f64(ev.y), f64(ev.z), f64(ev.su), f64(ev.sv),
               np.ascontiguousarray(ev.layer, np.int32), ns, seed_hits, int(binned), out_hits,
               par, cov, c2, ndf, st, tie, visit, cnt, int(n_threads))
    return dict(hits=out_hits, par=par, cov=cov, chi2=c2, ndf=ndf, status=st, tie=tie,
                visit=visit, n_prop=int(cnt[0]), n_upd=int(cnt[1]))


def field(cfg, x):
    """Parametrised field at x (cm) [3] -> B [3] (T)."""
    B = np.zeros(3)
    lib().orc_field(cfg.ref, np.ascontiguousarray(x, np.float64), B)
    return B


def rk_path(cfg, p, l):
    """State after 3D path length l through the parametrised field."""
    out = np.zeros(6)
    lib().orc_rk_path(cfg.ref, np.ascontiguousarray(p, np.float64), float(l), out)
    return out


def clean_seeds(par, chi2, status, event, hits, deta=0.01, dphi=0.01, dc=0.05):
    """Seed cleaning (paper Sec. 3.2) by its definition, pairwise within each
    event.  par [n, 6], chi2 [n], status [n] (0 = takes part), event [n],
    hits [n, 3].  Returns (keep [n] bool, tie [n] bool)."""
    n = int(np.asarray(chi2).shape[0])
    keep = np.zeros(n, np.int32)
    tie = np.zeros(n, np.int32)
    lib().orc_clean_seeds(n, np.ascontiguousarray(par, np.float64).reshape(-1),
                          np.ascontiguousarray(chi2, np.float64),
                          np.ascontiguousarray(status, np.int32),
                          np.ascontiguousarray(event, np.int32),
                          np.ascontiguousarray(hits, np.int32).reshape(-1), float(deta), float(dphi),
                          float(dc), keep, tie)
    return keep.astype(bool), tie.astype(bool)


def dedx(p, m=0.13957):
    """Mean ionisation loss in silicon [MeV cm^2/g] (Bethe, no density effect)."""
    return lib().orc_dedx(float(p), float(m))


def material(cfg, layer, q, Pk):
    """Material effects (scattering noise, mean energy loss) at a crossing of
    `layer` by state q: returns (q', Pk')."""
    q = np.ascontiguousarray(q, np.float64).copy()
    Pk = np.ascontiguousarray(Pk, np.float64).copy()
    lib().orc_material(cfg.ref, int(layer), q, Pk)
    return q, Pk


def dedup(hits, chi2, status, event, frac=0.5):
    """Duplicate removal of found tracks by its definition, pairwise within
    each event.  hits [n, nl] (-1 none).  Returns keep [n] bool."""
    hits = np.ascontiguousarray(hits, np.int32)
    n, nl = hits.shape
    keep = np.zeros(n, np.int32)
    lib().orc_dedup(n, nl, hits.reshape(-1), np.ascontiguousarray(chi2, np.float64),
                    np.ascontiguousarray(status, np.int32), np.ascontiguousarray(event, np.int32),
                    float(frac), keep)
    return keep.astype(bool)
