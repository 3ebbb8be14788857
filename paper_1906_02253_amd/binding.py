"""ctypes binding of libkfmi.so over torch device tensors.

Argument marshalling only: every step of the path runs in the HIP kernels of
libkfmi.so.  If the library is missing the import of this module raises; there
is no fallback implementation.
"""
import ctypes as C
import numpy as np
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# KFMI_LIB selects another build of the same library (e.g. an instrumented one)
LIB_PATH = os.environ.get("KFMI_LIB") or os.path.join(HERE, "libkfmi.so")

KF_OK, KF_EINVAL, KF_EHIP, KF_ENOMEM, KF_EUNSUPPORTED = 0, -1, -2, -3, -4
ST_OK, ST_UNREACHABLE, ST_NOCONV, ST_FALLBACK, ST_NONPD, ST_NAN, ST_BADINPUT = 0, 1, 2, 4, 8, 16, 32
ST_DUPLICATE, ST_DUPTRACK = 64, 128
PREC_MIXED, PREC_FP32, PREC_FP64 = 0, 1, 2
INIT_MLP, NO_MATERIAL, PER_LAYER, CLEAN_SEEDS, REMOVE_DUPLICATES = 4, 8, 16, 32, 64

class KfLayer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nbin_phi", C.c_int32), ("nbin_2", C.c_int32),
                ("reserved", C.c_int32), ("r_or_z", C.c_double), ("lo", C.c_double),
                ("hi", C.c_double), ("x0", C.c_double), ("win_su", C.c_double),
                ("win_sv", C.c_double)]


class KfParams(C.Structure):
    _fields_ = [("bz", C.c_double), ("chi2_cut", C.c_double), ("newton_tol", C.c_double),
                ("mass", C.c_double), ("max_cands", C.c_int32), ("max_newton", C.c_int32),
                ("max_miss", C.c_int32), ("mlp_max_iter", C.c_int32), ("field_z0", C.c_double),
                ("field_step", C.c_double), ("clean_deta", C.c_double), ("clean_dphi", C.c_double),
                ("clean_dc", C.c_double), ("dup_frac", C.c_double)]


class KfMaterial(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("r_max", C.c_double), ("z_min", C.c_double),
                ("z_max", C.c_double), ("x0", C.c_void_p), ("xi", C.c_void_p)]


class KfRegion(C.Structure):
    _fields_ = [("eta_lo", C.c_double), ("eta_hi", C.c_double), ("n_layers", C.c_int32),
                ("layers", C.c_int32 * 64)]


class KfTracks(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64), ("par", C.c_void_p), ("cov", C.c_void_p),
                ("chi2", C.c_void_p), ("ndf", C.c_void_p), ("status", C.c_void_p)]


class KfHits(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("su", C.c_void_p), ("sv", C.c_void_p), ("layer", C.c_void_p)]


class KfTrainCfg(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


MLP_NPARAM, MLP_NIN = 4801, 8
N_COUNTERS = 8      # propagations, updates, chi2 tests, Newton evaluations, disk tests,
                    # learned guesses, learned guesses that fell back, children kept


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build()); "
                           "there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.kf_create.argtypes = [C.POINTER(vp), C.POINTER(KfLayer), i32, C.POINTER(KfParams)]
    L.kf_create.restype = C.c_int
    L.kf_destroy.argtypes = [vp]
    L.kf_last_error.argtypes = [vp]
    L.kf_last_error.restype = C.c_char_p
    L.kf_last_error_global.restype = C.c_char_p
    L.kf_seed.argtypes = [vp, C.POINTER(KfHits), vp, C.POINTER(KfTracks), C.c_int, vp]
    L.kf_propagate.argtypes = [vp, C.POINTER(KfTracks), vp, vp, vp, C.c_int, vp]
    L.kf_fit.argtypes = [vp, C.POINTER(KfTracks), C.POINTER(KfHits), vp, vp, i32, C.c_int, vp]
    L.kf_find.argtypes = [vp, C.POINTER(KfHits), vp, i32, C.POINTER(KfTracks), vp, vp, vp,
                          C.POINTER(KfTracks), vp, C.c_int, vp]
    L.kf_find_noalloc.argtypes = [vp, C.POINTER(KfHits), vp, i32, C.POINTER(KfTracks), vp, vp, vp,
                                  C.POINTER(KfTracks), vp, C.c_int, vp]
    L.kf_find_batched.argtypes = [vp, C.POINTER(KfHits), vp, i32, vp, vp, vp, C.POINTER(KfTracks),
                                  vp, C.POINTER(KfTracks), vp, C.c_int, vp]
    L.kf_set_material.argtypes = [vp, C.POINTER(KfMaterial)]
    L.kf_set_steering.argtypes = [vp, C.POINTER(KfRegion), i32]
    L.kf_remove_duplicates.argtypes = [vp, C.POINTER(KfHits), C.POINTER(KfTracks), vp, vp, C.c_int,
                                       vp]
    L.kf_clean_seeds.argtypes = [vp, C.POINTER(KfHits), i32, C.POINTER(KfTracks), vp, vp, C.c_int,
                                 vp]
    L.kf_set_find_config.argtypes = [vp, i32, i32]
    L.kf_get_find_config.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.kf_autotune.argtypes = [vp, C.POINTER(KfHits), vp, i32, C.POINTER(KfTracks), vp, vp, vp,
                              C.POINTER(KfTracks), C.c_int, i32, C.POINTER(C.c_float), vp]
    L.kf_set_timing.argtypes = [vp, i32]
    L.kf_timings.argtypes = [vp, C.POINTER(C.c_float)]
    fp = C.POINTER(C.c_float)
    L.kf_mlp_load.argtypes = [vp, fp]
    L.kf_mlp_get.argtypes = [vp, fp]
    L.kf_mlp_features.argtypes = [vp, C.POINTER(KfTracks), vp, vp, C.c_int, vp]
    L.kf_mlp_forward.argtypes = [vp, vp, i64, i64, vp, vp]
    L.kf_mlp_targets.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    L.kf_mlp_grad.argtypes = [vp, vp, vp, i64, i64, vp, i32, vp, vp, vp]
    L.kf_mlp_train.argtypes = [vp, vp, vp, i64, i64, vp, i32, i32, C.POINTER(KfTrainCfg), vp, vp]
    for f in ("kf_seed", "kf_propagate", "kf_fit", "kf_find", "kf_find_batched", "kf_find_noalloc",
              "kf_set_find_config", "kf_get_find_config", "kf_autotune", "kf_set_timing",
              "kf_timings", "kf_mlp_load", "kf_mlp_get", "kf_mlp_features", "kf_mlp_forward",
              "kf_mlp_targets",
              "kf_mlp_grad", "kf_mlp_train"):
        getattr(L, f).restype = C.c_int
    return L


lib = _load()


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def round_ld(n):
    return max(64, (n + 63) // 64 * 64)


class Tracks:
    """SoA track states on the GPU: par [6, ld], cov [21, ld], chi2 [ld], ndf, status.

    Storage types follow the precision: MIXED and FP32 float32, FP64 float64."""

    def __init__(self, n, ld=None, prec=PREC_MIXED, device="cuda"):
        self.n = int(n)
        self.ld = int(ld or round_ld(n))
        self.prec = prec
        pd = torch.float64 if prec == PREC_FP64 else torch.float32
        cd = pd
        self.par = torch.zeros((6, self.ld), dtype=pd, device=device)
        self.cov = torch.zeros((21, self.ld), dtype=cd, device=device)
        self.chi2 = torch.zeros(self.ld, dtype=pd, device=device)
        self.ndf = torch.zeros(self.ld, dtype=torch.int32, device=device)
        self.status = torch.zeros(self.ld, dtype=torch.int32, device=device)

    def c(self):
        return KfTracks(self.n, self.ld, _ptr(self.par), _ptr(self.cov), _ptr(self.chi2),
                        _ptr(self.ndf), _ptr(self.status))

    @staticmethod
    def from_numpy(par, cov, prec=PREC_MIXED, ld=None):
        n = par.shape[0]
        t = Tracks(n, ld, prec)
        t.par[:, :n] = torch.as_tensor(par.T, dtype=t.par.dtype)
        t.cov[:, :n] = torch.as_tensor(cov.T, dtype=t.cov.dtype)
        return t

    def numpy(self):
        n = self.n
        return dict(par=self.par[:, :n].T.double().cpu().numpy(),
                    cov=self.cov[:, :n].T.double().cpu().numpy(),
                    chi2=self.chi2[:n].double().cpu().numpy(),
                    ndf=self.ndf[:n].cpu().numpy(),
                    status=self.status[:n].cpu().numpy())


class Hits:
    """SoA float32 hits on the GPU."""

    def __init__(self, x, y, z, su, sv, layer, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32, device=device).contiguous()
        self.x, self.y, self.z, self.su, self.sv = f(x), f(y), f(z), f(su), f(sv)
        self.layer = torch.as_tensor(layer, dtype=torch.int32, device=device).contiguous()
        self.n = int(self.x.shape[0])

    @staticmethod
    def from_event(ev, device="cuda"):
        return Hits(ev.x, ev.y, ev.z, ev.su, ev.sv, ev.layer, device)

    def c(self):
        return KfHits(self.n, _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.su),
                      _ptr(self.sv), _ptr(self.layer))


class KFError(RuntimeError):
    pass


class Context:
    """A kf_ctx: geometry + parameters (+ workspace) for one device."""

    def __init__(self, geom, bz=3.8, chi2_cut=30.0, max_cands=6, max_newton=10, newton_tol=1e-4,
                 mass=0.13957, max_miss=2, mlp_max_iter=3, field_z0=0.0, field_step=2.0,
                 clean_deta=0.01, clean_dphi=0.01, clean_dc=0.05, dup_frac=0.5):
        arr = (KfLayer * len(geom))()
        for i, L in enumerate(geom):
            arr[i] = KfLayer(int(L["kind"]), int(L["nbin_phi"]), int(L["nbin_2"]), 0,
                             L["r_or_z"], L["lo"], L["hi"], L["x0"], L["win_su"], L["win_sv"])
        self.n_layers = len(geom)
        prm = KfParams(bz, chi2_cut, newton_tol, mass, max_cands, max_newton, max_miss, mlp_max_iter,
                       field_z0, field_step, clean_deta, clean_dphi, clean_dc, dup_frac)
        h = C.c_void_p()
        torch.cuda.current_device()          # make sure the runtime is up on this device
        r = lib.kf_create(C.byref(h), arr, len(geom), C.byref(prm))
        if r != KF_OK:
            raise KFError(f"kf_create failed ({r}): {lib.kf_last_error_global().decode()}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib.kf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, r, what):
        if r != KF_OK:
            raise KFError(f"{what} failed ({r}): {lib.kf_last_error(self.h).decode()}")

    def seed(self, hits, seed_hits, out, flags=0):
        """seed_hits: int32 [3, ld] hit indices."""
        self._check(lib.kf_seed(self.h, C.byref(hits.c()), _ptr(seed_hits), C.byref(out.c()),
                                flags, _stream()), "kf_seed")

    def propagate(self, tracks, target, path_len=None, iters=None, flags=0):
        self._check(lib.kf_propagate(self.h, C.byref(tracks.c()), _ptr(target), _ptr(path_len),
                                     _ptr(iters), flags, _stream()), "kf_propagate")

    def fit(self, tracks, hits, layer_seq, hit_idx, max_steps, flags=0):
        self._check(lib.kf_fit(self.h, C.byref(tracks.c()), C.byref(hits.c()), _ptr(layer_seq),
                               _ptr(hit_idx), int(max_steps), flags, _stream()), "kf_fit")

    def set_timing(self, n=1):
        """Record phase events for the next n kf_find / kf_find_batched calls (0: off)."""
        self._check(lib.kf_set_timing(self.h, int(n)), "kf_set_timing")

    def timings(self):
        """Mean (seeding + seed fit, binning, seed ordering, finding kernel) ms
        over the recorded calls, and the number of calls recorded."""
        ms = (C.c_float * 5)()
        self._check(lib.kf_timings(self.h, ms), "kf_timings")
        return tuple(ms[:4]), int(ms[4])

    def set_find_config(self, width=64, largest_first=False):
        self._check(lib.kf_set_find_config(self.h, int(width), int(bool(largest_first))),
                    "kf_set_find_config")

    def find_config(self):
        w, lf = C.c_int32(), C.c_int32()
        self._check(lib.kf_get_find_config(self.h, C.byref(w), C.byref(lf)), "kf_get_find_config")
        return int(w.value), bool(lf.value)

    def set_steering(self, regions):
        """Tracking regions and layer plans: [dict(eta_lo, eta_hi, layers=[...]),
        ...] (at most 8, plans of at most 64 layers), or None for dynamic
        navigation."""
        if not regions:
            self._check(lib.kf_set_steering(self.h, None, 0), "kf_set_steering")
            return
        arr = (KfRegion * len(regions))()
        for g, R in enumerate(regions):
            lay = list(R["layers"])
            if len(lay) > 64:
                raise KFError("set_steering: a plan holds at most 64 layers")
            arr[g].eta_lo, arr[g].eta_hi, arr[g].n_layers = R["eta_lo"], R["eta_hi"], len(lay)
            for q, l in enumerate(lay):
                arr[g].layers[q] = int(l)
        self._check(lib.kf_set_steering(self.h, arr, len(regions)), "kf_set_steering")

    def set_material(self, m):
        """r-z material map: dict(r_max, z_min, z_max, x0 [nr, nz], xi [nr, nz])
        (host arrays, copied), or None to remove it."""
        if m is None:
            self._check(lib.kf_set_material(self.h, None), "kf_set_material")
            return
        x0 = np.ascontiguousarray(m["x0"], np.float32)
        xi = np.ascontiguousarray(m["xi"], np.float32)
        if x0.shape != xi.shape or x0.ndim != 2:
            raise KFError("set_material: x0 and xi must be 2-D arrays of one shape")
        km = KfMaterial(x0.shape[0], x0.shape[1], m["r_max"], m["z_min"], m["z_max"],
                        x0.ctypes.data, xi.ctypes.data)
        self._check(lib.kf_set_material(self.h, C.byref(km)), "kf_set_material")

    def remove_duplicates(self, hits, tracks, track_hits, track_event, flags=0):
        """Duplicate removal of found tracks: sets ST_DUPTRACK in tracks.status on
        removed tracks.  track_hits int32 [n, n_layers]; track_event int32 [n]."""
        self._check(lib.kf_remove_duplicates(self.h, C.byref(hits.c()), C.byref(tracks.c()),
                                             _ptr(track_hits), _ptr(track_event), flags, _stream()),
                    "kf_remove_duplicates")

    def clean_seeds(self, hits, n_events, seeds, seed_event, seed_hits, flags=0):
        """Seed cleaning: sets ST_DUPLICATE in seeds.status on removed seeds.
        seed_event int32 [ld]; seed_hits int32 [3, ld]."""
        self._check(lib.kf_clean_seeds(self.h, C.byref(hits.c()), int(n_events), C.byref(seeds.c()),
                                       _ptr(seed_event), _ptr(seed_hits), flags, _stream()),
                    "kf_clean_seeds")

    def find(self, hits, event_off, seeds, seed_event, seed_hits, out_hits, out, counters=None,
             flags=0):
        """event_off: int32 [n_events+1]; seed_event: int32 [n_seeds];
        seed_hits: int32 [3, seeds.ld]; out_hits: int32 [n_seeds, n_layers];
        counters: optional int64 [8], accumulated."""
        n_events = int(event_off.shape[0]) - 1
        self._check(lib.kf_find(self.h, C.byref(hits.c()), _ptr(event_off), n_events,
                                C.byref(seeds.c()), _ptr(seed_event), _ptr(seed_hits),
                                _ptr(out_hits), C.byref(out.c()), _ptr(counters), flags,
                                _stream()), "kf_find")

    def find_noalloc(self, hits, event_off, seeds, seed_event, seed_hits, out_hits, out,
                     counters=None, flags=0):
        """kf_find with the library's static scratch (no device allocation)."""
        n_events = int(event_off.shape[0]) - 1
        self._check(lib.kf_find_noalloc(self.h, C.byref(hits.c()), _ptr(event_off), n_events,
                                        C.byref(seeds.c()), _ptr(seed_event), _ptr(seed_hits),
                                        _ptr(out_hits), C.byref(out.c()), _ptr(counters), flags,
                                        _stream()), "kf_find_noalloc")

    def find_batched(self, hits, event_off, seed_hits, seed_layers, seed_event, seeds, out_hits,
                     out, counters=None, flags=0):
        """Seed, seed fit and find in one captured graph (replayed while the
        arrays stay the same).  seeds: scratch Tracks for the seed states."""
        n_events = int(event_off.shape[0]) - 1
        self._check(lib.kf_find_batched(self.h, C.byref(hits.c()), _ptr(event_off), n_events,
                                        _ptr(seed_hits), _ptr(seed_layers), _ptr(seed_event),
                                        C.byref(seeds.c()), _ptr(out_hits), C.byref(out.c()),
                                        _ptr(counters), flags, _stream()), "kf_find_batched")

    def autotune(self, hits, event_off, seeds, seed_event, seed_hits, out_hits, out, flags=0,
                 reps=3):
        """Times every (width, tile order); keeps the fastest.  Returns
        {(width, largest_first): ms}."""
        n_events = int(event_off.shape[0]) - 1
        tab = (C.c_float * 8)()
        self._check(lib.kf_autotune(self.h, C.byref(hits.c()), _ptr(event_off), n_events,
                                    C.byref(seeds.c()), _ptr(seed_event), _ptr(seed_hits),
                                    _ptr(out_hits), C.byref(out.c()), flags, int(reps), tab,
                                    _stream()), "kf_autotune")
        return {(w, bool(lf)): tab[2 * i + lf] for i, w in enumerate((32, 64, 128, 256))
                for lf in (0, 1) if tab[2 * i + lf] >= 0}

    # ---- learned initial guess
    def mlp_load(self, w):
        """w: numpy float32 [4801] (flat: W1, b1, W2, b2, w3, b3)."""
        import numpy as np
        a = np.ascontiguousarray(w, dtype=np.float32)
        if a.shape != (MLP_NPARAM,):
            raise ValueError("expected 4801 parameters")
        self._check(lib.kf_mlp_load(self.h, a.ctypes.data_as(C.POINTER(C.c_float))), "kf_mlp_load")

    def mlp_get(self):
        import numpy as np
        a = np.zeros(MLP_NPARAM, np.float32)
        self._check(lib.kf_mlp_get(self.h, a.ctypes.data_as(C.POINTER(C.c_float))), "kf_mlp_get")
        return a

    def mlp_features(self, tracks, target, feats, flags=0):
        """feats: float32 [8, tracks.ld] on the GPU."""
        self._check(lib.kf_mlp_features(self.h, C.byref(tracks.c()), _ptr(target), _ptr(feats),
                                        flags, _stream()), "kf_mlp_features")

    def mlp_targets(self, feats, path_len, n, target):
        """Training targets [ld] from inputs feats [8, ld] and path lengths [ld]."""
        self._check(lib.kf_mlp_targets(self.h, _ptr(feats), _ptr(path_len), int(n),
                                       int(feats.shape[1]), _ptr(target), _stream()),
                    "kf_mlp_targets")

    def mlp_forward(self, feats, n, out):
        self._check(lib.kf_mlp_forward(self.h, _ptr(feats), int(n), int(feats.shape[1]), _ptr(out),
                                       _stream()), "kf_mlp_forward")

    def mlp_grad(self, feats, target, n, rows, grad, loss=None):
        self._check(lib.kf_mlp_grad(self.h, _ptr(feats), _ptr(target), int(n), int(feats.shape[1]),
                                    _ptr(rows), int(rows.shape[0]), _ptr(grad), _ptr(loss),
                                    _stream()), "kf_mlp_grad")

    def mlp_train(self, feats, target, n, rows, batch, n_steps, lr=1e-3, beta1=0.9, beta2=0.999,
                  eps=1e-8, loss=None):
        cfg = KfTrainCfg(lr, beta1, beta2, eps)
        self._check(lib.kf_mlp_train(self.h, _ptr(feats), _ptr(target), int(n), int(feats.shape[1]),
                                     _ptr(rows), int(batch), int(n_steps), C.byref(cfg), _ptr(loss),
                                     _stream()), "kf_mlp_train")
