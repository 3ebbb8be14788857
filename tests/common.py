"""Shared helpers for the parity tests: input marshalling and the comparison
rules (tolerances stated once, here)."""
import numpy as np

# Parameter parity: |d| <= REL * max(|p_oracle|, floor); phi compared modulo 2 pi.
REL = 1e-4
FLOORS = np.array([1.0, 1.0, 1.0, 0.01, 1.0, 1.0])     # cm, cm, cm, 1/GeV, rad, rad
CHI2_REL = 1e-3                                        # |dchi2| <= 1e-3 * max(chi2, ndf, 1)


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def par_error(gpu_par, orc_par):
    """Relative parameter error |d| / max(|p_oracle|, floor), phi modulo 2 pi
    (REL is the tolerance on it)."""
    d = gpu_par - orc_par
    d[:, 4] = wrap(d[:, 4])
    scale = np.maximum(np.abs(orc_par), FLOORS)
    return np.abs(d) / scale


def chi2_error(gpu_chi2, orc_chi2, ndf):
    return np.abs(gpu_chi2 - orc_chi2) / np.maximum(np.maximum(np.abs(orc_chi2), ndf), 1.0)


def seed_hits(ev):
    """[n_trk, 3] first three hits in crossing order (tracks with >= 3 hits)."""
    return ev.seq_hit[:, :3]


def ld_of(n):
    return max(64, (n + 63) // 64 * 64)


def soa_int(a, ld, fill=-1):
    """[n, k] int array -> [k, ld] int32 (SoA) padded with `fill`."""
    n, k = a.shape
    out = np.full((k, ld), fill, np.int32)
    out[:, :n] = a.T
    return out


def oracle_find_events(orc, geom, events, inp, n_threads=8, **cfg_kw):
    """Run the oracle finder event by event on the seeds of `inp`
    (eventgen.find_inputs); hit lists are returned as global hit indices."""
    cfg = orc.Config(geom, **cfg_kw)
    ns = inp["seed_hits"].shape[0]
    nl = len(geom)
    out = dict(hits=np.full((ns, nl), -1, np.int64), par=np.zeros((ns, 6)), cov=np.zeros((ns, 21)),
               chi2=np.zeros(ns), ndf=np.zeros(ns, np.int64), status=np.zeros(ns, np.int64),
               tie=np.full(ns, -1, np.int64), visit=np.full((ns, nl), -1, np.int64), n_prop=0,
               n_upd=0)
    for e, ev in enumerate(events):
        m = np.nonzero(inp["seed_event"] == e)[0]
        if m.size == 0:
            continue
        r = orc.find(cfg, ev, inp["seed_hits_local"][m], binned=True, n_threads=n_threads)
        off = inp["event_off"][e]
        out["hits"][m] = np.where(r["hits"] >= 0, r["hits"] + off, -1)
        for k in ("par", "cov", "chi2", "ndf", "status", "tie", "visit"):
            out[k][m] = r[k]
        out["n_prop"] += r["n_prop"]
        out["n_upd"] += r["n_upd"]
    return out


# Excused seeds (oracle ties) may be at most this fraction of all seeds.
MAX_EXCUSED_FRAC = 1e-3


def compare_find(g, o):
    """Found-hit-list parity: returns (n_exact, n_excused_mismatch, bad_seed_indices).
    A differing seed is excused iff the oracle took a decision within 1e-3
    of its threshold somewhere in that seed's walk (its tie step >= 0): a
    close pruning decision at one step chooses between lineages whose hit
    lists can differ at any earlier layer, so the step of the first
    difference does not locate the decision.  Callers bound the excused count
    (MAX_EXCUSED_FRAC)."""
    same = (g["hits"] == o["hits"]).all(axis=1)
    tie = o["tie"] >= 0
    bad = np.nonzero(~same & ~tie)[0]
    return int(same.sum()), int((~same & tie).sum()), bad


def perturb_ulp(ev, rng):
    """A copy of event `ev` with every hit coordinate moved by one float32
    ulp in a random direction (the resolution the hits are given in)."""
    import copy
    out = copy.copy(ev)

    def f(a):
        a32 = np.asarray(a, np.float32)
        to = np.where(rng.random(a32.shape) < 0.5, np.float32(np.inf), np.float32(-np.inf))
        return np.nextafter(a32, to).astype(np.asarray(a).dtype)
    out.x, out.y, out.z = f(ev.x), f(ev.y), f(ev.z)
    return out


def oracle_sensitivity(orc, geom, events, inp, seeds, trials=4, seed=0, **cfg_kw):
    """Condition estimate of the oracle's result at the hits' resolution: for
    each seed in `seeds` (global indices into inp), the largest relative
    parameter change (par_error) of the FP64 oracle's found track over
    `trials` runs on its event with every hit moved by one float32 ulp; inf
    where a perturbed run finds another hit list."""
    cfg = orc.Config(geom, **cfg_kw)
    rng = np.random.default_rng(seed)
    seeds = np.asarray(seeds)
    sens = np.zeros(seeds.size)
    for e in np.unique(inp["seed_event"][seeds]):
        m = np.nonzero(inp["seed_event"][seeds] == e)[0]
        sl = inp["seed_hits_local"][seeds[m]]
        r0 = orc.find(cfg, events[e], sl, binned=True)
        for _ in range(trials):
            r1 = orc.find(cfg, perturb_ulp(events[e], rng), sl, binned=True)
            d = par_error(r1["par"].copy(), r0["par"]).max(axis=1)
            d[~(r1["hits"] == r0["hits"]).all(axis=1)] = np.inf
            sens[m] = np.maximum(sens[m], d)
    return sens


def check_find_params(g, o, label, sens_fn):
    """Parameter and chi2 parity of the seeds whose hit lists are identical:
    |dp| < REL (par_error), |dchi2| < CHI2_REL, same ndf.  A seed above REL is
    accepted only if it is ill-conditioned at the hits' resolution: the
    oracle's own result moves by at least 0.1 REL when the hits move by one
    float32 ulp (sens_fn(seed indices) -> oracle_sensitivity), and then it
    must lie within 10 times that movement; such seeds are counted and may
    be at most MAX_EXCUSED_FRAC of the seeds."""
    # status bit 4 (the learned guess fell back) only informs
    same = (g["hits"] == o["hits"]).all(axis=1) & (o["status"] == 0) & ((g["status"] & ~4) == 0)
    idx = np.nonzero(same)[0]
    err = par_error(g["par"][same], o["par"][same])
    e1 = err.max(axis=1)
    over = idx[e1 >= REL]
    print(f"{label}: max rel par err {err.max(axis=0) if err.size else 0}; "
          f"{over.size} seeds above {REL:g}")
    if over.size:
        sens = sens_fn(over)
        eo = e1[e1 >= REL]
        print(f"{label}: ill-conditioned seeds {over.tolist()[:10]}: errors {eo[:10]}, oracle "
              f"one-ulp sensitivity {sens[:10]}")
        assert (sens >= 0.1 * REL).all(), (label, over[sens < 0.1 * REL], eo[sens < 0.1 * REL])
        assert (eo < 10 * sens).all(), (label, eo, sens)
        assert over.size <= MAX_EXCUSED_FRAC * max(len(same), 1000)
    cerr = chi2_error(g["chi2"][same], o["chi2"][same], o["ndf"][same])
    assert cerr.size == 0 or cerr.max() < CHI2_REL, cerr.max()
    assert np.array_equal(g["ndf"][same], o["ndf"][same])


def check_fit_params(g, o, label, sens_fn):
    """Fit parity: status equal, |dp| < REL, |dchi2| < CHI2_REL on the tracks
    the oracle fitted.  A track above REL is accepted only if it is
    ill-conditioned at the hits' resolution (sens_fn(track indices) -> the
    oracle's largest relative parameter change over refits with its hits
    moved by one float32 ulp, >= 0.1 REL) and lies within 10 times that
    change; such tracks may be at most MAX_EXCUSED_FRAC of the tracks."""
    assert np.array_equal(g["status"], o["status"]), label
    ok = np.nonzero(o["status"] == 0)[0]
    err = par_error(g["par"][ok], o["par"][ok])
    e1 = err.max(axis=1)
    cerr = chi2_error(g["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
    over = ok[e1 >= REL]
    print(f"{label}: {ok.size} tracks, max rel par err per parameter {err.max(axis=0)}, "
          f"{over.size} above {REL:g}, chi2 err / tol {cerr.max() / CHI2_REL:.3f}")
    if over.size:
        sens = sens_fn(over)
        eo = e1[e1 >= REL]
        print(f"{label}: ill-conditioned tracks {over.tolist()[:10]}: errors {eo[:10]}, oracle "
              f"one-ulp sensitivity {sens[:10]}")
        assert (sens >= 0.1 * REL).all() and (eo < 10 * sens).all(), (label, eo, sens)
        assert over.size <= MAX_EXCUSED_FRAC * max(ok.size, 1000)
    assert cerr.max() < CHI2_REL
