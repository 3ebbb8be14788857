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
    """Relative parameter error in units of the parity scale (1 = at tolerance)."""
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
               tie=np.full(ns, -1, np.int64), n_prop=0, n_upd=0)
    for e, ev in enumerate(events):
        m = np.nonzero(inp["seed_event"] == e)[0]
        if m.size == 0:
            continue
        r = orc.find(cfg, ev, inp["seed_hits_local"][m], binned=True, n_threads=n_threads)
        off = inp["event_off"][e]
        out["hits"][m] = np.where(r["hits"] >= 0, r["hits"] + off, -1)
        for k in ("par", "cov", "chi2", "ndf", "status", "tie"):
            out[k][m] = r[k]
        out["n_prop"] += r["n_prop"]
        out["n_upd"] += r["n_upd"]
    return out


def compare_find(g, o):
    """Found-hit-list parity: returns (n_exact, n_excused_mismatch, bad_seed_indices)."""
    same = (g["hits"] == o["hits"]).all(axis=1)
    tie = o["tie"] >= 0
    bad = np.nonzero(~same & ~tie)[0]
    return int(same.sum()), int((~same & tie).sum()), bad
