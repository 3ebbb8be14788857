"""Duplicate seeds from detector-module overlaps (synthetic): where a track
crosses two overlapping modules of one layer it leaves two measurements of
that layer, and every combination of the hits on its first three layers
makes a seed, so one particle yields up to eight seeds.  Input generation
only.

Overlap model: on each of a track's first three crossings, with probability
p_barrel (barrel) or p_disk (disk), a second measurement of the same true
crossing, smeared independently with the layer's resolution, is appended to
the event's hits (same layer and track id)."""
import itertools
from dataclasses import replace

import numpy as np

from . import geometry as G
from .generate import _layer_sigmas, _make_hits, batch_events, find_events

N_FIRST = 3


def add_overlaps(rng, geom, ev, p_barrel=0.1, p_disk=0.3):
    """Returns (event with the overlap hits appended, ovl [n_trk, 3]: index of
    the second hit on the track's k-th crossing, -1 none)."""
    lay = ev.seq_layer[:, :N_FIRST]
    kind = np.array([L["kind"] for L in geom])
    p = np.where(lay >= 0, np.where(kind[np.maximum(lay, 0)] == 0, p_barrel, p_disk), 0.0)
    pick = (rng.random(lay.shape) < p) & (lay >= 0)
    sel = np.where(pick, lay, -1)
    ti, si, hl, hx, hy, hz, hsu, hsv = _make_hits(rng, geom, sel, ev.truth_at[:, :N_FIRST],
                                                  _layer_sigmas(geom))
    n0 = ev.n_hits
    ovl = np.full(lay.shape, -1, np.int32)
    ovl[ti, si] = n0 + np.arange(ti.shape[0])
    f32 = lambda a, b: np.concatenate([a, np.asarray(b, np.float32)])
    ev2 = replace(ev, x=f32(ev.x, hx), y=f32(ev.y, hy), z=f32(ev.z, hz), su=f32(ev.su, hsu),
                  sv=f32(ev.sv, hsv), layer=np.concatenate([ev.layer, hl.astype(np.int32)]),
                  sim=np.concatenate([ev.sim, ti.astype(np.int32)]))
    return ev2, ovl


def overlap_inputs(events, ovls):
    """Like eventgen.find_inputs, with one seed per combination of the hits on
    a track's first three crossings (tracks with >= 3 hits), in track order."""
    from . import concat_events
    cat = concat_events(events)
    se, st, sh, shl, sl = [], [], [], [], []
    for i, (e, ovl) in enumerate(zip(events, ovls)):
        nh = e.n_track_hits()
        off = int(cat["event_off"][i])
        for t in np.nonzero(nh >= N_FIRST)[0]:
            opts = [[int(e.seq_hit[t, k])] + ([int(ovl[t, k])] if ovl[t, k] >= 0 else [])
                    for k in range(N_FIRST)]
            for combo in itertools.product(*opts):
                se.append(i)
                st.append(t)
                shl.append(combo)
                sh.append([h + off for h in combo])
                sl.append(e.seq_layer[t, :N_FIRST])
    cat.update(seed_event=np.asarray(se, np.int32), seed_track=np.asarray(st, np.int32),
               seed_hits=np.asarray(sh, np.int32).reshape(-1, 3),
               seed_hits_local=np.asarray(shl, np.int32).reshape(-1, 3),
               seed_layers=np.asarray(sl, np.int32).reshape(-1, 3))
    return cat


def overlap_find_events(n_events=5, n_tracks=800, n_noise=50_000, seed=8, p_barrel=0.3):
    """The finding workload (ten barrels, 0.02 X0) with overlap hits on the
    first three layers at probability p_barrel.  Returns (geom, events, ovls)."""
    geom, evs = find_events(n_events=n_events, n_tracks=n_tracks, n_noise=n_noise, seed=seed)
    rng = np.random.default_rng(seed + 500)
    out = [add_overlaps(rng, geom, e, p_barrel=p_barrel) for e in evs]
    return geom, [o[0] for o in out], [o[1] for o in out]


def overlap_batch(seed=9, p_barrel=0.1, p_disk=0.3, **kw):
    """The uneven-multiplicity batch (ten barrels + 2 x 7 disks) with overlap
    hits: p_barrel on barrels, p_disk on disks (overlaps are densest in the
    endcaps).  Returns (geom, events, ovls)."""
    geom, evs = batch_events(seed=seed, **kw)
    rng = np.random.default_rng(seed + 500)
    out = [add_overlaps(rng, geom, e, p_barrel=p_barrel, p_disk=p_disk) for e in evs]
    return geom, [o[0] for o in out], [o[1] for o in out]


def seed_set(n=6000, n_events=3, seed=11, n_hits=20_000):
    """Synthetic seed collection for the cleaning alone: dense clusters of
    seeds (so that duplicates chain) placed across eta-phi cell edges and the
    phi = +-pi seam, hits drawn from a small pool (shared hits), chi2 on a
    coarse grid (equal values occur), a few seeds with a failed-fit status;
    n_events * n_hits hits in all.  Returns dict: par [n, 6] float32, chi2 [n] float32, status [n] uint32,
    event [n] int32, hits [n, 3] int32."""
    rng = np.random.default_rng(seed)
    n_cl = n // 6
    ce = rng.uniform(-2.9, 2.9, n_cl)
    cp = np.where(rng.random(n_cl) < 0.2, np.pi - 0.003, rng.uniform(-np.pi, np.pi, n_cl))
    cc = rng.uniform(-2.0, 2.0, n_cl)
    which = rng.integers(0, n_cl, n)
    eta = ce[which] + rng.normal(0, 0.006, n)
    phi = cp[which] + rng.normal(0, 0.006, n)
    phi = (phi + np.pi) % (2 * np.pi) - np.pi
    c = cc[which] + rng.normal(0, 0.03, n)
    par = np.zeros((n, 6), np.float32)
    par[:, 0] = rng.normal(0, 5, n)
    par[:, 1] = rng.normal(0, 5, n)
    par[:, 2] = rng.normal(0, 5, n)
    par[:, 3] = c
    par[:, 4] = phi
    par[:, 5] = 2 * np.arctan(np.exp(-eta))
    chi2 = (rng.integers(0, 400, n) * 0.05).astype(np.float32)
    status = np.where(rng.random(n) < 0.02, 2, 0).astype(np.uint32)
    event = rng.integers(0, n_events, n).astype(np.int32)
    # hit indices are global: event e owns [e n_hits, (e + 1) n_hits)
    hits = (rng.integers(0, n_hits, (n, 3)) + event[:, None] * n_hits).astype(np.int32)
    hits[rng.random((n, 3)) < 0.05] = -1
    return dict(par=par, chi2=chi2, status=status, event=event, hits=hits)


def track_set(n=5000, n_events=3, nl=10, seed=13, pool=400):
    """Synthetic found-track collection for duplicate removal alone: groups
    of 1-6 tracks derived from a base hit list (each entry kept, replaced or
    dropped at random), so that shared fractions fall on both sides of the
    usual thresholds; chi2 on a coarse grid (equal values occur); 2% with a
    failed status.  Hit indices are global: layer l of event e draws from its
    own range.  Returns dict: hits [n, nl] int32, chi2 [n] float32, status
    [n] uint32, event [n] int32, n_hits."""
    rng = np.random.default_rng(seed)
    hits = np.full((n, nl), -1, np.int32)
    event = np.zeros(n, np.int32)
    i = 0
    while i < n:
        e = int(rng.integers(0, n_events))
        base = rng.integers(0, pool, nl)
        nb = int(rng.integers(3, nl + 1))
        for _ in range(int(rng.integers(1, 7))):
            if i >= n:
                break
            row = np.where(rng.random(nl) < 0.75, base, rng.integers(0, pool, nl))
            row = np.where(rng.random(nl) < 0.15, -1, row)
            row[nb:] = -1
            ok = row >= 0
            hits[i] = np.where(ok, row + (e * nl + np.arange(nl)) * pool, -1)
            event[i] = e
            i += 1
    chi2 = (rng.integers(0, 50, n) * 0.5).astype(np.float32)
    status = np.where(rng.random(n) < 0.02, 8, 0).astype(np.uint32)
    return dict(hits=hits, chi2=chi2, status=status, event=event, n_hits=n_events * nl * pool)


__all__ = ["track_set", "add_overlaps", "overlap_inputs", "overlap_find_events", "overlap_batch", "seed_set",
           "G"]
