"""Seeded synthetic inputs shared by tests, smoke() and bench.py.

Holds the detector descriptions and the event generator only; no part of the
Kalman-filter arithmetic lives here.
"""
import numpy as np

from . import geometry
from .generate import (Event, fit_sample, precision_sample, find_events,
                       batch_events, make_event, pt_uniform, pt_power2,
                       pt_two_values, sig_loguniform, KAPPA, propagation_pairs, batch_propagation_pairs,
                       mlp_init)


def concat_events(events):
    """Concatenate events into one hit list; returns dict of arrays with
    event offsets and global (concatenated) hit indices for track sequences."""
    offs = np.zeros(len(events) + 1, np.int64)
    for i, e in enumerate(events):
        offs[i + 1] = offs[i] + e.n_hits
    cat = lambda name: np.concatenate([getattr(e, name) for e in events])
    seq_hit = []
    for i, e in enumerate(events):
        s = e.seq_hit.astype(np.int64)
        seq_hit.append(np.where(s >= 0, s + offs[i], -1))
    width = max(e.seq_hit.shape[1] for e in events)
    pad = lambda a, v: np.pad(a, ((0, 0), (0, width - a.shape[1])), constant_values=v)
    return dict(
        x=cat("x"), y=cat("y"), z=cat("z"), su=cat("su"), sv=cat("sv"),
        layer=cat("layer"), sim=cat("sim"), event_off=offs,
        seq_hit=np.concatenate([pad(s, -1) for s in seq_hit]).astype(np.int32),
        seq_layer=np.concatenate([pad(e.seq_layer, -1) for e in events]).astype(np.int32),
        track_event=np.concatenate([np.full(e.n_tracks, i, np.int32)
                                    for i, e in enumerate(events)]),
    )


def find_inputs(events, min_hits=3):
    """Concatenated hits of several events plus one seed per track with at
    least `min_hits` hits (its first three hits in crossing order).

    Returns a dict: hits arrays (x, y, z, su, sv, layer, sim), event_off
    [n_events+1], seed_event [n_seeds], seed_track [n_seeds] (track index
    within its event), seed_hits [n_seeds, 3] global hit indices,
    seed_hits_local [n_seeds, 3] event-local indices, seed_layers [n_seeds, 3].
    """
    cat = concat_events(events)
    se, st, sh, shl, sl = [], [], [], [], []
    for i, e in enumerate(events):
        nh = e.n_track_hits()
        sel = np.nonzero(nh >= min_hits)[0]
        se.append(np.full(sel.shape[0], i, np.int32))
        st.append(sel.astype(np.int32))
        loc = e.seq_hit[sel, :3].astype(np.int64)
        shl.append(loc.astype(np.int32))
        sh.append((loc + cat["event_off"][i]).astype(np.int32))
        sl.append(e.seq_layer[sel, :3].astype(np.int32))
    cat.update(seed_event=np.concatenate(se), seed_track=np.concatenate(st),
               seed_hits=np.concatenate(sh), seed_hits_local=np.concatenate(shl),
               seed_layers=np.concatenate(sl))
    return cat


__all__ = ["find_inputs", "geometry", "Event", "fit_sample", "precision_sample", "find_events",
           "batch_events", "make_event", "concat_events", "pt_uniform",
           "pt_power2", "pt_two_values", "sig_loguniform", "KAPPA", "propagation_pairs", "batch_propagation_pairs",
           "mlp_init"]
