"""Seeded synthetic inputs shared by tests, smoke() and bench.py.

Holds the detector descriptions and the event generator only; no part of the
Kalman-filter arithmetic lives here.
"""
import numpy as np

from . import geometry
from .generate import (Event, fit_sample, precision_sample, find_events,
                       batch_events, make_event, pt_uniform, pt_power2,
                       pt_two_values, sig_loguniform, KAPPA)


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


__all__ = ["geometry", "Event", "fit_sample", "precision_sample", "find_events",
           "batch_events", "make_event", "concat_events", "pt_uniform",
           "pt_power2", "pt_two_values", "sig_loguniform", "KAPPA"]
