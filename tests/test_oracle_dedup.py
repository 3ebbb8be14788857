"""Pins of the oracle's duplicate removal of found tracks (several seeds of
one particle give the same track; Sec. 4 names removing them as the cleaning
of the final collection): answers fixed by construction, brute force with
Python sets on small random collections, invariants of the rule, and the
result on module-overlap events found without seed cleaning."""
import itertools

import numpy as np

import eventgen.overlap as EO
from tests import common as CM


def _tracks(lists, nl=10):
    h = np.full((len(lists), nl), -1, np.int32)
    for i, L in enumerate(lists):
        h[i, :len(L)] = L
    return h


def test_threshold_and_ranking_by_construction(orc):
    z = lambda n: np.zeros(n, int)
    # 5 of 10 shared: duplicates at frac 0.5; 4 of 10: not
    a = list(range(10))
    b = list(range(5)) + list(range(100, 105))
    c = list(range(4)) + list(range(200, 206))
    keep = orc.dedup(_tracks([a, b]), [1.0, 2.0], z(2), z(2))
    assert keep.tolist() == [True, False]
    keep = orc.dedup(_tracks([a, c]), [1.0, 2.0], z(2), z(2))
    assert keep.tolist() == [True, True]
    # more hits wins over a lower chi2; then chi2; then the index
    short = list(range(6))
    keep = orc.dedup(_tracks([short, a]), [0.1, 50.0], z(2), z(2))
    assert keep.tolist() == [False, True]
    keep = orc.dedup(_tracks([a, a]), [3.0, 2.0], z(2), z(2))
    assert keep.tolist() == [False, True]
    keep = orc.dedup(_tracks([a, a, a]), [2.0, 2.0, 2.0], z(3), z(3))
    assert keep.tolist() == [True, False, False]
    # other events and failed tracks take no part
    keep = orc.dedup(_tracks([a, a]), [1.0, 2.0], z(2), np.array([0, 1]))
    assert keep.all()
    keep = orc.dedup(_tracks([a, a]), [1.0, 2.0], np.array([2, 0]), z(2))
    assert keep.all()
    # other fractions
    keep = orc.dedup(_tracks([a, c]), [1.0, 2.0], z(2), z(2), frac=0.4)
    assert keep.tolist() == [True, False]


def test_brute_force_with_sets(orc):
    """Small random collections with heavy sharing: the rule evaluated with
    Python sets pair by pair."""
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(2, 40))
        lists = [sorted(set(rng.integers(0, 60, int(rng.integers(1, 10))).tolist())) for _ in range(n)]
        h = _tracks(lists)
        chi2 = rng.integers(0, 5, n).astype(float)
        ev = rng.integers(0, 2, n)
        st = np.where(rng.random(n) < 0.1, 8, 0)
        frac = float(rng.choice([0.3, 0.5, 0.75]))
        keep = orc.dedup(h, chi2, st, ev, frac=frac)
        want = np.ones(n, bool)
        for j, i in itertools.permutations(range(n), 2):
            if st[i] or st[j] or ev[i] != ev[j]:
                continue
            sh = len(set(lists[i]) & set(lists[j]))
            mn = min(len(lists[i]), len(lists[j]))
            if mn == 0 or sh < frac * mn:
                continue
            ki = (-len(lists[i]), np.float32(chi2[i]), i)
            kj = (-len(lists[j]), np.float32(chi2[j]), j)
            if ki < kj:
                want[j] = False
        assert np.array_equal(keep, want), trial


def test_overlap_events_found_without_cleaning(orc):
    """Module-overlap events (2 x 800 tracks, up to 8 seeds per particle)
    found without seed cleaning: the found collection holds about 2.2 tracks
    per particle; after duplicate removal nearly every particle keeps exactly
    one, no kept pair is a duplicate, and a kept track has at least as many
    hits as any removed track of its particle."""
    geom, evs, ovls = EO.overlap_find_events(n_events=2, n_tracks=800, n_noise=20_000)
    inp = EO.overlap_inputs(evs, ovls)
    o = CM.oracle_find_events(orc, geom, evs, inp)
    keep = orc.dedup(o["hits"], o["chi2"], o["status"], inp["seed_event"])
    key = inp["seed_event"].astype(np.int64) * 100_000 + inp["seed_track"]
    _, inv = np.unique(key, return_inverse=True)
    ok = o["status"] == 0
    per = np.bincount(inv[ok])
    kept = np.bincount(inv[ok], weights=keep[ok])
    print(f"found tracks per particle {per.mean():.2f}; kept per particle {kept.mean():.3f}; "
          f"particles with one kept {(kept == 1).mean():.4f}")
    assert per.mean() > 2.0
    assert (kept >= 1).mean() > 0.995
    assert kept.mean() < 1.02
    nh = (o["hits"] >= 0).sum(axis=1)
    for g in np.nonzero(kept >= 1)[0][:500]:
        m = np.nonzero((inv == g) & ok)[0]
        assert nh[m[keep[m]]].max() >= nh[m].max()
