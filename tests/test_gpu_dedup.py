"""GPU parity of duplicate removal of found tracks against the FP64 oracle:
the removal alone on synthetic collections (bit-exact keep decisions: the
rule takes integer counts and float chi2 comparisons that both sides make
alike), and finding with removal on module-overlap events, eager and as the
captured graph, with and without seed cleaning."""
import numpy as np
import pytest

import eventgen.overlap as EO
from tests import common as CM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_02253_amd as K
    from paper_1906_02253_amd import pipeline
    K.pipeline = pipeline
    return K


def _gpu_dedup(K, s, calls=1, frac=0.5):
    import torch
    import eventgen as E
    n, nl = s["hits"].shape
    geom = E.geometry.barrel10(x0=0.0)[:nl]
    ld = CM.ld_of(n)
    t = K.Tracks(n, ld)
    t.chi2[:n] = torch.as_tensor(s["chi2"], device="cuda")
    t.status[:n] = torch.as_tensor(s["status"].astype(np.int32), device="cuda")
    rows = torch.as_tensor(s["hits"], device="cuda")
    ev = torch.as_tensor(s["event"], device="cuda")
    nh = s["n_hits"]
    hits = K.Hits(*(np.zeros(nh, np.float32) for _ in range(5)), np.zeros(nh, np.int32))
    ctx = K.Context(geom, dup_frac=frac)
    for _ in range(calls):
        ctx.remove_duplicates(hits, t, rows, ev)
    torch.cuda.synchronize()
    return t.status[:n].cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("frac", [0.5, 0.3, 0.8])
def test_dedup_parity_synthetic(K, orc, frac):
    s = EO.track_set(n=5000, n_events=3, seed=13)
    st = _gpu_dedup(K, s, frac=frac)
    keep = orc.dedup(s["hits"], s["chi2"].astype(np.float64), s["status"].astype(np.int32),
                     s["event"], frac=frac)
    g_keep = (st & K.ST_DUPTRACK) == 0
    print(f"frac {frac}: kept {keep.sum()} of {keep.size}, mismatches {(g_keep != keep).sum()}")
    assert 0.2 * keep.size < keep.sum() < 0.9 * keep.size
    assert np.array_equal(g_keep, keep)
    bad = s["status"] != 0
    assert np.array_equal(st[bad], s["status"][bad].astype(np.int64))


def test_dedup_repeatable(K):
    s = EO.track_set(n=3000, n_events=2, seed=14)
    assert np.array_equal(_gpu_dedup(K, s, calls=1), _gpu_dedup(K, s, calls=3))


@pytest.mark.parametrize("mode", ["eager", "graph", "graph+clean"])
def test_find_with_dedup_matches_oracle(K, orc, mode):
    """Overlap events (3 x 800 tracks, 30% overlaps, 50,000 noise hits):
    found tracks removed on the GPU == oracle (its finder's lists, then its
    removal), the kept tracks one per particle almost always."""
    import torch
    geom, evs, ovls = EO.overlap_find_events(n_events=3, n_tracks=800, n_noise=50_000)
    inp = EO.overlap_inputs(evs, ovls)
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    flags = K.REMOVE_DUPLICATES | (K.CLEAN_SEEDS if mode == "graph+clean" else 0)
    if mode == "eager":
        fp.seed_fit()
        fp.find(flags)
    else:
        fp.run_batched(flags)
        fp.run_batched(flags)
    torch.cuda.synchronize()
    g = fp.results()
    if mode == "graph+clean":
        from tests.test_gpu_clean import _oracle_clean_find
        ckeep, _, kept, o_sub = _oracle_clean_find(orc, geom, evs, inp)
        o = {k: np.zeros((ckeep.size,) + v.shape[1:], v.dtype) for k, v in o_sub.items()
             if isinstance(v, np.ndarray)}
        for k in o:
            o[k][kept] = o_sub[k]
        o["status"][~ckeep] = K.ST_DUPLICATE
        o["hits"][~ckeep] = -1
    else:
        o = CM.oracle_find_events(orc, geom, evs, inp)
    same = (g["hits"] == o["hits"]).all(axis=1) | (o["status"] != 0)
    assert same.mean() > 0.99
    keep = orc.dedup(o["hits"], o["chi2"], o["status"], inp["seed_event"])
    part = o["status"] == 0
    g_keep = (g["status"] & K.ST_DUPTRACK) == 0
    mism = np.nonzero(part & (g_keep != keep))[0]
    print(f"{mode}: {part.sum()} taking part, oracle keeps {keep[part].sum()}, GPU keeps "
          f"{g_keep[part].sum()}, mismatches {mism.size}")
    assert mism.size <= (~same).sum()
    key = inp["seed_event"].astype(np.int64) * 100_000 + inp["seed_track"]
    _, inv = np.unique(key, return_inverse=True)
    kept_pp = np.bincount(inv[part], weights=(g_keep & part)[part])
    assert (kept_pp >= 1).mean() > 0.99 and kept_pp.mean() < 1.05


def test_overlap_batch_full(K, orc):
    """The bench's overlap batch at full size (64 events, 247,857 seeds) with
    seed cleaning and duplicate removal in the captured pass: seeds removed,
    hit lists of the searched seeds and found tracks removed, against the
    oracle's seed fit, cleaning, finding and removal."""
    import torch
    from tests.test_gpu_clean import _oracle_clean_find
    geom, evs, ovls = EO.overlap_batch(seed=9)
    inp = EO.overlap_inputs(evs, ovls)
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    flags = K.CLEAN_SEEDS | K.REMOVE_DUPLICATES
    fp.run_batched(flags)
    fp.run_batched(flags)
    torch.cuda.synchronize()
    g = fp.results()
    ckeep, ctie, kept, o_sub = _oracle_clean_find(orc, geom, evs, inp)
    g_ckeep = (g["status"] & K.ST_DUPLICATE) == 0
    print(f"cleaning: {ckeep.size} seeds, oracle keeps {ckeep.sum()}, GPU keeps {g_ckeep.sum()}, "
          f"ties {ctie.sum()}, mismatches {(g_ckeep != ckeep).sum()}")
    assert np.array_equal(g_ckeep[~ctie], ckeep[~ctie])
    both = np.nonzero(ckeep & g_ckeep)[0]
    pos = np.searchsorted(kept, both)
    n_same, n_exc, bad = CM.compare_find(dict(hits=g["hits"][both]),
                                         dict(hits=o_sub["hits"][pos], tie=o_sub["tie"][pos]))
    print(f"searched on both: {both.size}, identical {n_same}, excused {n_exc}, unexplained {bad.size}")
    assert bad.size == 0
    # removal on the oracle's own collection (seeds it removed take no part)
    n = ckeep.size
    o_hits = np.full((n, len(geom)), -1, np.int64)
    o_chi2, o_st = np.zeros(n), np.full(n, K.ST_DUPLICATE, np.int64)
    o_hits[kept], o_chi2[kept], o_st[kept] = o_sub["hits"], o_sub["chi2"], o_sub["status"]
    dkeep = orc.dedup(o_hits, o_chi2, o_st, inp["seed_event"])
    part = o_st == 0
    g_keep = (g["status"] & K.ST_DUPTRACK) == 0
    same = np.zeros(n, bool)
    same[both] = (g["hits"][both] == o_sub["hits"][pos]).all(axis=1)
    mism = np.nonzero(part & (g_keep != dkeep))[0]
    print(f"removal: {part.sum()} taking part, oracle keeps {dkeep[part].sum()}, GPU keeps "
          f"{g_keep[part & g_ckeep].sum()}, mismatches {mism.size}")
    assert mism.size <= (part & ~same).sum() + (g_ckeep != ckeep).sum()


def test_dedup_edge_cases(K):
    """No tracks; a single track; tracks without hits (never duplicates)."""
    import torch
    import eventgen as E
    geom = E.geometry.barrel10(x0=0.0)
    ctx = K.Context(geom)
    hits = K.Hits(*(np.zeros(10, np.float32) for _ in range(5)), np.zeros(10, np.int32))
    t = K.Tracks(0, 64)
    z = torch.zeros((64, 10), dtype=torch.int32, device="cuda")
    ctx.remove_duplicates(hits, t, z, z[:, 0].contiguous())
    one = dict(hits=np.array([[0, 1, 2, -1, -1, -1, -1, -1, -1, -1]], np.int32),
               chi2=np.array([1.0], np.float32), status=np.zeros(1, np.uint32),
               event=np.zeros(1, np.int32), n_hits=10)
    assert _gpu_dedup(K, one).tolist() == [0]
    empty = dict(hits=np.full((3, 10), -1, np.int32), chi2=np.ones(3, np.float32),
                 status=np.zeros(3, np.uint32), event=np.zeros(3, np.int32), n_hits=10)
    assert _gpu_dedup(K, empty).tolist() == [0, 0, 0]
