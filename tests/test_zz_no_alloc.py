"""kf_find_noalloc (the finding pass with the library's static scratch, for
callers that cannot allocate) against kf_find on the same inputs: two calls
in a row on one context, the second with a smaller input, each bit for bit
equal to kf_find's results; and a call too large for the static scratch is
refused with an error."""
import numpy as np
import pytest

import eventgen as E
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


def _run(K, ctx, inp, noalloc, flags=0):
    import torch
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.seed_fit(flags)
    fp.out_hits.fill_(-7)
    if noalloc:
        ctx.find_noalloc(fp.hits, fp.event_off, fp.seeds, fp.seed_event, fp.seed_hits,
                         fp.out_hits, fp.out, fp.counters, flags)
    else:
        fp.find(flags)
    torch.cuda.synchronize()
    return fp.results()


def _same(a, b, label):
    for k in ("hits", "par", "cov", "chi2", "ndf", "status", "counters"):
        assert np.array_equal(a[k], b[k]), (label, k)


def test_noalloc_matches_find_twice(K, orc):
    geom, evs = E.find_events(n_events=3, n_tracks=800, n_noise=50_000, seed=1)
    big, small = E.find_inputs(evs), E.find_inputs(evs[:1])
    ctx = K.Context(geom)
    r_big = _run(K, ctx, big, noalloc=True)
    r_small = _run(K, ctx, small, noalloc=True)
    ref_ctx = K.Context(geom)
    _same(r_big, _run(K, ref_ctx, big, noalloc=False), "first call")
    _same(r_small, _run(K, ref_ctx, small, noalloc=False), "second, smaller call")
    # and the results are the oracle's
    o = CM.oracle_find_events(orc, geom, evs[:1], small)
    n_same, n_exc, bad = CM.compare_find(r_small, o)
    assert bad.size == 0


def test_noalloc_with_cleaning_and_removal(K):
    geom, evs = E.find_events(n_events=2, n_tracks=600, n_noise=20_000, seed=3)
    inp = E.find_inputs(evs)
    flags = K.CLEAN_SEEDS | K.REMOVE_DUPLICATES
    a = _run(K, K.Context(geom), inp, noalloc=True, flags=flags)
    b = _run(K, K.Context(geom), inp, noalloc=False, flags=flags)
    _same(a, b, "cleaning and duplicate removal")


def test_noalloc_refuses_oversize(K):
    """A batch whose scratch exceeds the static array is refused before any
    device work (the 64-event batch needs well over 64 MiB)."""
    geom, evs = E.batch_events(n_events=8)
    inp = E.find_inputs(evs)
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.seed_fit()
    with pytest.raises(K.KFError, match="static scratch"):
        ctx.find_noalloc(fp.hits, fp.event_off, fp.seeds, fp.seed_event, fp.seed_hits,
                         fp.out_hits, fp.out, fp.counters)
