"""GPU parity of the batched finding workload: 64 events with track counts
~ Poisson(lambda), lambda ~ U(200, 4000), 60 noise hits per track, barrel
plus 2 x 7 disks, |eta| < 2.5, 0.02 X0 per layer (the full-size batch, all
seeds compared with the FP64 oracle)."""
import numpy as np
import pytest

import eventgen as E
from tests import common as CM
from tests.test_gpu_find import K, _gpu_find, _check_parity, _sens  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg2():
    geom, evs = E.batch_events()
    return geom, evs, E.find_inputs(evs)


def test_batch_parity_full(K, orc, cfg2):
    geom, evs, inp = cfg2
    g = _gpu_find(K, geom, inp)
    o = CM.oracle_find_events(orc, geom, evs, inp)
    _check_parity(g, o, "batch", _sens(orc, geom, evs, inp))
    assert abs(int(g["counters"][0]) - o["n_prop"]) <= 0.01 * o["n_prop"]


def test_batch_widths_identical(K, cfg2):
    geom, evs, inp = cfg2
    ref = _gpu_find(K, geom, inp, 256, True)
    for w, lf in ((64, False), (128, True)):
        r = _gpu_find(K, geom, inp, w, lf)
        for k in ("hits", "par", "chi2", "ndf", "status"):
            assert np.array_equal(r[k], ref[k]), (w, lf, k)


def _same(r, ref, label):
    for k in ("hits", "par", "cov", "chi2", "ndf", "status"):
        assert np.array_equal(r[k], ref[k]), (label, k)


def test_batched_graph_replays_match_eager(K, cfg2):
    """kf_find_batched (seed, seed fit, binning, seed order and the finding
    kernel captured as one graph) gives the eager path's results on every
    replay, with eager work and synchronisations between the replays; a
    smaller input on the same context captures again and matches too."""
    import torch
    geom, evs, inp = cfg2
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run()
    torch.cuda.synchronize()
    ref = fp.results()
    c_eager = ref["counters"].copy()
    assert c_eager[0] > 0
    for rep in range(4):
        fp.out_hits.fill_(-7)
        fp.out.par.zero_()
        fp.counters.zero_()
        fp.run_batched()
        torch.cuda.synchronize()
        r = fp.results()
        _same(r, ref, f"replay {rep}")
        assert np.array_equal(r["counters"], c_eager), rep
        # eager work on the same context between replays
        fp.find()
        torch.cuda.synchronize()
    # a smaller batch (the first 8 events) on the same context
    small_inp = E.find_inputs(evs[:8])
    fs = K.pipeline.FindProblem(ctx, small_inp)
    fs.run()
    torch.cuda.synchronize()
    ref_s = fs.results()
    for rep in range(2):
        fs.out_hits.fill_(-7)
        fs.run_batched()
        torch.cuda.synchronize()
        _same(fs.results(), ref_s, f"small replay {rep}")


def test_batched_phase_timing(K, cfg2):
    import torch
    geom, evs, inp = cfg2
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run_batched()
    ctx.set_timing(3)
    for _ in range(3):
        fp.run_batched()
    fp.run_batched()          # beyond the requested sets: not recorded
    torch.cuda.synchronize()
    ms, n = ctx.timings()
    assert n == 3
    assert all(m > 0 for m in ms), ms
    ctx.set_timing(0)
    fp.run_batched()
    torch.cuda.synchronize()


def test_autotune_keeps_fastest_and_results(K, cfg2):
    """The autotuner times every width and both tile orders, keeps the
    fastest, and the tuned configuration gives the same results."""
    import torch
    geom, evs, inp = cfg2
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run()
    torch.cuda.synchronize()
    ref = fp.results()
    tab = fp.autotune(reps=2)
    print("autotune table (ms):", tab)
    assert len(tab) == 8, tab
    best = min(tab, key=tab.get)
    assert ctx.find_config() == best
    fp.out_hits.fill_(-7)
    fp.run()
    torch.cuda.synchronize()
    _same(fp.results(), ref, "tuned")


def test_batched_edge_cases(K):
    """A single small event through the graph, and an empty seed list."""
    import torch
    rng = np.random.default_rng(91)
    geom = E.geometry.barrel10_disks14(x0=0.02)
    ev = E.make_event(rng, geom, 7, E.pt_power2(0.5, 50.0), 2.5, 20)
    inp = E.find_inputs([ev])
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run()
    torch.cuda.synchronize()
    ref = fp.results()
    fp.out_hits.fill_(-7)
    fp.run_batched()
    fp.run_batched()
    torch.cuda.synchronize()
    _same(fp.results(), ref, "one event")
    # no seeds: nothing to do, no error
    empty = dict(inp)
    for key in ("seed_event", "seed_track"):
        empty[key] = inp[key][:0]
    for key in ("seed_hits", "seed_hits_local", "seed_layers"):
        empty[key] = inp[key][:0]
    fe = K.pipeline.FindProblem(ctx, empty)
    fe.run()
    fe.run_batched()
    torch.cuda.synchronize()
    assert int(fe.counters[0].item()) == 0


def test_batch_steered_full(K, orc, cfg2):
    """The full batch following the five-region layer plans, as the bench's
    steered pass runs it (graph replays), against the FP64 oracle with the
    same plans."""
    import torch
    geom, evs, inp = cfg2
    plans = E.geometry.steering_plans(geom)
    ctx = K.Context(geom)
    ctx.set_find_config(64, False)
    ctx.set_steering(plans)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run_batched()
    fp.run_batched()
    torch.cuda.synchronize()
    g = fp.results()
    o = CM.oracle_find_events(orc, geom, evs, inp, steering=plans)
    _check_parity(g, o, "batch steered", _sens(orc, geom, evs, inp, steering=plans))
