"""Parity at the sizes the bench times: the fused fit of the 1M-track sets
built exactly as bench.py builds them (the parametrised-field set and the
material-map set), launched as bench.py launches them, with 2,000 sampled
tracks compared one by one against the FP64 oracle."""
import numpy as np
import pytest

import bench
from tests import common as CM

pytestmark = pytest.mark.gpu

N = 1_000_000


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_02253_amd as K
    return K


def _gpu_fit(K, ctx, ld, hits_np, lseq_np, hidx_np, n):
    import torch
    hits = K.Hits(hits_np["x"], hits_np["y"], hits_np["z"], hits_np["su"], hits_np["sv"],
                  hits_np["layer"])
    lseq = torch.as_tensor(lseq_np, device="cuda")
    hidx = torch.as_tensor(hidx_np, device="cuda")
    t = K.Tracks(n, ld)
    ctx.seed(hits, hidx[:3].contiguous(), t)
    ctx.fit(t, hits, lseq, hidx, 10)
    torch.cuda.synchronize()
    return t.numpy()


def _oracle_sample(orc, cfg, ld, hits_np, lseq_np, hidx_np, rows):
    """Oracle seed and fit of the sampled tracks from the same arrays."""
    n = rows.size
    h = {k: hits_np[k] for k in ("x", "y", "z", "su", "sv")}
    seq_layer = lseq_np[:, rows].T.copy()
    seq_hit = hidx_np[:, rows].T.copy()
    par0, cov0 = np.zeros((n, 6)), np.zeros((n, 21))
    for i in range(n):
        hs = [np.array([h["x"][j], h["y"][j], h["z"][j]], np.float64) for j in seq_hit[i, :3]]
        par0[i], cov0[i] = orc.seed(*hs)
    return orc.fit(cfg, h, seq_layer, seq_hit, par0, cov0, n_threads=8)


def _sample(lseq, seed):
    """2,000 tracks with at least the three seed hits."""
    ok = np.nonzero(lseq[2, :N] >= 0)[0]
    return np.sort(np.random.default_rng(seed).choice(ok, 2000, replace=False))


def _compare(g, o, rows, label, sens_fn):
    gs = {k: g[k][rows] for k in ("par", "chi2", "status")}
    CM.check_fit_params(gs, o, label, sens_fn)


def _sens_fn(orc, cfg, ld, hits_np, lseq_np, hidx_np, rows, trials=4):
    """One-ulp sensitivity of the oracle's fit of sampled tracks (indices
    into rows): refits with every hit coordinate of the track moved by one
    float32 ulp in a random direction."""
    def f(idx):
        rng = np.random.default_rng(11)
        base = _oracle_sample(orc, cfg, ld, hits_np, lseq_np, hidx_np, rows[idx])
        sens = np.zeros(len(idx))
        for _ in range(trials):
            hp = dict(hits_np)
            for k in ("x", "y", "z"):
                a = np.array(hits_np[k], np.float32)
                sel = hidx_np[:, rows[idx]]
                sel = sel[sel >= 0]
                to = np.where(rng.random(sel.size) < 0.5, np.float32(np.inf), np.float32(-np.inf))
                a[sel] = np.nextafter(a[sel], to)
                hp[k] = a
            o1 = _oracle_sample(orc, cfg, ld, hp, lseq_np, hidx_np, rows[idx])
            sens = np.maximum(sens, CM.par_error(o1["par"].copy(), base["par"]).max(axis=1))
        return sens
    return f


def test_field_fit_bench_set(K, orc):
    geom, ld, hits, lseq, hidx, _, _ = bench.build_field_fit_set(N)
    ctx = K.Context(geom, field_z0=bench.FIELD_Z0, field_step=bench.FIELD_STEP)
    g = _gpu_fit(K, ctx, ld, hits, lseq, hidx, N)
    rows = _sample(lseq, 7)
    cfg = orc.Config(geom, field_z0=bench.FIELD_Z0, field_step=bench.FIELD_STEP)
    _compare(g, _oracle_sample(orc, cfg, ld, hits, lseq, hidx, rows), rows, "field fit set",
             _sens_fn(orc, cfg, ld, hits, lseq, hidx, rows))


def test_material_fit_bench_set(K, orc):
    import eventgen.material as EM
    fgeom, fmat, fev = EM.eloss_sample(n_tracks=100_000, seed=24)
    ld, hits, lseq, hidx = bench.tile_fit_set(fev, N)
    ctx = K.Context(fgeom)
    ctx.set_material(fmat)
    g = _gpu_fit(K, ctx, ld, hits, lseq, hidx, N)
    rows = _sample(lseq, 8)
    cfg = orc.Config(fgeom, material_map=fmat)
    _compare(g, _oracle_sample(orc, cfg, ld, hits, lseq, hidx, rows), rows, "material fit set",
             _sens_fn(orc, cfg, ld, hits, lseq, hidx, rows))


def test_large_find_set(K, orc):
    """The finding pass over the bench's 512-event set (the 64-event batch
    replicated eight times at distinct addresses), replayed as the bench
    replays it: every copy gives the first copy's results bit for bit, and
    2,000 sampled seeds of the first copy match the FP64 oracle (hit lists
    under the finding tests' tie rule, parameters at the parity bars)."""
    import torch
    import eventgen as E
    from paper_1906_02253_amd import pipeline
    geom, evs = E.batch_events()
    big = list(evs) * bench.LARGE_COPIES
    inp = E.find_inputs(big)
    ctx = K.Context(geom)
    fp = pipeline.FindProblem(ctx, inp)
    fp.run_batched()
    fp.run_batched()
    torch.cuda.synchronize()
    g = fp.results()
    ns1 = int((inp["seed_event"] < len(evs)).sum())
    assert g["hits"].shape[0] == bench.LARGE_COPIES * ns1
    for c in range(1, bench.LARGE_COPIES):
        sl = slice(c * ns1, (c + 1) * ns1)
        off = int(inp["event_off"][c * len(evs)])
        gh = np.where(g["hits"][sl] >= 0, g["hits"][sl] - off, -1)
        assert np.array_equal(gh, g["hits"][:ns1]), c
        for k in ("par", "cov", "chi2", "ndf", "status"):
            assert np.array_equal(g[k][sl], g[k][:ns1]), (c, k)
    rows = np.sort(np.random.default_rng(9).choice(ns1, 2000, replace=False))
    inp1 = E.find_inputs(evs)
    sub = {k: (v[rows] if k in ("seed_hits", "seed_hits_local", "seed_event", "seed_track",
                                "seed_layers") and hasattr(v, "shape") and v.shape[0] == ns1
               else v) for k, v in inp1.items()}
    o = CM.oracle_find_events(orc, geom, evs, sub, n_threads=16)
    gs = {k: g[k][rows] for k in ("hits", "par", "cov", "chi2", "ndf", "status")}
    n_same, n_exc, bad = CM.compare_find(gs, o)
    print(f"512-event set: copies identical; sampled {n_same}/2000 identical, {n_exc} excused")
    assert bad.size == 0 and n_exc <= 2
    CM.check_find_params(gs, o, "512-event set", lambda s: CM.oracle_sensitivity(
        orc, geom, evs, sub, s))
