"""GPU parity of kf_seed / kf_propagate / kf_fit against the FP64 oracle.

Tolerances (stated in tests/common.py): parameters 1e-4 relative with floors
(1 cm, 0.01 1/GeV, 1 rad), chi2 1e-3 relative to max(chi2, ndf).
"""
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
    return K


def _gpu_inputs(K, ev, ld):
    import torch
    hits = K.Hits.from_event(ev)
    sh = torch.as_tensor(CM.soa_int(ev.seq_hit[:, :3], ld), device="cuda")
    lseq = torch.as_tensor(CM.soa_int(ev.seq_layer, ld), device="cuda")
    hidx = torch.as_tensor(CM.soa_int(ev.seq_hit, ld), device="cuda")
    return hits, sh, lseq, hidx


def _gpu_fit(K, geom, ev, flags=0, ld=None):
    import torch
    n = ev.n_tracks
    ld = ld or CM.ld_of(n)
    ctx = K.Context(geom)
    hits, sh, lseq, hidx = _gpu_inputs(K, ev, ld)
    t = K.Tracks(n, ld, flags & 3)
    ctx.seed(hits, sh, t, flags)
    ctx.fit(t, hits, lseq, hidx, ev.seq_layer.shape[1], flags)
    torch.cuda.synchronize()
    return t.numpy()


def _oracle_fit(orc, geom, ev):
    cfg = orc.Config(geom)
    par0, cov0 = orc.seeds_for_event(ev)
    hits = dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv)
    return orc.fit(cfg, hits, ev.seq_layer, ev.seq_hit, par0, cov0, n_threads=8)


def test_seed_parity(K, orc):
    import torch
    geom, ev = E.fit_sample(n_tracks=1000, seed=0)
    ld = CM.ld_of(ev.n_tracks)
    ctx = K.Context(geom)
    hits, sh, _, _ = _gpu_inputs(K, ev, ld)
    t = K.Tracks(ev.n_tracks, ld)
    ctx.seed(hits, sh, t)
    torch.cuda.synchronize()
    g = t.numpy()
    par0, cov0 = orc.seeds_for_event(ev)
    err = CM.par_error(g["par"], par0)
    assert err.max() < CM.REL, err.max(axis=0)
    assert np.allclose(g["cov"], cov0)


def test_fit_parity_config0(K, orc):
    """1,000 helix tracks, ten barrel layers, no material: mixed-precision GPU
    fit vs the FP64 oracle (several 256-lane blocks and a ragged tail)."""
    geom, ev = E.fit_sample(n_tracks=1000, seed=0)
    g = _gpu_fit(K, geom, ev)
    o = _oracle_fit(orc, geom, ev)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["ndf"], o["ndf"])
    ok = o["status"] == 0
    err = CM.par_error(g["par"][ok], o["par"][ok])
    print("max rel par err:", err.max(axis=0))
    assert err.max() < CM.REL
    cerr = CM.chi2_error(g["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
    print("max chi2 err / tol:", cerr.max() / CM.CHI2_REL)
    assert cerr.max() < CM.CHI2_REL
    # covariance: diagonal within 1e-3 relative
    for i, j in [(0, 0), (2, 2), (3, 3), (4, 4), (5, 5)]:
        idx = i * (11 - i) // 2 + j
        rel = np.abs(g["cov"][ok, idx] / o["cov"][ok, idx] - 1)
        assert np.quantile(rel, 0.999) < 1e-3, (i, rel.max())


def test_fit_fp64_equals_oracle(K, orc):
    """All-FP64 GPU path: same algorithm as the oracle, differences only from
    rounding order."""
    geom, ev = E.fit_sample(n_tracks=1000, seed=0)
    g = _gpu_fit(K, geom, ev, flags=K.PREC_FP64)
    o = _oracle_fit(orc, geom, ev)
    ok = o["status"] == 0
    err = CM.par_error(g["par"][ok], o["par"][ok])
    print("fp64 max rel err:", err.max())
    assert err.max() < 1e-9
    assert np.abs(g["chi2"][ok] - o["chi2"][ok]).max() < 1e-7 * max(1, o["chi2"].max())


def test_fit_per_layer_matches_oracle(K, orc):
    """One launch per step (the state through HBM in FP32 between steps)
    against the FP64 oracle at the parity bars, on the fit workload and on the
    precision workload's tracks (its first 20,000); the fused fit keeps the
    state in registers between steps, so the two differ by storage rounding."""
    for geom, ev in (E.fit_sample(n_tracks=777, seed=4), E.precision_sample(20_000)):
        a = _gpu_fit(K, geom, ev, flags=K.PER_LAYER)
        o = _oracle_fit(orc, geom, ev)
        assert np.array_equal(a["status"], o["status"])
        assert np.array_equal(a["ndf"], o["ndf"])
        ok = o["status"] == 0
        err = CM.par_error(a["par"][ok], o["par"][ok])
        cerr = CM.chi2_error(a["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
        print(f"per layer: max rel par err {err.max(axis=0)}, chi2 err / tol "
              f"{cerr.max() / CM.CHI2_REL:.3f}")
        assert err.max() < CM.REL and cerr.max() < CM.CHI2_REL


def test_fit_ld_padding_and_empty(K):
    import torch
    geom, ev = E.fit_sample(n_tracks=130, seed=6)
    a = _gpu_fit(K, geom, ev)
    b = _gpu_fit(K, geom, ev, ld=512)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ctx = K.Context(geom)
    t = K.Tracks(0, 64)
    hits = K.Hits.from_event(ev)
    z = torch.zeros((10, 64), dtype=torch.int32, device="cuda")
    ctx.fit(t, hits, z, z, 10)
    torch.cuda.synchronize()


def test_bad_indices_flagged(K):
    import torch
    geom, ev = E.fit_sample(n_tracks=64, seed=6)
    ld = 64
    ctx = K.Context(geom)
    hits, sh, lseq, hidx = _gpu_inputs(K, ev, ld)
    t = K.Tracks(64, ld)
    ctx.seed(hits, sh, t)
    lseq[3, 5] = 99
    hidx[4, 7] = ev.n_hits + 5
    ctx.fit(t, hits, lseq, hidx, ev.seq_layer.shape[1])
    torch.cuda.synchronize()
    st = t.status.cpu().numpy()
    assert st[5] & K.ST_BADINPUT and st[7] & K.ST_BADINPUT
    with pytest.raises(K.KFError):
        bad = K.Tracks(10, 64)
        bad.ld = 63
        ctx.fit(bad, hits, lseq, hidx, 10)


def test_propagate_parity(K, orc):
    """kf_propagate (mixed) vs oracle: states at their crossing of layer k,
    propagated to layer k+1 with material noise."""
    import torch
    geom, evs = E.find_events(n_events=1, n_tracks=3000, n_noise=0, seed=12)
    ev = evs[0]
    cfg = orc.Config(geom)
    rng = np.random.default_rng(3)
    rows = []
    for t in range(ev.n_tracks):
        nh = ev.n_track_hits()[t]
        if nh < 2:
            continue
        k = rng.integers(0, nh - 1)
        rows.append((ev.truth_out[t, k], ev.seq_layer[t, k + 1]))
    n = len(rows)
    ld = CM.ld_of(n)
    # the oracle starts from the same FP32-stored inputs the kernel reads
    par = np.array([r[0] for r in rows]).astype(np.float32).astype(np.float64)
    P = np.diag([1e-4, 1e-4, 2e-3, 1e-4, 1e-5, 1e-5])
    cov = np.tile(orc.pack(P), (n, 1)).astype(np.float32).astype(np.float64)
    tgt = np.array([r[1] for r in rows], np.int32)
    t = K.Tracks.from_numpy(par, cov, ld=ld)
    target = torch.full((ld,), -1, dtype=torch.int32, device="cuda")
    target[:n] = torch.as_tensor(tgt, device="cuda")
    plen = torch.zeros(ld, device="cuda")
    its = torch.zeros(ld, dtype=torch.int32, device="cuda")
    ctx = K.Context(geom)
    ctx.propagate(t, target, plen, its)
    torch.cuda.synchronize()
    g = t.numpy()
    op = np.zeros((n, 6))
    oc = np.zeros((n, 21))
    os_ = np.zeros(n)
    for i in range(n):
        st, op[i], oc[i], os_[i], _ = orc.propagate(cfg, tgt[i], par[i], cov[i], noise=True)
        assert st == 0
    assert (g["status"] == 0).all()
    err = CM.par_error(g["par"], op)
    print("propagate: max rel par err", err.max(axis=0))
    assert err.max() < CM.REL, err.max(axis=0)
    assert np.abs(plen.cpu().numpy()[:n] - os_).max() < 1e-4 * max(1, os_.max())
    for idx in (0, 6, 11, 15, 18, 20):
        assert np.abs(g["cov"][:, idx] / oc[:, idx] - 1).max() < 1e-3, idx
