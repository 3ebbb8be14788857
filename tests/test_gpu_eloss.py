"""GPU parity with an r-z material map (scattering from the map's cell at
each crossing, mean ionisation energy loss) against the FP64 oracle:
propagation, the fit and finding, on tracks simulated with scattering and
energy loss from the same map.  Tolerances as in tests/common.py; the
all-FP64 path to rounding."""
import numpy as np
import pytest

import eventgen as E
import eventgen.material as EM
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


@pytest.fixture(scope="module")
def sample():
    return EM.eloss_sample(n_tracks=3000, seed=22)


def _fit(K, ctx, ev, flags=0):
    import torch
    n = ev.n_tracks
    ld = CM.ld_of(n)
    hits = K.Hits.from_event(ev)
    sh = torch.as_tensor(CM.soa_int(ev.seq_hit[:, :3], ld), device="cuda")
    lseq = torch.as_tensor(CM.soa_int(ev.seq_layer, ld), device="cuda")
    hidx = torch.as_tensor(CM.soa_int(ev.seq_hit, ld), device="cuda")
    t = K.Tracks(n, ld, flags & 3)
    ctx.seed(hits, sh, t, flags)
    ctx.fit(t, hits, lseq, hidx, ev.seq_layer.shape[1], flags)
    torch.cuda.synchronize()
    return t.numpy()


def _oracle_fit(orc, geom, mat, ev):
    par0, cov0 = orc.seeds_for_event(ev)
    cfg = orc.Config(geom, material_map=mat)
    return orc.fit(cfg, dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv), ev.seq_layer, ev.seq_hit,
                   par0, cov0, n_threads=8)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_map_propagate_parity(K, orc, sample, prec):
    """States at their crossing of layer k (after that layer's material)
    propagated to layer k+1 with the map's scattering and energy loss."""
    import torch
    geom, mat, ev = sample
    rng = np.random.default_rng(5)
    nh = ev.n_track_hits()
    rows = [(t, rng.integers(0, nh[t] - 1)) for t in range(ev.n_tracks) if nh[t] >= 2]
    par = np.array([ev.truth_out[t, k] for t, k in rows])
    tgt = np.array([ev.seq_layer[t, k + 1] for t, k in rows], np.int32)
    n = par.shape[0]
    cov = np.tile(orc.pack(np.diag([1e-4, 1e-4, 2e-3, 1e-4, 1e-5, 1e-5])), (n, 1))
    ld = CM.ld_of(n)
    pflag = K.PREC_FP64 if prec == "fp64" else K.PREC_MIXED
    ctx = K.Context(geom)
    ctx.set_material(mat)
    t = K.Tracks.from_numpy(par, cov, prec=pflag, ld=ld)
    target = torch.full((ld,), -1, dtype=torch.int32, device="cuda")
    target[:n] = torch.as_tensor(tgt, device="cuda")
    ctx.propagate(t, target, flags=pflag)
    torch.cuda.synchronize()
    g = t.numpy()
    cfg = orc.Config(geom, material_map=mat)
    op, oc = np.zeros((n, 6)), np.zeros((n, 21))
    for i in range(n):
        st, op[i], oc[i], _, _ = orc.propagate(cfg, tgt[i], par[i], cov[i], noise=True)
        assert st == 0
    assert (g["status"] == 0).all()
    err = CM.par_error(g["par"], op)
    # energy loss changed c by a visible amount relative to the tolerance
    assert np.abs(op[:, 3] / par[:, 3] - 1).mean() > 10 * CM.REL
    rel = 1e-9 if prec == "fp64" else CM.REL
    print(f"{prec}: {n} propagations, max rel par err {err.max():.2e}")
    assert err.max() < rel, err.max(axis=0)
    crel = 1e-9 if prec == "fp64" else 1e-3
    for idx in (0, 6, 11, 15, 18, 20):
        assert np.quantile(np.abs(g["cov"][:, idx] / oc[:, idx] - 1), 0.999) < crel, idx


def test_map_fit_parity(K, orc, sample):
    geom, mat, ev = sample
    o = _oracle_fit(orc, geom, mat, ev)
    ctx = K.Context(geom)
    ctx.set_material(mat)
    g = _fit(K, ctx, ev)
    assert np.array_equal(g["status"], o["status"])
    ok = o["status"] == 0
    err = CM.par_error(g["par"][ok], o["par"][ok])
    cerr = CM.chi2_error(g["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
    print(f"mixed: max rel par err {err.max():.2e}, chi2 err / tol {cerr.max() / CM.CHI2_REL:.3f}")
    assert err.max() < CM.REL, err.max(axis=0)
    assert cerr.max() < CM.CHI2_REL
    g64 = _fit(K, ctx, ev, K.PREC_FP64)
    e64 = CM.par_error(g64["par"][ok], o["par"][ok])
    print(f"fp64: max rel par err {e64.max():.2e}")
    assert e64.max() < 1e-9
    # one launch per step (FP32 state through HBM) with the map too
    b = _fit(K, ctx, ev, K.PER_LAYER)
    eb = CM.par_error(b["par"][ok], o["par"][ok])
    cb = CM.chi2_error(b["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
    print(f"per layer: max rel par err {eb.max():.2e}, chi2 err / tol {cb.max() / CM.CHI2_REL:.3f}")
    assert np.array_equal(b["status"], o["status"])
    assert eb.max() < CM.REL and cb.max() < CM.CHI2_REL


def test_map_removed_restores_plain(K, sample):
    """set_material(None) gives back exactly the results of a context that
    never had a map (the layers' own x0, no energy loss)."""
    geom, mat, ev = sample
    geom2 = [dict(L, x0=0.03) for L in geom]
    a = _fit(K, K.Context(geom2), ev)
    ctx = K.Context(geom2)
    ctx.set_material(mat)
    m = _fit(K, ctx, ev)
    ctx.set_material(None)
    b = _fit(K, ctx, ev)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert not np.array_equal(a["par"], m["par"])


def test_bad_map_rejected(K, sample):
    geom, mat, _ = sample
    ctx = K.Context(geom)
    for bad in (dict(mat, r_max=-1.0), dict(mat, z_min=400.0), dict(mat, x0=-mat["x0"] - 1),
                dict(mat, xi=np.full_like(mat["xi"], np.nan))):
        with pytest.raises(K.KFError):
            ctx.set_material(bad)


@pytest.mark.parametrize("batched", [False, True])
def test_map_find_matches_oracle(K, orc, batched):
    """Finding on 3 events of 800 tracks and 50,000 noise hits, material and
    energy loss from the map: hit lists against the FP64 oracle under the
    finding tests' tie rules; eager and as the captured graph (recaptured
    when the map changes)."""
    import torch
    geom, mat, evs = EM.eloss_find_events(n_events=3, n_tracks=800, n_noise=50_000)
    inp = E.find_inputs(evs)
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    if batched:
        fp.run_batched()                 # captured without a map, then with it
        ctx.set_material(mat)
        fp.run_batched()
    else:
        ctx.set_material(mat)
        fp.run()
    torch.cuda.synchronize()
    g = fp.results()
    o = CM.oracle_find_events(orc, geom, evs, inp, material_map=mat)
    n_same, n_exc, bad = CM.compare_find(g, o)
    print(f"map find: {n_same}/{g['hits'].shape[0]} identical, {n_exc} excused, {bad.size} unexplained")
    assert bad.size == 0
    assert n_exc <= CM.MAX_EXCUSED_FRAC * max(g["hits"].shape[0], 1000)
    CM.check_find_params(g, o, "params", lambda s: CM.oracle_sensitivity(
        orc, geom, evs, inp, s, material_map=mat))


def _coarse_map(geom, base=0.04, n_r=50, n_z=50):
    """A smaller grid (50 x 50 cells over the same r-z area) with the same
    kind of thickness profile along each barrel; no barrel radius falls on a
    cell edge (2.4 cm rows)."""
    r_max, z_min, z_max = EM.R_MAX, EM.Z_MIN, EM.Z_MAX
    dr, dz = r_max / n_r, (z_max - z_min) / n_z
    zc = z_min + (np.arange(n_z) + 0.5) * dz
    x0 = np.zeros((n_r, n_z), np.float32)
    for L in geom:
        ir = int(np.floor(L["r_or_z"] / dr))
        u = np.clip(zc / max(abs(L["lo"]), abs(L["hi"])), -1, 1)
        x0[ir, :] = base * (1 + 0.5 * u ** 2)
    return dict(r_max=r_max, z_min=z_min, z_max=z_max, x0=x0, xi=(x0 * EM.X0_SI).astype(np.float32))


def test_map_swap_recaptures_graph(K, orc):
    """The captured pass takes the map's pointers and sizes by value: setting
    another map (same cell count, other values; then a smaller grid) makes the
    next kf_find_batched capture again, and every pass matches the FP64 oracle
    run with the map then set."""
    import torch
    geom, mat, evs = EM.eloss_find_events(n_events=2, n_tracks=600, n_noise=30_000)
    inp = E.find_inputs(evs)
    ctx = K.Context(geom)
    fp = K.pipeline.FindProblem(ctx, inp)
    mat_b = dict(mat, x0=(mat["x0"] * 1.8).astype(np.float32),
                 xi=(mat["xi"] * 1.8).astype(np.float32))
    prev = None
    for m, label in ((mat, "map"), (mat_b, "same cells, other values"), (_coarse_map(geom), "smaller grid")):
        ctx.set_material(m)
        for rep in range(2):
            fp.out_hits.fill_(-7)
            fp.run_batched()
            torch.cuda.synchronize()
        g = fp.results()
        o = CM.oracle_find_events(orc, geom, evs, inp, material_map=m)
        n_same, n_exc, bad = CM.compare_find(g, o)
        print(f"{label}: {n_same}/{g['hits'].shape[0]} identical, {n_exc} excused, {bad.size} unexplained")
        assert bad.size == 0
        CM.check_find_params(g, o, label, lambda s: CM.oracle_sensitivity(
            orc, geom, evs, inp, s, material_map=m))
        if prev is not None:
            assert not np.array_equal(prev, g["par"])
        prev = g["par"].copy()


def test_map_find_learned_start_matches_oracle(K, orc):
    """Finding with the map and the learned start of the barrel solves (its
    own kernel instance; a freshly initialised network, so most guesses fall
    back to the straight line): the solve stays exact, so the hit lists match
    the FP64 oracle's plain finder with the same map."""
    import torch
    geom, mat, evs = EM.eloss_find_events(n_events=2, n_tracks=600, n_noise=30_000)
    inp = E.find_inputs(evs)
    ctx = K.Context(geom)
    ctx.set_find_config(64, False)
    ctx.set_material(mat)
    ctx.mlp_load(E.mlp_init(5))
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run(K.INIT_MLP)
    torch.cuda.synchronize()
    g = fp.results()
    assert g["counters"][5] > 0                  # guesses were made
    o = CM.oracle_find_events(orc, geom, evs, inp, material_map=mat)
    n_same, n_exc, bad = CM.compare_find(g, o)
    print(f"learned map find: {n_same}/{g['hits'].shape[0]} identical, {n_exc} excused, "
          f"{bad.size} unexplained; guesses {g['counters'][5]}, fallbacks {g['counters'][6]}")
    assert bad.size == 0
    assert n_exc <= CM.MAX_EXCUSED_FRAC * max(g["hits"].shape[0], 1000)
    CM.check_find_params(g, o, "params", lambda s: CM.oracle_sensitivity(
        orc, geom, evs, inp, s, material_map=mat))


def test_map_energy_loss_cap(K, orc):
    """A cell far thicker than any detector (xi ~ 2 kg/cm^2): the loss is capped
    at half the kinetic energy on both sides and the state stays finite."""
    import torch
    geom = [dict(kind=0, r_or_z=50.0, lo=-100.0, hi=100.0, x0=0.0, nbin_phi=64, nbin_2=16,
                 win_su=0.01, win_sv=0.05)]
    x0 = np.full((250, 250), 0.05, np.float32)
    mat = dict(r_max=120.0, z_min=-300.0, z_max=300.0, x0=x0,
               xi=np.full((250, 250), 2000.0, np.float32))
    par = np.array([[0.0, 0.0, 0.0, 1 / 0.4, 0.3, 1.3], [0.0, 0.0, 0.0, -1 / 2.0, -1.0, 1.7]])
    cov = np.tile(orc.pack(np.eye(6) * 1e-5), (2, 1))
    ctx = K.Context(geom)
    ctx.set_material(mat)
    t = K.Tracks.from_numpy(par, cov, prec=K.PREC_FP64, ld=64)
    target = torch.full((64,), -1, dtype=torch.int32, device="cuda")
    target[:2] = 0
    ctx.propagate(t, target, flags=K.PREC_FP64)
    torch.cuda.synchronize()
    g = t.numpy()
    cfg = orc.Config(geom, material_map=mat)
    for i in range(2):
        st, q, Q, _, _ = orc.propagate(cfg, 0, par[i], cov[i], noise=True)
        assert st == 0 and g["status"][i] == 0
        assert np.all(np.isfinite(g["par"][i]))
        p0 = 1 / (abs(par[i, 3]) * np.sin(par[i, 5]))
        p1 = 1 / (abs(q[3]) * np.sin(q[5]))
        E0, E1 = np.hypot(p0, 0.13957), np.hypot(p1, 0.13957)
        assert E1 == pytest.approx(E0 - 0.5 * (E0 - 0.13957), rel=1e-12)   # the cap
        assert CM.par_error(g["par"][i:i + 1], q[None])[0].max() < 1e-9
