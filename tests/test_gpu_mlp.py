"""GPU checks of the learned path-length guess.

* Forward pass and gradient of the bf16 matrix-core kernels against the FP64
  oracle network run on the same bf16-rounded weights.  The forward output is
  held to the bound its split-bf16 activations imply; the gradient (whose
  products take single bf16 operands) to 1e-2 relative, norm-wise.
* The Adam kernel's first step against Adam's closed form for that step.
* Trained on pairs from the plain propagator (precision workload's
  distribution): propagation, fit and finding started from the learned guess
  give the plain results (path length within the 1e-4 cm convergence
  threshold, parameters and hit lists at the oracle parity bars), and the
  learned start needs fewer evaluations of r(s) than the straight line.
The network's guess itself is parity-unpinned: only the exact solve it
starts judges it.
"""
import numpy as np
import pytest

import eventgen as E
from oracle import mlp as M
from tests import common as CM

pytestmark = pytest.mark.gpu

BLOCKS = (("W1", 0, 512), ("b1", 512, 576), ("W2", 576, 4672), ("b2", 4672, 4736),
          ("w3", 4736, 4800), ("b3", 4800, 4801))


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_02253_amd as K
    from paper_1906_02253_amd import learned, pipeline
    K.learned = learned
    K.pipeline = pipeline
    return K


def _weights(seed):
    rng = np.random.default_rng(seed)
    w = E.mlp_init(seed).astype(np.float64)
    w += rng.normal(0, 0.05, w.shape)          # non-zero biases
    return w.astype(np.float32)


def _upload_feats(X):
    import torch
    n = X.shape[0]
    ld = CM.ld_of(n)
    f = torch.zeros((8, ld), dtype=torch.float32, device="cuda")
    f[:, :n] = torch.as_tensor(X.T.astype(np.float32))
    return f


@pytest.mark.parametrize("n", [1, 63, 1000])
def test_forward_matches_oracle(K, n):
    import torch
    rng = np.random.default_rng(80 + n)
    ctx = K.Context(E.geometry.barrel10(x0=0.0))
    w = _weights(80)
    ctx.mlp_load(w)
    X = rng.uniform(-1.5, 1.5, (n, 8)).astype(np.float32)
    f = _upload_feats(X)
    out = torch.zeros(n, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(f, n, out)
    torch.cuda.synchronize()
    y = out.cpu().numpy().astype(np.float64)
    wb = M.bf16_round(w)
    Xd = X.astype(np.float64)
    yo, (_, h1, _) = M.forward(wb, Xd)
    # The device uses the bf16 weights exactly and passes the inputs and the
    # first hidden layer as high + low bf16 parts (relative error <= 2^-16),
    # accumulating in FP32; tanh' <= 1, so per sample
    #   |dy| <= u * sum_j |w3_j| sum_k |W2_jk| (|h1_k| + sum_i |W1_ki| |x_i|)
    #           + e_t * sum_j |w3_j| (1 + sum_k |W2_jk|)
    # with u = 2^-14 (the split plus FP32 sums of up to 64 terms, 4x margin)
    # and e_t = 1e-6 for the exponential-based tanh.
    p = M.unpack(wb)
    a1 = np.abs(h1) + np.abs(Xd) @ np.abs(p["W1"]).T
    bound = (2.0 ** -14 * (a1 @ np.abs(p["W2"]).T) @ np.abs(p["w3"])
             + 1e-6 * np.abs(p["w3"]) @ (1 + np.abs(p["W2"]).sum(axis=1)))
    d = np.abs(y - yo)
    print(f"n={n}: max |dy| {d.max():.2e}, max |dy|/bound {(d / bound).max():.3f}, "
          f"rel norm {np.linalg.norm(y - yo) / np.linalg.norm(yo):.2e}")
    assert np.all(d <= bound)
    # master weights read back unchanged
    assert np.array_equal(ctx.mlp_get(), w)


def test_gradient_matches_oracle(K):
    import torch
    rng = np.random.default_rng(81)
    ctx = K.Context(E.geometry.barrel10(x0=0.0))
    w = _weights(81)
    ctx.mlp_load(w)
    n = 700
    X = rng.uniform(-1.5, 1.5, (n, 8)).astype(np.float32)
    t = rng.uniform(-1, 1, n).astype(np.float32)
    f = _upload_feats(X)
    tt = torch.zeros(f.shape[1], dtype=torch.float32, device="cuda")
    tt[:n] = torch.as_tensor(t)
    # a batch with repeated rows and a length that is not a multiple of 64
    rows = np.concatenate([rng.permutation(n)[:290], [3, 3, 7]]).astype(np.int32)
    g = torch.zeros(M.N_PARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.mlp_grad(f, tt, n, torch.as_tensor(rows, device="cuda"), g, loss)
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    Lo, go = M.grad(M.bf16_round(w), X[rows].astype(np.float64), t[rows].astype(np.float64))
    assert abs(loss.item() - Lo) < 1e-2 * Lo
    tot = np.linalg.norm(gg - go) / np.linalg.norm(go)
    print(f"gradient rel err {tot:.2e}")
    assert tot < 1e-2
    for name, a, b in BLOCKS:
        e = np.linalg.norm(gg[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        print(f"  {name}: {e:.2e}")
        assert e < 2e-2, name


def test_gradient_skips_rows_outside(K):
    """Rows outside [0, n) add nothing to the sum (they still count in the mean)."""
    import torch
    rng = np.random.default_rng(82)
    ctx = K.Context(E.geometry.barrel10(x0=0.0))
    w = _weights(82)
    ctx.mlp_load(w)
    n = 100
    X = rng.uniform(-1, 1, (n, 8)).astype(np.float32)
    t = rng.uniform(-1, 1, n).astype(np.float32)
    f = _upload_feats(X)
    tt = torch.zeros(f.shape[1], dtype=torch.float32, device="cuda")
    tt[:n] = torch.as_tensor(t)
    rows = np.arange(64, dtype=np.int32)
    bad = rows.copy()
    bad[10] = -1
    bad[20] = n + 5
    g = torch.zeros(M.N_PARAM, dtype=torch.float32, device="cuda")
    gb = torch.zeros_like(g)
    ctx.mlp_grad(f, tt, n, torch.as_tensor(rows, device="cuda"), g)
    ctx.mlp_grad(f, tt, n, torch.as_tensor(bad, device="cuda"), gb)
    keep = np.array([r for r in range(64) if r not in (10, 20)])
    _, go = M.grad(M.bf16_round(w), X[keep].astype(np.float64), t[keep].astype(np.float64))
    go *= keep.size / 64.0
    e = np.linalg.norm(gb.cpu().numpy() - go) / np.linalg.norm(go)
    assert e < 1e-2, e
    assert not np.allclose(g.cpu().numpy(), gb.cpu().numpy())


def test_first_adam_step(K):
    """Adam's first step moves every parameter by lr * g / (|g| + eps): by
    -lr * sign(g) wherever |g| >> eps.  Checked where the oracle gradient is
    clearly non-zero (bf16 errors cannot flip its sign there)."""
    import torch
    rng = np.random.default_rng(83)
    ctx = K.Context(E.geometry.barrel10(x0=0.0))
    w = _weights(83)
    ctx.mlp_load(w)
    n = 512
    X = rng.uniform(-1, 1, (n, 8)).astype(np.float32)
    t = rng.uniform(-1, 1, n).astype(np.float32)
    f = _upload_feats(X)
    tt = torch.zeros(f.shape[1], dtype=torch.float32, device="cuda")
    tt[:n] = torch.as_tensor(t)
    rows = torch.as_tensor(np.arange(n, dtype=np.int32), device="cuda")
    ctx.mlp_train(f, tt, n, rows, n, 1, lr=1e-3)
    w1 = ctx.mlp_get().astype(np.float64)
    _, go = M.grad(M.bf16_round(w), X.astype(np.float64), t.astype(np.float64))
    sig = np.abs(go) > 0.2 * np.sqrt(np.mean(go ** 2))
    assert sig.sum() > 1000
    want = w.astype(np.float64) - 1e-3 * np.sign(go)
    assert np.allclose(w1[sig], want[sig], rtol=0, atol=2e-7 + 1e-6 * np.abs(want[sig]))


def test_targets_match_oracle(K, orc):
    """Training targets made by the library (kf_mlp_features, the plain
    kf_propagate, kf_mlp_targets) against the FP64 oracle's: its features,
    its propagation's path length and its target.  The path the target
    encodes (s_line + h s_line^2 y) agrees to 2e-4 cm everywhere, and the
    target itself to 1e-3 relative where the correction exceeds 0.05 cm."""
    geom, states, tl = E.propagation_pairs(n_pairs=20_000, seed=14, n_tracks=5_000)
    ctx = K.Context(geom)
    ps = K.learned.PairSet(ctx, states, tl)
    n = ps.n
    tg = ps.target[:n].cpu().numpy().astype(np.float64)
    cfg = orc.Config(geom)
    kinds = np.array([geom[l]["kind"] for l in tl])
    tgt = np.array([geom[l]["r_or_z"] for l in tl])
    f = M.features(states, kinds, tgt)
    path = np.zeros(n)
    ok = np.zeros(n, bool)
    for i in range(n):
        st, _, _, s, _ = orc.propagate(cfg, int(tl[i]), states[i], np.zeros(21), noise=False)
        ok[i] = st == 0
        path[i] = s
    assert np.array_equal(ok, np.isin(np.arange(n), ps.ok_rows))
    to = M.target(f, path)
    k = np.where(f[:, 4] != 0, f[:, 3] * f[:, 5] ** 2 / np.where(f[:, 4] != 0, f[:, 4], 1), 0)
    dpath = 100.0 * np.abs(k * (tg - to))
    corr = np.abs(path - 100.0 * f[:, 5])
    big = ok & (corr > 0.05)
    rel = np.abs(tg - to)[big] / np.abs(to[big])
    print(f"targets: {ok.sum()} pairs, max path difference {dpath[ok].max():.2e} cm, "
          f"{big.sum()} with corrections > 0.05 cm, max rel target difference {rel.max():.2e}")
    assert dpath[ok].max() < 2e-4
    assert big.sum() > 1000 and rel.max() < 1e-3


@pytest.fixture(scope="module")
def trained(K):
    """Network trained on the device on 1e6 pairs (precision workload's
    distribution, seed 4): 20 epochs of batch 4096, Adam lr 1e-3."""
    geom, states, tl = E.propagation_pairs(n_pairs=1_000_000, seed=4)
    ctx = K.Context(geom)
    ps = K.learned.PairSet(ctx, states, tl)
    tr, va, te = K.learned.split_rows(ps.ok_rows, seed=4)
    w0 = E.mlp_init(4)
    ctx.mlp_load(w0)
    l0 = K.learned.eval_loss(ctx, ps, va)
    losses = K.learned.train(ctx, ps, tr, w0, epochs=20, batch=4096, lr=1e-3, seed=4)
    lv = K.learned.eval_loss(ctx, ps, va)
    print(f"pairs {ps.n}, ok {ps.ok_rows.size}; val loss {l0:.3e} -> {lv:.3e}; "
          f"train loss first {losses[:10].mean():.3e} last {losses[-50:].mean():.3e}")
    return dict(ctx=ctx, geom=geom, states=states, tl=tl, ps=ps, test=te, l0=l0, lv=lv,
                losses=losses)


def test_training_reduces_loss(trained):
    assert np.all(np.isfinite(trained["losses"]))
    assert trained["lv"] < 0.01 * trained["l0"]
    # rms error of the guess, in cm
    print(f"validation rms of the scaled correction: {np.sqrt(trained['lv']):.4f}")


def test_learned_start_same_answer_fewer_iterations(K, trained):
    te = trained["test"]
    r = K.learned.compare_starts(trained["ctx"], trained["states"][te], trained["tl"][te])
    p, l = r["plain"], r["learned"]
    frozen = lambda s: s & ~K.ST_FALLBACK
    assert np.array_equal(frozen(p["status"]), frozen(l["status"]))
    ok = p["status"] == 0
    assert ok.mean() > 0.99
    ds = np.abs(l["path"][ok] - p["path"][ok])
    err = CM.par_error(l["par"][ok], p["par"][ok])
    fb = (l["status"] & K.ST_FALLBACK) != 0
    it_p, it_l = p["iters"][ok], l["iters"][ok]
    print(f"{ok.sum()} test propagations: evaluations plain mean {it_p.mean():.3f} "
          f"p99 {np.percentile(it_p, 99):.0f}, learned mean {it_l.mean():.3f} "
          f"p99 {np.percentile(it_l, 99):.0f}; fallback rate {fb[ok].mean():.4f}; "
          f"max |ds| {ds.max():.2e} cm; max rel par diff {err.max():.2e}")
    assert ds.max() < 1e-4
    assert err.max() < CM.REL
    assert it_l.mean() < it_p.mean()
    assert fb[ok].mean() < 0.05


def test_learned_fit_matches_oracle(K, orc, trained):
    """The 1,000-track fit workload with the learned start against the FP64
    oracle (plain solve): same statuses, parameters within 1e-4 relative."""
    import torch
    geom, ev = E.fit_sample(n_tracks=1000, seed=0)
    ctx = K.Context(geom)
    ctx.mlp_load(trained["ctx"].mlp_get())
    n = ev.n_tracks
    ld = CM.ld_of(n)
    hits = K.Hits.from_event(ev)
    sh = torch.as_tensor(CM.soa_int(ev.seq_hit[:, :3], ld), device="cuda")
    lseq = torch.as_tensor(CM.soa_int(ev.seq_layer, ld), device="cuda")
    hidx = torch.as_tensor(CM.soa_int(ev.seq_hit, ld), device="cuda")
    t = K.Tracks(n, ld)
    ctx.seed(hits, sh, t)
    ctx.fit(t, hits, lseq, hidx, ev.seq_layer.shape[1], K.INIT_MLP)
    torch.cuda.synchronize()
    g = t.numpy()
    cfg = orc.Config(geom)
    par0, cov0 = orc.seeds_for_event(ev)
    o = orc.fit(cfg, dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv), ev.seq_layer, ev.seq_hit,
                par0, cov0, n_threads=8)
    assert np.array_equal(g["status"] & ~K.ST_FALLBACK, o["status"])
    ok = o["status"] == 0
    err = CM.par_error(g["par"][ok], o["par"][ok])
    assert err.max() < CM.REL, err.max(axis=0)
    cerr = CM.chi2_error(g["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
    assert cerr.max() < CM.CHI2_REL


def test_learned_find_matches_oracle(K, orc, trained):
    """Finding on 5 events of the 800-track workload with the learned start:
    hit lists against the FP64 oracle under the same tie rules."""
    import torch
    from tests.test_gpu_find import _check_parity
    geom, evs = E.find_events(n_events=5, n_tracks=800, n_noise=50_000, seed=1)
    inp = E.find_inputs(evs)
    ctx = K.Context(geom)                      # this workload's material
    ctx.mlp_load(trained["ctx"].mlp_get())
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run(K.INIT_MLP)
    torch.cuda.synchronize()
    g = fp.results()
    print("counters (prop, upd, chi2, newton, disk, guesses, fallbacks):", g["counters"])
    assert g["counters"][5] > 0
    o = CM.oracle_find_events(orc, geom, evs, inp)
    _check_parity(g, o, "learned find")


def test_learned_find_needs_width_64(K, trained):
    """The learned start runs a whole wave per guess: width 32 is refused,
    and the autotuner skips it under the learned flag."""
    import torch
    geom, evs = E.find_events(n_events=1, n_tracks=100, n_noise=2_000, seed=1)
    inp = E.find_inputs(evs)
    ctx = K.Context(geom)
    ctx.mlp_load(trained["ctx"].mlp_get())
    fp = K.pipeline.FindProblem(ctx, inp)
    ctx.set_find_config(32, False)
    with pytest.raises(K.KFError):
        fp.run(K.INIT_MLP)
    fp.run()                                  # the plain path accepts 32
    tab = fp.autotune(flags=K.INIT_MLP, reps=1)
    assert all(w >= 64 for (w, _) in tab), tab
    assert ctx.find_config()[0] >= 64
    torch.cuda.synchronize()


def test_learned_requires_loaded_model(K):
    geom, ev = E.fit_sample(n_tracks=10, seed=0)
    ctx = K.Context(geom)
    t = K.Tracks(10)
    import torch
    tl = torch.zeros(t.ld, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KFError):
        ctx.propagate(t, tl, flags=K.INIT_MLP)
