"""Pins of the oracle's parametrised-field propagation (solenoid-like field,
Runge-Kutta transport, propagate-to-radius) against facts outside its own
code: Maxwell's divergence-free condition, the field formula as the input
generator implements it, the closed-form helix in the uniform limit, a
high-accuracy adaptive integration of the equations of motion by scipy, the
fourth-order convergence of the integrator, and fit pulls on tracks traced by
the generator's independent fine-step integrator."""
import numpy as np
import pytest

import eventgen as E
import eventgen.field as EF

KAPPA = 0.00299792458


def _cfg(orc, z0=300.0, step=2.0, geom=None):
    return orc.Config(geom or E.geometry.barrel10(x0=0.0), field_z0=z0, field_step=step)


def _tracks(rng, n, pt_lo=0.5, pt_hi=10.0):
    pt = rng.uniform(pt_lo, pt_hi, n)
    th = rng.uniform(0.7, 2.4, n)
    return np.stack([rng.normal(0, 1, n), rng.normal(0, 1, n), rng.uniform(-40, 40, n),
                     rng.choice([-1, 1], n) / pt, rng.uniform(-np.pi, np.pi, n), th], axis=1)


def _ref_path(p, l, z0, b0=3.8):
    """The equations of motion integrated by scipy's DOP853 at rtol 1e-12."""
    from scipy.integrate import solve_ivp
    st = np.sin(p[5])
    kq = KAPPA * p[3] * st

    def f(_, y):
        u = y[2] / z0
        g = 1.0 / (1.0 + u * u)
        dbz = -2.0 * b0 * y[2] / z0 ** 2 * g * g
        bx, by, bz = -0.5 * dbz * y[0], -0.5 * dbz * y[1], b0 * g
        return [y[3], y[4], y[5], kq * (y[4] * bz - y[5] * by), kq * (y[5] * bx - y[3] * bz),
                kq * (y[3] * by - y[4] * bx)]

    y0 = [p[0], p[1], p[2], st * np.cos(p[4]), st * np.sin(p[4]), np.cos(p[5])]
    r = solve_ivp(f, (0.0, l), y0, method="DOP853", rtol=1e-12, atol=1e-12)
    return r.y[:, -1]


def test_field_divergence_free_and_symmetric(orc):
    cfg = _cfg(orc)
    rng = np.random.default_rng(100)
    for _ in range(20):
        x = rng.uniform(-100, 100, 3)
        x[2] = rng.uniform(-250, 250)
        d = 1e-3
        div = 0.0
        for i in range(3):
            a, b = x.copy(), x.copy()
            a[i] += d
            b[i] -= d
            div += (orc.field(cfg, a)[i] - orc.field(cfg, b)[i]) / (2 * d)
        assert abs(div) < 1e-9
        B = orc.field(cfg, x)
        xm = x.copy()
        xm[2] = -x[2]
        Bm = orc.field(cfg, xm)
        assert np.allclose([Bm[0], Bm[1], Bm[2]], [-B[0], -B[1], B[2]], rtol=1e-14, atol=1e-16)
        # the input generator's own implementation of the same formula
        g = EF.field(x[0], x[1], x[2], 3.8, 300.0)
        assert np.allclose(B, g, rtol=1e-13, atol=1e-15)
    assert orc.field(cfg, np.zeros(3))[2] == pytest.approx(3.8)
    assert orc.field(cfg, np.array([0.0, 0.0, 300.0]))[2] == pytest.approx(1.9)


def test_rk_uniform_limit_is_the_helix(orc):
    cfg = _cfg(orc, z0=1e15, step=1.0)
    rng = np.random.default_rng(101)
    for p in _tracks(rng, 30, 0.5, 10.0):
        for l in (5.0, 40.0, 100.0):
            q = orc.rk_path(cfg, p, l)
            h = orc.helix(p, l * np.sin(p[5]))
            assert np.allclose(q[:3], h[:3], atol=2e-6), (p, l)
            assert np.allclose(q[3], h[3], rtol=1e-9)
            assert np.allclose(q[5], h[5], atol=1e-9)


def test_rk_matches_adaptive_integration(orc):
    cfg = _cfg(orc)
    rng = np.random.default_rng(102)
    for p in _tracks(rng, 12):
        ref = _ref_path(p, 80.0, 300.0)
        q = orc.rk_path(cfg, p, 80.0)
        assert np.allclose(q[:3], ref[:3], atol=2e-5), (p, q[:3] - ref[:3])
        th = np.arctan2(np.hypot(ref[3], ref[4]), ref[5])
        assert q[5] == pytest.approx(th, abs=1e-6)


def test_rk_is_fourth_order(orc):
    rng = np.random.default_rng(103)
    p = _tracks(rng, 1, 0.5, 0.6)[0]
    ref = _ref_path(p, 60.0, 300.0)
    err = []
    for step in (4.0, 2.0, 1.0):
        q = orc.rk_path(_cfg(orc, step=step), p, 60.0)
        err.append(np.linalg.norm(q[:3] - ref[:3]))
    r1, r2 = err[0] / err[1], err[1] / err[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, (err, r1, r2)


def test_field_propagation_to_radius(orc):
    """The converged crossing lies on the cylinder, at the place the
    adaptive integration of the same trajectory crosses it."""
    from scipy.integrate import solve_ivp
    cfg = _cfg(orc)
    geom = cfg.geom
    rng = np.random.default_rng(104)
    P0 = np.zeros(21)
    n_ok = 0
    for p in _tracks(rng, 20, 1.0, 10.0):
        p[0] = p[1] = 0.0
        layer = 7                                  # r = 65 cm
        st, q, _, l, it = orc.propagate(cfg, layer, p, P0, noise=False)
        if st:
            continue
        n_ok += 1
        r_l = geom[layer]["r_or_z"]
        assert np.hypot(q[0], q[1]) == pytest.approx(r_l, abs=1e-5)
        ref = _ref_path(p, l, 300.0)
        assert np.allclose(q[:3], ref[:3], atol=5e-5)
        assert 1 <= it <= 10
    assert n_ok >= 15


def test_field_fit_pulls(orc):
    """Fit in the parametrised field of tracks traced by the generator's
    fine-step integrator: unit pulls at the last layer and chi2/ndf near 1
    (the transport Jacobian is the helix one in the start point's field, an
    approximation the pulls must tolerate)."""
    geom, ev = EF.field_sample(n_tracks=1500, seed=5)
    cfg = _cfg(orc, geom=geom)
    par0, cov0 = orc.seeds_for_event(ev)
    r = orc.fit(cfg, dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv), ev.seq_layer, ev.seq_hit,
                par0, cov0, n_threads=8)
    nh = ev.n_track_hits()
    ok = (r["status"] == 0) & (nh == 10)
    assert ok.sum() > 1200
    truth = ev.truth_at[ok, 9]
    P = orc.unpack(r["cov"][ok])
    d = r["par"][ok] - truth
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    for k in (2, 3, 4, 5):
        pull = d[:, k] / np.sqrt(P[:, k, k])
        assert abs(pull.mean()) < 0.1, (k, pull.mean())
        assert 0.9 < pull.std() < 1.1, (k, pull.std())
    c2 = r["chi2"][ok] / r["ndf"][ok]
    assert 0.9 < c2.mean() < 1.1


def test_field_find_follows_the_field(orc):
    """Finding in the parametrised field (next surface = next barrel by the
    Runge-Kutta radius solve) on tracks traced by the generator's fine-step
    integrator among uniform noise: it recovers nearly every true hit beyond
    the seed, with chi2/ndf near 1; the same finder in the uniform field of
    the central value loses hits and its chi2 is inflated (the field falls by
    up to a third over the barrels' length)."""
    from tests import common as CM
    geom, evs = EF.field_find_events(n_events=2, n_tracks=500, n_noise=20_000, seed=26)
    inp = E.find_inputs(evs)

    def eff(r):
        found = tot = 0
        for s in range(inp["seed_hits"].shape[0]):
            e, t = inp["seed_event"][s], inp["seed_track"][s]
            true = evs[e].seq_hit[t]
            true = set((true[true >= 0][3:] + inp["event_off"][e]).tolist())
            got = set(r["hits"][s][r["hits"][s] >= 0].tolist())
            found += len(true & got)
            tot += len(true)
        return found / tot

    f = CM.oracle_find_events(orc, geom, evs, inp, field_z0=300.0, field_step=2.0)
    u = CM.oracle_find_events(orc, geom, evs, inp)
    ef, eu = eff(f), eff(u)
    c2f = np.median(f["chi2"] / np.maximum(f["ndf"], 1))
    c2u = np.median(u["chi2"] / np.maximum(u["ndf"], 1))
    print(f"hit efficiency: field {ef:.4f}, uniform {eu:.4f}; median chi2/ndf {c2f:.3f} vs {c2u:.3f}")
    assert (f["status"] == 0).mean() > 0.99
    assert ef > 0.99
    assert eu < ef - 0.01
    assert 0.8 < c2f < 1.1
    assert c2u > c2f + 0.15


def test_field_find_uniform_limit_equals_helix_finder(orc):
    """With Z0 = 1e9 cm the parametrised field is uniform over the detector:
    finding with Runge-Kutta transport (0.5 cm steps) reproduces the
    closed-form helix finder on the same events hit for hit, with the same
    propagations, states to 1e-9 relative and chi2 to 1e-8."""
    from tests import common as CM
    geom, evs = E.find_events(n_events=2, n_tracks=300, n_noise=20_000, seed=41)
    inp = E.find_inputs(evs)
    u = CM.oracle_find_events(orc, geom, evs, inp)
    f = CM.oracle_find_events(orc, geom, evs, inp, field_z0=1e9, field_step=0.5)
    assert np.array_equal(u["hits"], f["hits"])
    assert np.array_equal(u["status"], f["status"])
    assert u["n_prop"] == f["n_prop"]
    ok = u["status"] == 0
    assert ok.mean() > 0.99
    assert CM.par_error(f["par"][ok], u["par"][ok]).max() < 1e-9
    assert np.max(np.abs(f["chi2"][ok] - u["chi2"][ok]) / np.maximum(u["chi2"][ok], 1.0)) < 1e-8


# ---------------------------------------------------------------- disks in the field
def test_field_propagation_to_disk(orc):
    """Propagate-to-z in the parametrised field: the converged crossing lies
    on the disk plane, at the place the adaptive integration of the same
    trajectory reaches after the same path length; in the uniform limit it
    is the closed-form helix crossing of the plane."""
    from tests import bruteforce as BF
    geom = E.geometry.barrel10_disks14(x0=0.0)
    cfg = _cfg(orc, geom=geom)
    cfg_u = _cfg(orc, z0=1e9, step=0.5, geom=geom)
    rng = np.random.default_rng(110)
    P0 = np.zeros(21)
    n_ok = 0
    for p in _tracks(rng, 40, 1.0, 10.0):
        p[0] = p[1] = 0.0
        p[2] = rng.uniform(-5, 5)
        p[5] = rng.uniform(0.2, 0.6) if rng.random() < 0.5 else np.pi - rng.uniform(0.2, 0.6)
        layer = 12 if np.cos(p[5]) > 0 else 19          # z = +-110 cm
        zd = geom[layer]["r_or_z"]
        st, q, _, l, it = orc.propagate(cfg, layer, p, P0, noise=False)
        assert st == 0
        n_ok += 1
        assert q[2] == pytest.approx(zd, abs=1e-9)
        ref = _ref_path(p, l, 300.0)
        assert np.allclose(q[:3], ref[:3], atol=5e-5)
        assert 1 <= it <= 10
        st, qu, _, lu, _ = orc.propagate(cfg_u, layer, p, P0, noise=False)
        cf, s_cf = BF.cf_disk(p, zd, 3.8)
        assert lu * np.sin(p[5]) == pytest.approx(s_cf, rel=1e-9)
        assert np.allclose(qu[:3], cf[:3], atol=1e-6)
    assert n_ok == 40
    # a disk behind the track is unreachable
    p = np.array([0.0, 0.0, 0.0, 0.5, 0.3, 0.4])
    st, *_ = orc.propagate(cfg, 19, p, P0, noise=False)
    assert st == orc.ST_UNREACHABLE
    # so is one more than 1000 cm of path ahead (z = 30 cm at cot(theta) =
    # 0.02), which the uniform field's closed form still reaches
    p = np.array([0.0, 0.0, 0.0, 0.1, 0.3, np.pi / 2 - 0.02])
    st, *_ = orc.propagate(cfg, 10, p, P0, noise=False)
    assert st == orc.ST_UNREACHABLE
    assert orc.propagate(_cfg(orc, z0=0.0, geom=geom), 10, p, P0, noise=False)[0] == 0
    p[5] = np.pi / 2 - 0.04                             # 750 cm: reached
    assert orc.propagate(cfg, 10, p, P0, noise=False)[0] == 0


def test_field_disk_fit_pulls(orc):
    """Fit in the parametrised field of barrel and endcap tracks (|eta| < 2.5)
    traced by the generator's fine-step integrator through barrels and disks:
    unit pulls at the last surface and chi2/ndf near 1 (disks reached by the
    Runge-Kutta z solve)."""
    geom, evs = EF.field_disk_events(n_events=1, n_tracks=1500, n_noise=0, seed=31)
    ev = evs[0]
    cfg = _cfg(orc, geom=geom)
    par0, cov0 = orc.seeds_for_event(ev)
    r = orc.fit(cfg, dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv), ev.seq_layer, ev.seq_hit,
                par0, cov0, n_threads=8)
    nh = ev.n_track_hits()
    kinds = np.array([L["kind"] for L in geom])
    last = ev.seq_layer[np.arange(ev.n_tracks), np.maximum(nh - 1, 0)]
    ok = (r["status"] == 0) & (nh >= 7)
    disk_end = ok & (kinds[last] == 1)
    assert disk_end.sum() > 300 and ok.sum() > 1000
    truth = ev.truth_at[np.arange(ev.n_tracks), np.maximum(nh - 1, 0)][ok]
    P = orc.unpack(r["cov"][ok])
    d = r["par"][ok] - truth
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    for k in (3, 4, 5):
        pull = d[:, k] / np.sqrt(P[:, k, k])
        assert abs(pull.mean()) < 0.1, (k, pull.mean())
        assert 0.9 < pull.std() < 1.1, (k, pull.std())
    c2 = r["chi2"][ok] / r["ndf"][ok]
    assert 0.9 < c2.mean() < 1.1


def test_field_find_with_disks(orc):
    """Finding in the parametrised field over barrels and disks (the next
    surface the first reached of the next barrel and the disks ahead, each by
    its Runge-Kutta solve) on tracks traced by the generator among uniform
    noise: nearly every true hit beyond the seed is found, chi2/ndf near 1,
    and the binned search equals the all-hits scan."""
    from tests import common as CM
    geom, evs = EF.field_disk_events(n_events=2, n_tracks=400, n_noise=24_000, seed=32)
    inp = E.find_inputs(evs)
    f = CM.oracle_find_events(orc, geom, evs, inp, field_z0=300.0, field_step=2.0)
    found = tot = 0
    disk_hits = 0
    kinds = np.array([L["kind"] for L in geom])
    for s in range(inp["seed_hits"].shape[0]):
        e, t = inp["seed_event"][s], inp["seed_track"][s]
        true = evs[e].seq_hit[t]
        true = set((true[true >= 0][3:] + inp["event_off"][e]).tolist())
        got = f["hits"][s][f["hits"][s] >= 0]
        disk_hits += int((kinds[np.nonzero(f["hits"][s] >= 0)[0]] == 1).sum())
        found += len(true & set(got.tolist()))
        tot += len(true)
    c2 = np.median(f["chi2"] / np.maximum(f["ndf"], 1))
    print(f"field finding with disks: efficiency {found / tot:.4f}, disk hits {disk_hits}, "
          f"median chi2/ndf {c2:.3f}")
    assert found / tot > 0.99 and disk_hits > 1000
    assert 0.8 < c2 < 1.1
    ev = evs[0]
    m = np.nonzero(inp["seed_event"] == 0)[0]
    cfg = _cfg(orc, geom=geom)
    rb = orc.find(cfg, ev, inp["seed_hits_local"][m], binned=True)
    ra = orc.find(cfg, ev, inp["seed_hits_local"][m], binned=False)
    assert np.array_equal(rb["hits"], ra["hits"])


def test_field_find_with_disks_uniform_limit(orc):
    """With Z0 = 1e9 cm, finding in the field over barrels and disks
    reproduces the closed-form helix finder on the same events (uniform-field
    barrel + endcap events) hit for hit, states to 1e-8."""
    from tests import common as CM
    rng = np.random.default_rng(33)
    geom = E.geometry.barrel10_disks14(x0=0.0)
    evs = [E.make_event(rng, geom, 300, E.pt_power2(0.5, 50.0), 2.5, 1000) for _ in range(2)]
    inp = E.find_inputs(evs)
    u = CM.oracle_find_events(orc, geom, evs, inp)
    f = CM.oracle_find_events(orc, geom, evs, inp, field_z0=1e9, field_step=0.5)
    kinds = np.array([L["kind"] for L in geom])
    assert (u["hits"][:, kinds == 1] >= 0).sum() > 500
    same = (u["hits"] == f["hits"]).all(axis=1)
    assert same.mean() > 0.995, same.mean()
    ok = same & (u["status"] == 0)
    assert CM.par_error(f["par"][ok], u["par"][ok]).max() < 1e-8
