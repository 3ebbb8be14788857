"""Pins of the FP64 oracle against things other than itself: closed forms,
invariants, finite differences, textbook special cases, brute force.

Each test names the part of the method it pins:
  helix / propagation   - the analytic helix and its closed-form crossings
  Jacobian              - central finite differences, straight-line limit
  update                - standard / information forms, normal equations
  fit                   - Gauss-Newton batch least squares, pull widths, chi2
  finding               - binned == all-hits scan, noise-free special case,
                          exhaustive enumeration on tiny events
"""
import math

import numpy as np
import pytest
from scipy import stats

import eventgen as E
from eventgen import generate as GEN
from tests import bruteforce as BF

BZ = 3.8


def rand_states(rng, n, r0max=40.0):
    """Random states inside the tracker, moving outward."""
    out = []
    while len(out) < n:
        r0 = rng.uniform(0.0, r0max)
        a = rng.uniform(-np.pi, np.pi)
        phi = wrap(a + rng.uniform(-1.0, 1.0))
        pt = math.exp(rng.uniform(math.log(0.4), math.log(100.0)))
        c = rng.choice([-1, 1]) / pt
        th = 2 * math.atan(math.exp(-rng.uniform(-1.2, 1.2)))
        out.append(np.array([r0 * math.cos(a), r0 * math.sin(a), rng.uniform(-5, 5), c, phi, th]))
    return out


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


# ---------------------------------------------------------------- helix
def test_helix_invariants(orc):
    rng = np.random.default_rng(11)
    for p in rand_states(rng, 200):
        C, h = BF.circle(p, BZ)
        for s in (0.0, 1e-3, 7.3, 55.0, 180.0):
            q = orc.helix(p, s, BZ)
            Cq, hq = BF.circle(q, BZ)
            assert abs(np.hypot(q[0] - C[0], q[1] - C[1]) - 1 / abs(h)) < 1e-9 * max(1, 1 / abs(h))
            assert np.allclose(Cq, C, rtol=0, atol=1e-8 * max(1.0, 1 / abs(h)))
            assert q[3] == p[3] and q[5] == p[5]
            assert abs(q[2] - p[2] - s / math.tan(p[5])) < 1e-12 * max(1, s)
            assert abs(wrap(q[4] - p[4] - h * s)) < 1e-12 * max(1, abs(h * s))
            # tangent: numerical derivative of the position is (cos phi(s), sin phi(s))
            e = 1e-5
            qa, qb = orc.helix(p, s + e, BZ), orc.helix(p, s - e, BZ)
            d = (qa[:2] - qb[:2]) / (2 * e)
            assert np.allclose(d, [math.cos(q[4]), math.sin(q[4])], atol=1e-8)


def test_helix_matches_difference_form(orc):
    """sin/cos difference form of the same circle (textbook), away from h -> 0."""
    rng = np.random.default_rng(12)
    for p in rand_states(rng, 100):
        h = -E.KAPPA * BZ * p[3]
        s = 40.0
        q = orc.helix(p, s, BZ)
        xd = p[0] + (math.sin(p[4] + h * s) - math.sin(p[4])) / h
        yd = p[1] + (math.cos(p[4]) - math.cos(p[4] + h * s)) / h
        assert abs(q[0] - xd) < 1e-9 and abs(q[1] - yd) < 1e-9


def test_newton_equals_closed_form(orc):
    """T1: propagate-to-radius Newton solution equals the circle-circle
    intersection.  The stopping rule (|r - r_l| < 1e-4 cm, then one more Newton
    step) leaves a quadratic remainder well below 1e-7 cm."""
    cfg = orc.Config(E.geometry.barrel10(), max_newton=30)
    rng = np.random.default_rng(13)
    n_ok, worst = 0, 0.0
    for p in rand_states(rng, 400):
        r0 = math.hypot(p[0], p[1])
        for r_l in (5.0, 25.0, 50.0, 100.0):
            if r_l <= r0 + 0.05:
                continue
            cf = BF.cf_barrel(p, r_l, BZ)
            st, s, it = orc.solve_barrel(cfg, p, r_l)
            C, h = BF.circle(p, BZ)
            reach = np.hypot(*C) + 1 / abs(h) >= r_l
            if not reach:
                assert st == orc.ST_UNREACHABLE
                continue
            assert st == 0, (p, r_l)
            assert cf is not None
            assert abs(s - cf[1]) < 1e-7, (s, cf[1], it)
            worst = max(worst, abs(s - cf[1]))
            q = orc.helix(p, s, BZ)
            assert abs(math.hypot(q[0], q[1]) - r_l) < 1e-7
            assert np.allclose(q[:3], cf[0][:3], atol=1e-7)
            n_ok += 1
    assert n_ok > 500
    print("worst |s - s_closed_form| =", worst)


def test_track_from_origin_closed_form(orc):
    """A track from the origin reaches radius r after s = 2R asin(r / 2R)."""
    cfg = orc.Config(E.geometry.barrel10())
    for pt in (0.5, 1.0, 3.0, 100.0):
        R = pt / (E.KAPPA * BZ)
        for r_l in E.geometry.BARREL_R:
            p = np.array([0, 0, 0, 1 / pt, 0.3, 1.1])
            st, s, it = orc.solve_barrel(cfg, p, r_l)
            if r_l > 2 * R:
                assert st == orc.ST_UNREACHABLE
                continue
            assert st == 0
            assert abs(s - 2 * R * math.asin(r_l / (2 * R))) < 1e-10 * r_l
            assert it <= 4


def test_newton_iteration_budget(orc):
    """Straight-line start converges within a handful of evaluations for
    ordinary layer-to-layer steps; the bracket keeps near-apex cases converging."""
    cfg = orc.Config(E.geometry.barrel10(), max_newton=10)
    geom, ev = E.fit_sample(n_tracks=300, seed=5)
    iters = []
    for t in range(ev.n_tracks):
        for k in range(ev.seq_layer.shape[1] - 1):
            l0, l1 = ev.seq_layer[t, k], ev.seq_layer[t, k + 1]
            if l1 < 0:
                break
            st, s, it = orc.solve_barrel(cfg, ev.truth_at[t, k], geom[l1]["r_or_z"])
            assert st == 0
            iters.append(it)
    iters = np.array(iters)
    assert iters.max() <= 6 and iters.mean() < 3.5


def test_disk_propagation_closed_form(orc):
    geom = E.geometry.barrel10_disks14()
    cfg = orc.Config(geom)
    rng = np.random.default_rng(14)
    for p in rand_states(rng, 100, r0max=10):
        p[5] = 2 * math.atan(math.exp(-rng.uniform(1.2, 2.4)))      # forward
        st, q, Q, s, it = orc.propagate(cfg, 12, p, orc.pack(np.eye(6)), noise=False)
        ref, s_ref = BF.cf_disk(p, geom[12]["r_or_z"], BZ)
        assert st == 0 and abs(s - s_ref) < 1e-10 * s_ref
        assert np.allclose(q[:3], ref[:3], atol=1e-9)
    # behind the track: unreachable
    p = np.array([1.0, 0, 0, 0.5, 0.0, 2.8])       # moving to -z
    st, *_ = orc.propagate(cfg, 12, p, orc.pack(np.eye(6)))
    assert st == orc.ST_UNREACHABLE


# ---------------------------------------------------------------- Jacobian
@pytest.mark.parametrize("layer", [3, 7, 9, 12, 20])
def test_jacobian_finite_differences(orc, layer):
    """T3: analytic transport Jacobian (with the path-length derivative)
    against central finite differences of the propagated state."""
    geom = E.geometry.barrel10_disks14()
    cfg = orc.Config(geom, max_newton=30)
    rng = np.random.default_rng(100 + layer)
    L = geom[layer]
    steps = np.array([1e-5, 1e-5, 1e-5, 1e-7, 1e-7, 1e-7])
    n = 0
    for p in rand_states(rng, 300, r0max=3.0):
        if L["kind"] == 1:
            eta = rng.uniform(1.3, 2.4) * (1 if L["r_or_z"] > 0 else -1)
            p[5] = 2 * math.atan(math.exp(-eta))
        st, F = orc.jacobian(cfg, layer, p)
        if st:
            continue
        st2, q, *_ = orc.propagate(cfg, layer, p, orc.pack(np.eye(6)), noise=False)
        if abs(abs(q[4]) - math.pi) < 0.1:
            continue

        def fun(pp):
            s_, qq, *_ = orc.propagate(cfg, layer, pp, orc.pack(np.eye(6)), noise=False)
            assert s_ == 0
            return qq
        Fn = BF.num_jacobian(fun, p, steps)
        assert np.allclose(F, Fn, rtol=1e-6, atol=1e-6 * np.abs(F).max()), (p, F - Fn)
        n += 1
    assert n > 100


def test_jacobian_straight_line_limit(orc):
    """T3: as B -> 0 the Jacobian becomes the textbook straight-line one."""
    geom = E.geometry.barrel10()
    cfg = orc.Config(geom, bz=1e-12)
    rng = np.random.default_rng(21)
    for p in rand_states(rng, 50, r0max=3.0):
        r_l = geom[6]["r_or_z"]

        def line(pp):
            x, y, z, c, phi, th = pp
            u = np.array([math.cos(phi), math.sin(phi)])
            pu = x * u[0] + y * u[1]
            s = -pu + math.sqrt(pu * pu - x * x - y * y + r_l * r_l)
            return np.array([x + s * u[0], y + s * u[1], z + s / math.tan(th), c, phi, th])
        Fl = BF.num_jacobian(line, p, np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-7, 1e-7]))
        st, F = orc.jacobian(cfg, 6, p)
        assert st == 0
        assert np.allclose(F, Fl, atol=1e-6)


# ---------------------------------------------------------------- update
def _rand_spd(rng, scale):
    A = rng.normal(size=(6, 6))
    M = A @ A.T + 0.5 * np.eye(6)
    d = np.sqrt(scale)
    return M * np.outer(d, d)


@pytest.mark.parametrize("kind", [0, 1])
def test_update_forms_agree(orc, kind):
    """T4: Joseph form == standard form == information form (FP64)."""
    rng = np.random.default_rng(30 + kind)
    for _ in range(200):
        P = _rand_spd(rng, np.array([1e-2, 1e-2, 1e-2, 1e-3, 1e-4, 1e-4]))
        ph = rng.uniform(-np.pi, np.pi)
        r = 30.0
        p = np.array([r * math.cos(ph), r * math.sin(ph), 3.0, 0.7, ph + 0.2, 1.2])
        hit = np.array([r * math.cos(ph + 1e-3), r * math.sin(ph + 1e-3), 3.01, 0.01, 0.05])
        st, pu, Pu, c2 = orc.update(p, orc.pack(P), hit, kind)
        assert st == 0
        rho = math.hypot(hit[0], hit[1])
        cp, sp = hit[0] / rho, hit[1] / rho
        H = np.zeros((2, 6))
        H[0, :2] = [-sp, cp]
        if kind == 0:
            H[1, 2] = 1
        else:
            H[1, :2] = [cp, sp]
        res = BF.measure(p, hit, kind)
        V = np.diag([hit[3] ** 2, hit[4] ** 2])
        S = H @ P @ H.T + V
        K = P @ H.T @ np.linalg.inv(S)
        P_std = (np.eye(6) - K @ H) @ P
        P_inf = np.linalg.inv(np.linalg.inv(P) + H.T @ np.linalg.inv(V) @ H)
        p_inf = p + P_inf @ H.T @ np.linalg.inv(V) @ res
        Pu_full = orc.unpack(Pu)
        scale = np.sqrt(np.outer(np.diag(P_inf), np.diag(P_inf)))
        assert np.abs((Pu_full - P_std) / scale).max() < 1e-10
        assert np.abs((Pu_full - P_inf) / scale).max() < 1e-9
        d = pu - p_inf
        d[4] = wrap(d[4])
        assert np.abs(d / np.sqrt(np.diag(P_inf))).max() < 1e-9
        assert abs(c2 - res @ np.linalg.solve(S, res)) < 1e-10 * max(1, c2)


def test_linear_kf_equals_normal_equations(orc):
    """T4/T5: with a linear model (fixed transport matrices), a forward KF made of
    the oracle's update steps gives exactly the batch least-squares (normal
    equations with prior) estimate."""
    rng = np.random.default_rng(40)
    geom = E.geometry.barrel10()
    for trial in range(20):
        p_ref = rand_states(rng, 1, r0max=3.0)[0]
        p_ref[3] = rng.choice([-1, 1]) / rng.uniform(1, 10)
        P0 = np.diag([1, 1, 1, 4, 0.01, 0.01]).astype(float)
        # linear transport matrices taken from the closed-form helix around the reference
        steps = np.array([1e-6, 1e-6, 1e-6, 1e-8, 1e-8, 1e-8])
        x_lin = p_ref + rng.normal(size=6) * np.sqrt(np.diag(P0)) * 0.1
        Fs, refs = [], []
        cur = p_ref
        for l in range(10):
            nxt = BF.propagate_cf(cur, l, geom, BZ, nearest=True)
            Fs.append(BF.num_jacobian(lambda q: BF.propagate_cf(q, l, geom, BZ, nearest=True), cur, steps))
            refs.append((cur, nxt))
            cur = nxt
        # hits: measurements generated from the linear model around the references
        est, Pk = x_lin.copy(), orc.pack(P0)
        dev = x_lin - p_ref                           # linear deviation from reference
        A_rows, b_rows = [], []
        Ftot = np.eye(6)
        state_dev, cov = dev.copy(), P0.copy()
        for l in range(10):
            F = Fs[l]
            state_dev = F @ state_dev
            cov = F @ cov @ F.T
            Ftot = F @ Ftot
            ref_l = refs[l][1]
            q = ref_l + state_dev
            rho = np.hypot(ref_l[0], ref_l[1])
            phh = math.atan2(ref_l[1], ref_l[0]) + rng.normal() * 1e-4
            hit = np.array([rho * math.cos(phh), rho * math.sin(phh), ref_l[2] + rng.normal() * 0.05,
                            0.01, 0.05])
            st, qn, Pn, c2 = orc.update(q, orc.pack(cov), hit, 0)
            assert st == 0
            state_dev = qn - ref_l
            state_dev[4] = wrap(state_dev[4])
            cov = orc.unpack(Pn)
            # normal-equation rows in terms of the initial deviation
            rhoh = math.hypot(hit[0], hit[1])
            cp, sp = hit[0] / rhoh, hit[1] / rhoh
            H = np.zeros((2, 6))
            H[0, :2] = [-sp, cp]
            H[1, 2] = 1
            z0 = BF.measure(ref_l, hit, 0)          # residual at zero deviation
            W = np.diag([1 / 0.01, 1 / 0.05])
            A_rows.append(W @ H @ Ftot)
            b_rows.append(W @ z0)
        A = np.vstack(A_rows)
        b = np.concatenate(b_rows)
        P0i = np.linalg.inv(P0)
        N = A.T @ A + P0i
        dev_hat = np.linalg.solve(N, A.T @ b + P0i @ dev)
        final_dev = Ftot @ dev_hat
        final_cov = Ftot @ np.linalg.inv(N) @ Ftot.T
        d = state_dev - final_dev
        sig = np.sqrt(np.maximum(np.diag(final_cov), 1e-30))
        keep = np.diag(final_cov) > 1e-14
        assert np.abs(d[keep] / sig[keep]).max() < 1e-7, d / sig
        assert np.allclose(cov, final_cov, rtol=1e-6, atol=1e-12)


# ---------------------------------------------------------------- fit
def _fit(orc, geom, ev, cfg=None):
    cfg = cfg or orc.Config(geom)
    par0, cov0 = orc.seeds_for_event(ev)
    hits = dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv)
    return orc.fit(cfg, hits, ev.seq_layer, ev.seq_hit, par0, cov0)


def _pulls(orc, ev, r):
    # the filter adds a layer's scattering noise at that layer, so its final
    # state describes the track after the last kick
    nh = ev.n_track_hits()
    tr = ev.truth_out[np.arange(ev.n_tracks), nh - 1]
    P = orc.unpack(r["cov"])
    d = r["par"] - tr
    d[:, 4] = wrap(d[:, 4])
    pp = np.arctan2(tr[:, 1], tr[:, 0])
    du = -np.sin(pp) * d[:, 0] + np.cos(pp) * d[:, 1]
    Huu = (np.sin(pp) ** 2 * P[:, 0, 0] + np.cos(pp) ** 2 * P[:, 1, 1]
           - 2 * np.sin(pp) * np.cos(pp) * P[:, 0, 1])
    return {"u": du / np.sqrt(Huu), "z": d[:, 2] / np.sqrt(P[:, 2, 2]),
            "c": d[:, 3] / np.sqrt(P[:, 3, 3]), "phi": d[:, 4] / np.sqrt(P[:, 4, 4]),
            "theta": d[:, 5] / np.sqrt(P[:, 5, 5])}


def test_fit_equals_batch_least_squares(orc):
    """T5: the EKF (no material) agrees with the Gauss-Newton-converged batch
    weighted least squares (independent closed-form propagation, numerical
    derivatives) to a small fraction of a standard deviation."""
    geom, ev = E.fit_sample(n_tracks=40, seed=7)
    r = _fit(orc, geom, ev)
    worst = 0.0
    for t in range(ev.n_tracks):
        nh = ev.n_track_hits()[t]
        if nh < 6 or r["status"][t]:
            continue
        hs = [np.array([ev.x[i], ev.y[i], ev.z[i], ev.su[i], ev.sv[i]], float)
              for i in ev.seq_hit[t, :nh]]
        lays = list(ev.seq_layer[t, :nh])
        p_seed, P0k = orc.seed(hs[0][:3], hs[1][:3], hs[2][:3])
        p_star, cov_star, chi2_wls = BF.wls_fit(p_seed, orc.unpack(P0k), hs, lays, geom, BZ)
        fin = BF.propagate_cf(p_star, lays[-1], geom, BZ, nearest=True)
        P = orc.unpack(r["cov"][t])
        d = r["par"][t] - fin
        d[4] = wrap(d[4])
        sig = np.sqrt(np.diag(P))
        z = np.abs(d[2:] / sig[2:])
        ph = math.atan2(fin[1], fin[0])
        du = -math.sin(ph) * d[0] + math.cos(ph) * d[1]
        su = math.sqrt(math.sin(ph) ** 2 * P[0, 0] + math.cos(ph) ** 2 * P[1, 1]
                       - 2 * math.sin(ph) * math.cos(ph) * P[0, 1])
        worst = max(worst, z.max(), abs(du) / su)
        # the EKF chi2 is not below the least-squares minimum (up to linearisation)
        assert r["chi2"][t] > chi2_wls - 0.05 * max(1.0, chi2_wls)
    assert worst < 0.2, worst


def test_fit_pulls_and_chi2(orc):
    """T6: 10^4 tracks, no material: pulls unit width, chi2/ndf ~ 1, flat p-value."""
    geom, ev = E.fit_sample(n_tracks=10_000, seed=8)
    r = _fit(orc, geom, ev)
    ok = r["status"] == 0
    assert ok.mean() > 0.999
    for k, v in _pulls(orc, ev, r).items():
        v = v[ok]
        assert abs(v.mean()) < 0.03, (k, v.mean())
        assert abs(v.std() - 1) < 0.03, (k, v.std())
    assert abs((r["chi2"][ok] / r["ndf"][ok]).mean() - 1) < 0.03
    pv = stats.chi2.sf(r["chi2"][ok], r["ndf"][ok])
    assert stats.kstest(pv, "uniform").pvalue > 1e-3


def test_fit_pulls_with_material(orc):
    """T7: with 0.02 X0 per layer the scattering noise makes pulls unit width."""
    geom, evs = E.find_events(n_events=1, n_tracks=5000, n_noise=0, seed=9)
    ev = evs[0]
    r = _fit(orc, geom, ev)
    ok = (r["status"] == 0) & (ev.n_track_hits() >= 6)
    for k, v in _pulls(orc, ev, r).items():
        v = v[ok]
        assert abs(v.mean()) < 0.05, (k, v.mean())
        assert abs(v.std() - 1) < 0.05, (k, v.std())
    assert abs((r["chi2"][ok] / r["ndf"][ok]).mean() - 1) < 0.05


def test_scattering_noise_matches_kicks(orc):
    """The process noise Q the filter adds equals the covariance of the
    generator's Gaussian kicks (toy Monte Carlo, statistical tolerance)."""
    geom = E.geometry.barrel10(x0=0.05)
    cfg = orc.Config(geom)
    rng = np.random.default_rng(50)
    for c, phi, th, r_l in ((1.0, 0.3, 1.2, 25.0), (-0.2, -2.0, 0.9, 50.0), (3.0, 1.0, 1.35, 7.0)):
        pos_phi = phi - 0.1
        p = np.array([r_l * math.cos(pos_phi), r_l * math.sin(pos_phi), 1.0, c, phi, th])
        layer = E.geometry.BARREL_R.index(r_l)
        Pz = orc.pack(np.eye(6) * 1e-12)
        _, _, Qa, *_ = orc.propagate(cfg, layer, p, Pz, noise=True)
        _, _, Qb, *_ = orc.propagate(cfg, layer, p, Pz, noise=False)
        Q = orc.unpack(Qa) - orc.unpack(Qb)
        n = 400_000
        ones = np.ones(n)
        nc, nphi, nth = GEN.scatter_kick(rng, p[0] * ones, p[1] * ones, c * ones, phi * ones,
                                         th * ones, np.zeros(n, int), 0.05 * ones)
        D = np.stack([nc - c, wrap(nphi - phi), nth - th], axis=1)
        emp = np.cov(D.T)
        idx = [3, 4, 5]
        Qs = Q[np.ix_(idx, idx)]
        for i in range(3):
            assert abs(emp[i, i] / Qs[i, i] - 1) < 0.02, (i, emp[i, i], Qs[i, i])
        corr_q = Qs[0, 2] / math.sqrt(Qs[0, 0] * Qs[2, 2])
        corr_e = emp[0, 2] / math.sqrt(emp[0, 0] * emp[2, 2])
        assert abs(corr_q - corr_e) < 0.02


def test_generator_hits_on_surfaces_and_smearing(orc):
    """Generated crossings lie on the oracle's helix; smearing pulls are N(0,1)."""
    geom, ev = E.fit_sample(n_tracks=2000, seed=10)
    pu, pv = [], []
    for t in range(200):
        nh = ev.n_track_hits()[t]
        for k in range(nh - 1):
            a, b = ev.truth_at[t, k], ev.truth_at[t, k + 1]
            r_b = geom[ev.seq_layer[t, k + 1]]["r_or_z"]
            cfg = orc.Config(geom)
            st, s, it = orc.solve_barrel(cfg, a, r_b)
            q = orc.helix(a, s, 3.8)
            assert np.allclose(q[:3], b[:3], atol=1e-8)
    tr = ev.truth_at.reshape(-1, 6)
    hits = ev.seq_hit.reshape(-1)
    m = hits >= 0
    tr, hits = tr[m], hits[m]
    pt = np.arctan2(tr[:, 1], tr[:, 0])
    rt = np.hypot(tr[:, 0], tr[:, 1])
    ph = np.arctan2(ev.y[hits], ev.x[hits]).astype(float)
    du = wrap(ph - pt) * rt / ev.su[hits]
    dv = (ev.z[hits] - tr[:, 2]) / ev.sv[hits]
    assert stats.kstest(du, "norm").pvalue > 1e-3
    assert stats.kstest(dv, "norm").pvalue > 1e-3


# ---------------------------------------------------------------- finding
@pytest.fixture(scope="module")
def find_event():
    geom, evs = E.find_events(n_events=1, seed=1)
    return geom, evs[0]


def _seeds(ev):
    nh = ev.n_track_hits()
    sel = np.nonzero(nh >= 3)[0]
    return sel, ev.seq_hit[sel, :3]


def test_binned_equals_all_hits(orc, find_event):
    """T9: the binned window search and the scan of every hit of the layer give
    identical hit lists."""
    geom, ev = find_event
    cfg = orc.Config(geom)
    sel, seeds = _seeds(ev)
    seeds = seeds[:250]
    rb = orc.find(cfg, ev, seeds, binned=True)
    ra = orc.find(cfg, ev, seeds, binned=False)
    assert np.array_equal(rb["hits"], ra["hits"])
    assert np.array_equal(rb["chi2"], ra["chi2"])


def test_noise_free_finds_true_hits(orc):
    """T10: no noise, no scattering, sigma = 0.002 cm: every seed finds exactly
    its own track's hits."""
    rng = np.random.default_rng(60)
    geom = E.geometry.barrel10(x0=0.0, su=0.002, sv=0.002)
    ev = E.make_event(rng, geom, 800, E.pt_power2(0.5, 50.0), 1.0, 0)
    cfg = orc.Config(geom)
    sel, seeds = _seeds(ev)
    r = orc.find(cfg, ev, seeds)
    for k, t in enumerate(sel):
        want = np.full(len(geom), -1)
        nh = ev.n_track_hits()[t]
        want[ev.seq_layer[t, :nh]] = ev.seq_hit[t, :nh]
        assert np.array_equal(r["hits"][k], want), (t, r["hits"][k], want)
        # the walk reaches the layers after the three seed layers one per
        # step, in crossing order (ten barrels: radius order)
        walked = ev.seq_layer[t, 3:nh]
        assert np.array_equal(r["visit"][k][walked], np.arange(walked.size)), r["visit"][k]
        assert (r["visit"][k][ev.seq_layer[t, :3]] == -1).all()


def _exhaustive_best(orc, cfg, geom, ev, seed_hits):
    """All hit / no-hit combinations along the layer sequence (same stopping
    rules: 3 consecutive misses, end of detector), best by (hits, chi2)."""
    p, P = orc.seed(*[np.array([ev.x[i], ev.y[i], ev.z[i]], float) for i in seed_hits])
    chi2 = 0.0
    hits = {}
    for i in seed_hits:
        L = ev.layer[i]
        st, p, P, *_ = orc.propagate(cfg, L, p, P, noise=cfg.c.use_material)
        assert st == 0
        st, p, P, c2 = orc.update(p, P, np.array([ev.x[i], ev.y[i], ev.z[i], ev.su[i], ev.sv[i]],
                                                 float), geom[L]["kind"])
        chi2 += c2
        hits[L] = int(i)
    results = []
    layer_hits = {l: np.nonzero(ev.layer == l)[0] for l in range(len(geom))}

    def rec(p, P, chi2, hits, misses):
        rho = math.hypot(p[0], p[1])
        nxt = [l for l in range(len(geom)) if geom[l]["r_or_z"] > rho + 0.05]
        if not nxt:
            results.append((len(hits), chi2, dict(hits)))
            return
        l = min(nxt, key=lambda j: geom[j]["r_or_z"])
        st, q, Q, s, it = orc.propagate(cfg, l, p, P, noise=cfg.c.use_material)
        if st or abs(q[2]) > geom[l]["hi"]:
            results.append((len(hits), chi2, dict(hits)))
            return
        for i in layer_hits[l]:
            hit = np.array([ev.x[i], ev.y[i], ev.z[i], ev.su[i], ev.sv[i]], float)
            if hit[0] * q[0] + hit[1] * q[1] <= 0:
                continue
            c2 = orc.chi2(q, Q, hit, 0)
            if c2 < cfg.c.chi2_cut:
                st, pn, Pn, c2u = orc.update(q, Q, hit, 0)
                hits[l] = int(i)
                rec(pn, Pn, chi2 + c2, hits, 0)
                del hits[l]
        if misses + 1 > cfg.c.max_miss:
            results.append((len(hits), chi2, dict(hits)))
        else:
            rec(q, Q, chi2, hits, misses + 1)

    rec(p, P, chi2, hits, 0)
    results.sort(key=lambda r: (-r[0], r[1]))
    return results


def test_beam_search_equals_exhaustive(orc):
    """T11: with an unbounded candidate count the beam search returns the best
    of all hit/no-hit combinations (tiny events: 3 tracks, 20 noise hits, 6 layers)."""
    geom = E.geometry.barrel10(x0=0.02)[:6]
    cfg = orc.Config(geom, max_cands=100_000)
    rng = np.random.default_rng(70)
    n_checked = 0
    for trial in range(15):
        ev = E.make_event(rng, geom, 3, E.pt_power2(0.5, 5.0), 1.0, 0)
        # dense noise near the tracks so that branching really happens
        extra = []
        for t in range(3):
            for k in range(3, ev.n_track_hits()[t]):
                i = ev.seq_hit[t, k]
                for _ in range(2):
                    extra.append((ev.x[i], ev.y[i], ev.z[i], ev.layer[i]))
        extra = extra[:20]
        r = np.hypot([e[0] for e in extra], [e[1] for e in extra]).astype(float)
        ph = np.arctan2([e[1] for e in extra], [e[0] for e in extra]) + rng.normal(0, 0.002, len(extra))
        ev.x = np.concatenate([ev.x, (r * np.cos(ph)).astype(np.float32)])
        ev.y = np.concatenate([ev.y, (r * np.sin(ph)).astype(np.float32)])
        ev.z = np.concatenate([ev.z, np.array([e[2] for e in extra], np.float32) + rng.normal(0, 0.1, len(extra)).astype(np.float32)])
        ev.layer = np.concatenate([ev.layer, np.array([e[3] for e in extra], np.int32)])
        ev.su = np.concatenate([ev.su, np.full(len(extra), 0.01, np.float32)])
        ev.sv = np.concatenate([ev.sv, np.full(len(extra), 0.05, np.float32)])
        ev.sim = np.concatenate([ev.sim, np.full(len(extra), -1, np.int32)])
        sel, seeds = _seeds(ev)
        res = orc.find(cfg, ev, seeds, binned=False)
        for k, t in enumerate(sel):
            allr = _exhaustive_best(orc, cfg, geom, ev, seeds[k])
            best = allr[0]
            if len(allr) > 1 and allr[1][0] == best[0] and abs(allr[1][1] - best[1]) < 1e-9:
                continue
            want = np.full(len(geom), -1)
            for l, i in best[2].items():
                want[l] = i
            assert np.array_equal(res["hits"][k], want), (trial, t, res["hits"][k], want)
            assert abs(res["chi2"][k] - best[1]) < 1e-9 * max(1, best[1])
            n_checked += 1
    assert n_checked >= 30


def test_binned_equals_all_hits_with_disks(orc):
    """T9 on the barrel + disk geometry (|eta| < 2.5, noise 60 per track)."""
    geom, evs = E.batch_events(n_events=2, seed=21, lam_lo=300, lam_hi=400)
    cfg = orc.Config(geom)
    for ev in evs:
        sel, seeds = _seeds(ev)
        seeds = seeds[:150]
        rb = orc.find(cfg, ev, seeds, binned=True)
        ra = orc.find(cfg, ev, seeds, binned=False)
        assert np.array_equal(rb["hits"], ra["hits"])
        assert np.array_equal(rb["chi2"], ra["chi2"])


def test_disk_fit_pulls(orc):
    """Forward tracks crossing disks: fit pulls unit width with scattering."""
    rng = np.random.default_rng(22)
    geom = E.geometry.barrel10_disks14(x0=0.02)
    ev = E.make_event(rng, geom, 4000, E.pt_power2(0.5, 50.0), 2.5, 0)
    r = _fit(orc, geom, ev)
    nh = ev.n_track_hits()
    ok = (r["status"] == 0) & (nh >= 6)
    tr = ev.truth_out[np.arange(ev.n_tracks), nh - 1]
    P = orc.unpack(r["cov"])
    d = r["par"] - tr
    d[:, 4] = wrap(d[:, 4])
    for i, name in ((3, "c"), (4, "phi"), (5, "theta")):
        v = (d[:, i] / np.sqrt(P[:, i, i]))[ok]
        assert abs(v.mean()) < 0.05 and abs(v.std() - 1) < 0.05, (name, v.mean(), v.std())
    assert abs((r["chi2"][ok] / r["ndf"][ok]).mean() - 1) < 0.05


# ---------------------------------------------------------------- seed
@pytest.mark.parametrize("pt", [0.35, 1.0, 7.0, 100.0])
def test_seed_of_noise_free_helix_hits(orc, pt):
    """The three-hit seed (circle through the transverse positions, tangent at
    hit 1, dip from the arc) of noise-free hits on an analytic helix returns
    that helix's state at hit 1: position, q/pT, phi and theta to 1e-9.  The
    hits are the closed-form crossings of brute force (circle-circle
    intersection for barrels, the rotation about the centre for disks), both
    charges, |eta| up to 2.5, barrel and disk triplets."""
    geom = E.geometry.barrel10_disks14(x0=0.0)
    rng = np.random.default_rng(int(pt * 1000) + 7)
    n_checked = {0: 0, 1: 0}
    for trial in range(400):
        q = rng.choice([-1.0, 1.0])
        eta = rng.uniform(-2.5, 2.5)
        th = 2 * math.atan(math.exp(-eta))
        p = np.array([rng.normal(0, 0.01), rng.normal(0, 0.01), rng.normal(0, 0.01), q / pt,
                      rng.uniform(-np.pi, np.pi), th])
        # the first three surfaces the track crosses, by closed forms
        hits = []
        cur = p.copy()
        for _ in range(3):
            best = None
            for l, L in enumerate(geom):
                if L["kind"] == 0:
                    if L["r_or_z"] <= math.hypot(cur[0], cur[1]) + 1e-6:
                        continue
                    r = BF.cf_barrel(cur, L["r_or_z"], BZ)
                    if r is None or abs(r[0][2]) > L["hi"]:
                        continue
                else:
                    if (L["r_or_z"] - cur[2]) * math.cos(th) <= 1e-6:
                        continue
                    r = BF.cf_disk(cur, L["r_or_z"], BZ)
                    rho = math.hypot(r[0][0], r[0][1])
                    if not (L["lo"] <= rho <= L["hi"]):
                        continue
                if r[1] > 0 and (best is None or r[1] < best[1]):
                    best = (r[0], r[1], L["kind"])
            if best is None:
                break
            hits.append(best)
            cur = best[0]
        if len(hits) < 3:
            continue
        kinds = {k for _, _, k in hits}
        for k in kinds:
            n_checked[k] += 1
        want = hits[0][0]
        got, P = orc.seed(want[:3], hits[1][0][:3], hits[2][0][:3], BZ)
        assert np.abs(got[:3] - want[:3]).max() < 1e-9
        assert abs(got[3] - want[3]) < 1e-9 * max(abs(want[3]), 1.0)
        assert abs(wrap(got[4] - want[4])) < 1e-9
        assert abs(got[5] - want[5]) < 1e-9
        # the prior is the fixed diffuse diagonal
        assert np.allclose(orc.unpack(P), np.diag([1, 1, 1, 4, 0.01, 0.01]))
    assert n_checked[0] > 100 and n_checked[1] > 20, n_checked
