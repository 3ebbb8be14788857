"""Pins of the oracle's r-z material map and mean energy loss (Sec. 3.1:
scattering and energy loss from two-dimensional material arrays indexed in
r-z): the Bethe minimum against the PDG value for silicon, the input
generator's independent implementation, kinematics after the loss, the
Jacobian against finite differences, the map lookup by construction, and fit
pulls on tracks simulated with energy loss (unbiased with the correction,
biased without it)."""
import numpy as np
import pytest

import eventgen as E
import eventgen.material as EM
from eventgen.generate import _bethe_si

M_PI = 0.13957


def test_bethe_minimum_matches_pdg_silicon(orc):
    """Minimum ionisation in silicon: PDG 1.664 MeV cm^2/g near beta gamma
    3-3.5 (with the density effect, which lowers the minimum by ~2%; it is
    not modelled here)."""
    m = 0.10566
    bg = np.logspace(-0.3, 2.5, 400)
    d = np.array([orc.dedx(b * m, m) for b in bg])
    i = int(np.argmin(d))
    assert 2.5 < bg[i] < 4.0
    assert d[i] == pytest.approx(1.664, rel=0.03)
    # slow particles lose more (the 1/beta^2 rise below the minimum)
    assert d[0] > 3 * d[i]


def test_bethe_matches_generator_implementation(orc):
    """Two independent implementations of the same published formula (the
    oracle's C, the input generator's numpy) agree: catches a slipped
    constant or term in either."""
    for m in (M_PI, 0.10566, 0.938):
        for p in (0.1, 0.3, 1.0, 5.0, 100.0):
            assert orc.dedx(p, m) == pytest.approx(float(_bethe_si(np.array(p), m)), rel=1e-12)


def _one_barrel_map(orc, x0_pos, x0_neg=0.0, r=50.0):
    geom = [dict(kind=0, r_or_z=r, lo=-100.0, hi=100.0, x0=0.0, nbin_phi=64, nbin_2=16,
                 win_su=0.01, win_sv=0.05)]
    nr, nz = 250, 250
    x0 = np.zeros((nr, nz))
    ir = int(np.floor(r / (120.0 / nr)))
    zc = -300 + (np.arange(nz) + 0.5) * 600 / nz
    x0[ir] = np.where(zc > 0, x0_pos, x0_neg)
    mat = dict(r_max=120.0, z_min=-300.0, z_max=300.0, x0=x0, xi=x0 * EM.X0_SI)
    return geom, orc.Config(geom, material_map=mat)


def test_map_lookup_by_construction(orc):
    """A barrel with material only at z > 0: a crossing at z < 0 is left
    unchanged; at z > 0 the covariance gains exactly the noise of a layer of
    that thickness without a map, and c grows by the mean loss."""
    geom, cfg = _one_barrel_map(orc, 0.03)
    P = orc.pack(np.diag([1e-4, 1e-4, 1e-3, 1e-4, 1e-6, 1e-6]))
    for z, has in ((-20.0, False), (20.0, True)):
        q = np.array([50 * np.cos(0.3), 50 * np.sin(0.3), z, 1.2, 0.35, 1.4])
        q1, P1 = orc.material(cfg, 0, q, P)
        if not has:
            assert np.array_equal(q1, q) and np.array_equal(P1, P)
            continue
        geom2 = [dict(geom[0], x0=0.03)]
        q2, P2 = orc.material(orc.Config(geom2), 0, q, P)        # scattering only
        assert np.array_equal(q2, q)
        assert abs(q1[3]) > abs(q[3])
        assert np.array_equal(q1[[0, 1, 2, 4, 5]], q[[0, 1, 2, 4, 5]])
        # away from the c row/column the two agree exactly
        U1, U2 = orc.unpack(P1), orc.unpack(P2)
        keep = [0, 1, 2, 4, 5]
        assert np.allclose(U1[np.ix_(keep, keep)], U2[np.ix_(keep, keep)], rtol=1e-15, atol=0)


def test_energy_loss_kinematics(orc):
    """After the loss the energy is E - dE with dE = dE/dx * xi / cos(alpha),
    the direction and the charge are unchanged."""
    geom, cfg = _one_barrel_map(orc, 0.05)
    P = orc.pack(np.eye(6) * 1e-6)
    rng = np.random.default_rng(1)
    for _ in range(20):
        phi_pos = rng.uniform(-np.pi, np.pi)
        q = np.array([50 * np.cos(phi_pos), 50 * np.sin(phi_pos), rng.uniform(1, 90),
                      rng.choice([-1, 1]) / rng.uniform(0.3, 5), phi_pos + rng.uniform(-0.5, 0.5),
                      rng.uniform(0.8, 2.3)])
        q1, _ = orc.material(cfg, 0, q, P)
        assert np.sign(q1[3]) == np.sign(q[3])
        p0 = 1 / (abs(q[3]) * np.sin(q[5]))
        p1 = 1 / (abs(q1[3]) * np.sin(q1[5]))
        cosa = abs(np.sin(q[5]) * np.cos(q[4] - phi_pos))
        dE = orc.dedx(p0) * 0.05 * EM.X0_SI / cosa * 1e-3
        E0 = np.hypot(p0, M_PI)
        assert np.hypot(p1, M_PI) == pytest.approx(E0 - dE, rel=1e-13)


def test_energy_loss_jacobian(orc):
    """dc'/dc = (p/p')^3 E'/E against central differences, at minimum
    ionisation (where dE does not depend on p to first order) and a thick
    layer (p/p' ~ 1.07, so a wrong power of p/p' would show by ~7%)."""
    geom, cfg = _one_barrel_map(orc, 1.0)
    m = M_PI
    p = 3.6 * m
    q = np.array([50.0, 0.0, 10.0, 1 / p, 0.0, np.pi / 2])
    P = orc.pack(np.eye(6) * 1e-6)
    q1, P1 = orc.material(cfg, 0, q, P)
    J = np.sqrt(orc.unpack(P1)[3, 3] / 1e-6)
    h = 1e-6 * q[3]
    qa, qb = q.copy(), q.copy()
    qa[3] += h
    qb[3] -= h
    fd = (orc.material(cfg, 0, qa, P)[0][3] - orc.material(cfg, 0, qb, P)[0][3]) / (2 * h)
    ratio = q1[3] / q[3]
    assert ratio > 1.05
    assert J == pytest.approx(fd, rel=5e-3)


def _fit_pulls(orc, geom, mat, ev):
    par0, cov0 = orc.seeds_for_event(ev)
    cfg = orc.Config(geom, material_map=mat)
    r = orc.fit(cfg, dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv), ev.seq_layer, ev.seq_hit,
                par0, cov0, n_threads=8)
    nh = ev.n_track_hits()
    ok = (r["status"] == 0) & (nh >= 8)
    last = nh[ok] - 1
    truth = ev.truth_out[np.nonzero(ok)[0], last]
    P = orc.unpack(r["cov"][ok])
    d = r["par"][ok] - truth
    # signed by the charge: the loss raises |c| for both signs
    return np.sign(truth[:, 3]) * d[:, 3] / np.sqrt(P[:, 3, 3]), r["chi2"][ok] / r["ndf"][ok]


def test_fit_with_energy_loss_is_unbiased(orc):
    """3,000 tracks of pT 0.5-1 GeV through ten barrels of ~0.05 X0 from the
    map, simulated with scattering and energy loss: with the map's loss the
    curvature pull (signed by the charge) is centred with unit width; with the loss switched off (xi
    = 0, same scattering) it is biased by more than half a sigma."""
    geom, mat, ev = EM.eloss_sample(n_tracks=3000, seed=22)
    pull, c2 = _fit_pulls(orc, geom, mat, ev)
    print(f"with loss: c pull mean {pull.mean():.3f} std {pull.std():.3f}, chi2/ndf {c2.mean():.3f}")
    assert abs(pull.mean()) < 0.1
    assert 0.9 < pull.std() < 1.15
    assert 0.9 < c2.mean() < 1.15
    mat0 = dict(mat, xi=np.zeros_like(mat["xi"]))
    pull0, _ = _fit_pulls(orc, geom, mat0, ev)
    print(f"without loss: c pull mean {pull0.mean():.3f}")
    assert abs(pull0.mean()) > 0.5
