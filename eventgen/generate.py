"""Seeded synthetic helix events (input generator shared by the oracle tests,
the GPU parity tests and the benchmark).

The paper measures on simulated CMS ttbar events, which are not available;
these events stand in for them: charged helices in a uniform solenoid field,
one smeared hit per crossed detector surface, optional Gaussian
multiple-scattering kicks at every crossing, plus uniform noise hits.

The transport here is simulation, written independently of the filter code:
crossings use the closed-form intersection of the track circle with the
layer circle (barrel) or the linear z solution (disk), evaluated through the
centre-of-curvature rotation.  Hits are stored as float32, truth in float64.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import geometry as G

KAPPA = 0.00299792458           # GeV / (T cm): pT = KAPPA * B * R
PION_MASS = 0.13957             # GeV
NEXT_BARREL_EPS = 0.05          # cm: a barrel counts as "ahead" if r > rho + eps


@dataclass
class Event:
    """One event (or one track sample), hits in shuffled order."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    su: np.ndarray
    sv: np.ndarray
    layer: np.ndarray           # int32
    sim: np.ndarray             # int32, track id within the event, -1 = noise
    truth0: np.ndarray          # [n_trk, 6] float64 (x, y, z, c, phi, theta) at production
    seq_hit: np.ndarray         # [n_trk, max_steps] int32 hit index in crossing order, -1 pad
    seq_layer: np.ndarray       # [n_trk, max_steps] int32 layer crossed, -1 pad
    truth_at: np.ndarray        # [n_trk, max_steps, 6] float64 true state at each crossing (before kick)
    truth_out: np.ndarray = None  # same, after the scattering kick at that crossing

    @property
    def n_hits(self):
        return int(self.x.shape[0])

    @property
    def n_tracks(self):
        return int(self.truth0.shape[0])

    def n_track_hits(self):
        return (self.seq_hit >= 0).sum(axis=1)


def _wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def _pos_at(x, y, phi, h, s):
    """Transverse position after arc length s (textbook difference form)."""
    a = h * s
    return (x + (np.sin(phi + a) - np.sin(phi)) / h,
            y + (np.cos(phi) - np.cos(phi + a)) / h)


def _barrel_crossing(x, y, phi, h, r_l):
    """Arc length to the outward crossing of radius r_l (closed form, via the
    circle-circle intersection).  Returns (s, ok)."""
    inv = 1.0 / h
    cx = x - np.sin(phi) * inv
    cy = y + np.cos(phi) * inv
    rad = np.abs(inv)
    d = np.hypot(cx, cy)
    a = (r_l * r_l - rad * rad + d * d) / (2.0 * d)
    disc = r_l * r_l - a * a
    ok = disc >= 0.0
    hh = np.sqrt(np.where(ok, disc, 0.0))
    ux, uy = cx / d, cy / d
    best_s = np.full(x.shape, np.inf)
    for sgn in (1.0, -1.0):
        px = a * ux - sgn * hh * uy
        py = a * uy + sgn * hh * ux
        v0x, v0y = x - cx, y - cy
        v1x, v1y = px - cx, py - cy
        alpha = np.arctan2(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y)
        s = np.mod(np.sign(h) * alpha, 2.0 * np.pi) / np.abs(h)
        ph = phi + h * s
        outward = px * np.cos(ph) + py * np.sin(ph) > 0.0
        take = ok & outward & (s < best_s)
        best_s = np.where(take, s, best_s)
    return best_s, ok & np.isfinite(best_s)


def _highland(c, theta, t):
    p = 1.0 / (np.abs(c) * np.sin(theta))
    beta = p / np.sqrt(p * p + PION_MASS * PION_MASS)
    return 0.0136 / (beta * p) * np.sqrt(t) * (1.0 + 0.038 * np.log(t / (beta * beta)))


def _bethe_si(p, m):
    """Mean ionisation loss in silicon [MeV cm^2/g] (Bethe formula with the
    maximum energy transfer, no density effect): the truth simulation's
    energy loss."""
    me, K, za, I = 0.51099895, 0.307075, 0.49848, 173e-6
    M = m * 1e3
    E = np.sqrt((p * 1e3) ** 2 + M * M)
    beta = p * 1e3 / E
    gam = E / M
    bg2 = (beta * gam) ** 2
    tmax = 2 * me * bg2 / (1 + 2 * gam * me / M + (me / M) ** 2)
    return K * za / beta ** 2 * (0.5 * np.log(2 * me * bg2 * tmax / I ** 2) - beta ** 2)


def map_cell(mat, x, y, z):
    """Cell values (x0, xi) of a material map at points (x, y, z)."""
    nr, nz = mat["x0"].shape
    ir = np.clip(np.floor(np.hypot(x, y) / (mat["r_max"] / nr)).astype(np.int64), 0, nr - 1)
    iz = np.clip(np.floor((z - mat["z_min"]) / ((mat["z_max"] - mat["z_min"]) / nz)).astype(np.int64),
                 0, nz - 1)
    return mat["x0"][ir, iz].astype(np.float64), mat["xi"][ir, iz].astype(np.float64)


def transport(rng, st, q, geom, bz, smear_fn, max_steps=None, material=None):
    """Walk every track through the detector.

    st: dict of float64 arrays x, y, z, c, phi, theta (production point).
    Navigation: the next surface is the one reached first (smallest positive
    transverse arc length) among the next barrel outward (radius above the
    current one, crossing within its z extent) and the first disk ahead in z
    whose crossing lies within its radial extent.  Tracks stop after half a
    turn in the transverse plane or when no surface is left.  With a material
    map (dict r_max, z_min, z_max, x0 [nr, nz], xi [nr, nz]) the thickness at
    each crossing is the map's cell, and the particle also loses its mean
    ionisation energy there (momentum magnitude only).
    Returns per-track lists of crossings: (layer, state6 at crossing, s).
    """
    n = st["x"].shape[0]
    nl = len(geom)
    if max_steps is None:
        max_steps = nl
    barrels = [i for i, L in enumerate(geom) if L["kind"] == 0]
    disks = [i for i, L in enumerate(geom) if L["kind"] == 1]
    b_r = np.array([geom[i]["r_or_z"] for i in barrels])
    kb = KAPPA * bz
    x, y, z = st["x"].copy(), st["y"].copy(), st["z"].copy()
    c, phi, th = st["c"].copy(), st["phi"].copy(), st["theta"].copy()
    alive = np.ones(n, bool)
    turned = np.zeros(n)
    out_layer = np.full((n, max_steps), -1, np.int32)
    out_state = np.zeros((n, max_steps, 6))
    out_after = np.zeros((n, max_steps, 6))
    for step in range(max_steps):
        if not alive.any():
            break
        h = -kb * c
        rho = np.hypot(x, y)
        best_s = np.full(n, np.inf)
        best_l = np.full(n, -1, np.int64)
        # next barrel
        if barrels:
            k = np.searchsorted(b_r, rho + NEXT_BARREL_EPS, side="right")
            has = k < len(barrels)
            kk = np.minimum(k, len(barrels) - 1)
            r_l = b_r[kk]
            s_b, ok = _barrel_crossing(x, y, phi, h, r_l)
            zb = z + s_b * np.cos(th) / np.sin(th)
            lay = np.array(barrels)[kk]
            zmax = np.array([geom[i]["hi"] for i in barrels])[kk]
            ok &= has & (np.abs(zb) <= zmax) & (s_b > 1e-9)
            best_s = np.where(ok, s_b, best_s)
            best_l = np.where(ok, lay, best_l)
        # first disk ahead within its radial extent
        for i in disks:
            L = geom[i]
            s_d = (L["r_or_z"] - z) * np.tan(th)
            px, py = _pos_at(x, y, phi, h, s_d)
            rr = np.hypot(px, py)
            ok = (s_d > 1e-9) & (rr >= L["lo"]) & (rr <= L["hi"]) & (s_d < best_s)
            best_s = np.where(ok, s_d, best_s)
            best_l = np.where(ok, i, best_l)
        go = alive & (best_l >= 0) & (turned + np.abs(h) * np.where(np.isfinite(best_s), best_s, 0) <= np.pi)
        alive &= go
        if not go.any():
            break
        s = np.where(go, best_s, 0.0)
        nx, ny = _pos_at(x, y, phi, h, s)
        nz = z + s * np.cos(th) / np.sin(th)
        nphi = _wrap(phi + h * s)
        turned = turned + np.abs(h) * s
        x = np.where(go, nx, x)
        y = np.where(go, ny, y)
        z = np.where(go, nz, z)
        phi = np.where(go, nphi, phi)
        # snap onto the surface (removes round-off of the closed form)
        lay = np.where(go, best_l, 0)
        for i in set(lay[go].tolist()):
            m = go & (lay == i)
            if geom[i]["kind"] == 0:
                rr = np.hypot(x[m], y[m])
                x[m] *= geom[i]["r_or_z"] / rr
                y[m] *= geom[i]["r_or_z"] / rr
            else:
                z[m] = geom[i]["r_or_z"]
        out_layer[go, step] = best_l[go]
        out_state[go, step] = np.stack([x, y, z, c, phi, th], axis=1)[go]
        # multiple scattering at the crossed surface
        kind = np.array([geom[i]["kind"] for i in range(nl)])[lay]
        if material is None:
            x0 = np.array([geom[i]["x0"] for i in range(nl)])[lay]
            xi = np.zeros(n)
        else:
            x0, xi = map_cell(material, x, y, z)
        mat = go & (x0 > 0)
        if mat.any():
            c, phi, th = scatter_kick(rng, x, y, c, phi, th, kind, np.where(mat, x0, 0.0))
        el = go & (xi > 0)
        if el.any():
            pos_phi = np.arctan2(y, x)
            cosa = np.maximum(np.abs(np.where(kind == 0, np.sin(th) * np.cos(phi - pos_phi),
                                              np.cos(th))), 1e-6)
            p = 1.0 / (np.abs(c) * np.sin(th))
            E = np.sqrt(p * p + PION_MASS ** 2)
            dE = np.minimum(_bethe_si(p, PION_MASS) * xi / cosa * 1e-3, 0.5 * (E - PION_MASS))
            p1 = np.sqrt((E - dE) ** 2 - PION_MASS ** 2)
            c = np.where(el, c * p / p1, c)
        out_after[go, step] = np.stack([x, y, z, c, phi, th], axis=1)[go]
    return out_layer, out_state, out_after


def scatter_kick(rng, x, y, c, phi, th, kind, x0):
    """Gaussian multiple-scattering kick at a surface crossing: two independent
    projected angles of width theta0 (Highland), momentum unchanged.  Entries
    with x0 == 0 are returned unchanged."""
    n = c.shape[0]
    mat = x0 > 0
    pos_phi = np.arctan2(y, x)
    cosa = np.where(kind == 0, np.sin(th) * np.cos(phi - pos_phi), np.cos(th))
    t = np.where(mat, x0 / np.maximum(np.abs(cosa), 1e-6), 1.0)
    th0 = np.where(mat, _highland(c, th, t), 0.0)
    g1 = rng.standard_normal(n)
    g2 = rng.standard_normal(n)
    p = 1.0 / (np.abs(c) * np.sin(th))
    new_th = th + g1 * th0
    new_phi = _wrap(phi + g2 * th0 / np.sin(th))
    new_c = np.sign(c) / (p * np.sin(new_th))
    return (np.where(mat, new_c, c), np.where(mat, new_phi, phi), np.where(mat, new_th, th))


def _make_hits(rng, geom, layers, states, sig_fn):
    """Smear the true crossing points into hits (float64 here)."""
    m = layers >= 0
    ti, si = np.nonzero(m)
    lay = layers[ti, si]
    stt = states[ti, si]
    su, sv = sig_fn(rng, lay)
    du = rng.standard_normal(lay.shape[0]) * su
    dv = rng.standard_normal(lay.shape[0]) * sv
    kind = np.array([L["kind"] for L in geom])[lay]
    rt = np.hypot(stt[:, 0], stt[:, 1])
    pt = np.arctan2(stt[:, 1], stt[:, 0])
    ph = pt + du / rt
    barrel = kind == 0
    r_h = np.where(barrel, rt, rt + dv)
    z_h = np.where(barrel, stt[:, 2] + dv, stt[:, 2])
    return ti, si, lay, r_h * np.cos(ph), r_h * np.sin(ph), z_h, su, sv


def _noise(rng, geom, per_layer):
    xs, ys, zs, ls, sus, svs = [], [], [], [], [], []
    for i, L in enumerate(geom):
        k = int(per_layer)
        if k <= 0:
            continue
        ph = rng.uniform(-np.pi, np.pi, k)
        if L["kind"] == 0:
            r = np.full(k, L["r_or_z"])
            zz = rng.uniform(L["lo"], L["hi"], k)
        else:
            r = np.sqrt(rng.uniform(L["lo"] ** 2, L["hi"] ** 2, k))
            zz = np.full(k, L["r_or_z"])
        xs.append(r * np.cos(ph)); ys.append(r * np.sin(ph)); zs.append(zz)
        ls.append(np.full(k, i)); sus.append(np.full(k, L["sig_u"])); svs.append(np.full(k, L["sig_v"]))
    if not xs:
        e = np.zeros(0)
        return e, e, e, np.zeros(0, np.int64), e, e
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs),
            np.concatenate(ls), np.concatenate(sus), np.concatenate(svs))


def _layer_sigmas(geom):
    su = np.array([L["sig_u"] for L in geom])
    sv = np.array([L["sig_v"] for L in geom])
    return lambda rng, lay: (su[lay], sv[lay])


def make_event(rng, geom, n_tracks, pt_sampler, eta_max, n_noise_per_layer=0,
               bz=G.BZ_TESLA, sig_fn=None, vertex_sigma=0.01, material=None):
    """Generate one event: tracks from a Gaussian vertex, hits, noise, shuffle."""
    n = int(n_tracks)
    vx = rng.normal(0.0, vertex_sigma, n)
    vy = rng.normal(0.0, vertex_sigma, n)
    vz = rng.normal(0.0, vertex_sigma, n)
    pt = pt_sampler(rng, n)
    eta = rng.uniform(-eta_max, eta_max, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    theta = 2.0 * np.arctan(np.exp(-eta))
    c = q / pt
    st = dict(x=vx, y=vy, z=vz, c=c, phi=phi, theta=theta)
    truth0 = np.stack([vx, vy, vz, c, phi, theta], axis=1)
    layers, states, after = transport(rng, st, q, geom, bz, None, material=material)
    if sig_fn is None:
        sig_fn = _layer_sigmas(geom)
    ti, si, lay, hx, hy, hz, hsu, hsv = _make_hits(rng, geom, layers, states, sig_fn)
    nx_, ny_, nz_, nl_, nsu, nsv = _noise(rng, geom, n_noise_per_layer)
    n_sig = hx.shape[0]
    allx = np.concatenate([hx, nx_]); ally = np.concatenate([hy, ny_])
    allz = np.concatenate([hz, nz_]); alll = np.concatenate([lay, nl_])
    allsu = np.concatenate([hsu, nsu]); allsv = np.concatenate([hsv, nsv])
    sim = np.concatenate([ti, np.full(nx_.shape[0], -1)])
    perm = rng.permutation(allx.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    max_steps = layers.shape[1]
    seq_hit = np.full((n, max_steps), -1, np.int32)
    seq_hit[ti, si] = inv[np.arange(n_sig)]
    # compact each track's crossing sequence to the front (it already is)
    return Event(
        x=allx[perm].astype(np.float32), y=ally[perm].astype(np.float32),
        z=allz[perm].astype(np.float32), su=allsu[perm].astype(np.float32),
        sv=allsv[perm].astype(np.float32), layer=alll[perm].astype(np.int32),
        sim=sim[perm].astype(np.int32), truth0=truth0, seq_hit=seq_hit,
        seq_layer=layers.astype(np.int32), truth_at=states, truth_out=after)


# ---------------------------------------------------------------------------
# transverse-momentum spectra
def pt_uniform(lo, hi):
    return lambda rng, n: rng.uniform(lo, hi, n)


def pt_power2(lo, hi):
    """pdf ~ pT^-2 on [lo, hi] via the inverse CDF."""
    return lambda rng, n: 1.0 / (1.0 / lo - rng.random(n) * (1.0 / lo - 1.0 / hi))


def pt_two_values(a, b):
    return lambda rng, n: np.where(rng.random(n) < 0.5, a, b)


def sig_loguniform(lo, hi, ratio_v):
    def f(rng, lay):
        su = np.exp(rng.uniform(math.log(lo), math.log(hi), lay.shape[0]))
        return su, ratio_v * su
    return f


# ---------------------------------------------------------------------------
# the five workloads
def fit_sample(n_tracks=1000, seed=0, geom=None):
    """1,000 helix tracks, pT uniform 0.5-10 GeV, |eta|<1, ten barrel layers,
    sigma_rphi = 0.01 cm, sigma_z = 0.05 cm, no material (fit workload)."""
    rng = np.random.default_rng(seed)
    geom = geom or G.barrel10(x0=0.0)
    return geom, make_event(rng, geom, n_tracks, pt_uniform(0.5, 10.0), 1.0)


def precision_sample(n_tracks=200_000, seed=3):
    """pT 0.3 GeV loopers mixed with 100 GeV stiff tracks, hit sigma_u
    log-uniform in [0.002, 0.01] cm with sigma_v = 5 sigma_u, no material."""
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=0.0)
    return geom, make_event(rng, geom, n_tracks, pt_two_values(0.3, 100.0), 1.0,
                            sig_fn=sig_loguniform(0.002, 0.01, 5.0))


def find_events(n_events=20, n_tracks=800, n_noise=50_000, seed=1, x0=0.02):
    """Combinatorial-finding workload: 800 tracks (pT^-2 on 0.5-50 GeV, |eta|<1)
    and 50,000 uniform noise hits per event, ten barrel layers, 0.02 X0 per layer."""
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=x0)
    per_layer = n_noise // len(geom)
    evs = [make_event(rng, geom, n_tracks, pt_power2(0.5, 50.0), 1.0, per_layer)
           for _ in range(n_events)]
    return geom, evs


def batch_events(n_events=64, seed=2, noise_per_track=60, lam_lo=200.0, lam_hi=4000.0):
    """Uneven-multiplicity batch: N ~ Poisson(lambda), lambda ~ U(200, 4000),
    60 noise hits per track, barrel plus 2 x 7 disks, |eta| < 2.5, 0.02 X0."""
    rng = np.random.default_rng(seed)
    geom = G.barrel10_disks14(x0=0.02)
    evs = []
    for _ in range(n_events):
        lam = rng.uniform(lam_lo, lam_hi)
        n = max(1, int(rng.poisson(lam)))
        per_layer = noise_per_track * n // len(geom)
        evs.append(make_event(rng, geom, n, pt_power2(0.5, 50.0), 2.5, per_layer))
    return geom, evs


def propagation_pairs(n_pairs=1_000_000, seed=4, n_tracks=200_000):
    """Starting states and target layers for learning the propagation path
    length at the precision workload's distribution (pT 0.3 / 100 GeV, ten
    barrel layers, no material): every state a track passes through (its
    vertex and each crossing but the last) paired with the next layer it
    crosses, shuffled, the first n_pairs.  Returns (geom, state [n, 6] float64
    = (x, y, z, c, phi, theta), target layer [n] int32)."""
    geom, ev = precision_sample(n_tracks, seed=seed)
    nh = ev.n_track_hits()
    states = [ev.truth0]
    targets = [ev.seq_layer[:, 0]]
    for k in range(1, ev.seq_layer.shape[1]):
        m = nh > k
        states.append(ev.truth_out[m, k - 1])
        targets.append(ev.seq_layer[m, k])
    st = np.concatenate(states)
    tg = np.concatenate(targets).astype(np.int32)
    rng = np.random.default_rng(seed + 1000)
    sel = rng.permutation(st.shape[0])[:n_pairs]
    return geom, st[sel], tg[sel]


def batch_propagation_pairs(n_pairs=1_000_000, seed=5, n_events=64):
    """Starting states and target layers for learning the propagation path
    length at the batching workload's distribution (batch_events: ten barrels
    and 2 x 7 disks, |eta| < 2.5, pT^-2 on 0.5-50 GeV, 0.02 X0): every state
    a track passes through (its vertex and its state after each crossing,
    barrel or disk) paired with the next barrel outward (the smallest radius
    above rho + 0.05 cm), the surface whose radius solve the learned start
    begins during finding, whatever surface the track meets first; states with
    no barrel left are dropped.  Shuffled, the first n_pairs.  Returns (geom,
    state [n, 6] float64, target layer [n] int32)."""
    geom, evs = batch_events(n_events=n_events, seed=seed, noise_per_track=0)
    barrels = np.array([i for i, L in enumerate(geom) if L["kind"] == 0])
    radii = np.array([geom[i]["r_or_z"] for i in barrels])
    order = np.argsort(radii, kind="stable")
    barrels, radii = barrels[order], radii[order]
    states = []
    for ev in evs:
        nh = ev.n_track_hits()
        states.append(ev.truth0)
        for k in range(ev.truth_out.shape[1]):
            m = nh > k
            states.append(ev.truth_out[m, k])
    st = np.concatenate(states)
    rho = np.hypot(st[:, 0], st[:, 1])
    j = np.searchsorted(radii, rho + 0.05, side="right")
    keep = j < radii.size
    st = st[keep]
    tg = barrels[j[keep]].astype(np.int32)
    rng = np.random.default_rng(seed + 1000)
    sel = rng.permutation(st.shape[0])[:n_pairs]
    return geom, st[sel], tg[sel]


def mlp_init(seed=4, n_in=8, n_hidden=64):
    """Initial network parameters, flat float32 in the order W1[64][8], b1,
    W2[64][64], b2, w3[64], b3: weights uniform in +-sqrt(6 / (fan_in +
    fan_out)) (Glorot & Bengio 2010), biases zero."""
    rng = np.random.default_rng(seed)
    u = lambda fi, fo, shape: rng.uniform(-math.sqrt(6.0 / (fi + fo)), math.sqrt(6.0 / (fi + fo)), shape)
    parts = [u(n_in, n_hidden, (n_hidden, n_in)), np.zeros(n_hidden),
             u(n_hidden, n_hidden, (n_hidden, n_hidden)), np.zeros(n_hidden),
             u(n_hidden, 1, n_hidden), np.zeros(1)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
