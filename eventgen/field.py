"""Tracks in the parametrised solenoid-like field (synthetic): the field
model's parameters and a fine-step tracer that produces the true crossings of
barrel layers.  Input generation only: the tracer integrates with its own
small fixed step (default 0.05 cm), far below the reconstruction's.

Field: Bz = B0 / (1 + (z/Z0)^2), Br = -(r/2) dBz/dz, no azimuthal component
(divergence free, axially symmetric)."""
import numpy as np

from . import geometry as G
from .generate import Event, KAPPA, pt_uniform

Z0_DEFAULT = 300.0       # cm


def field(x, y, z, b0=G.BZ_TESLA, z0=Z0_DEFAULT):
    u = z / z0
    g = 1.0 / (1.0 + u * u)
    dbz = -2.0 * b0 * z / (z0 * z0) * g * g
    return -0.5 * dbz * x, -0.5 * dbz * y, b0 * g


def _deriv(Y, kq, b0, z0):
    bx, by, bz = field(Y[0], Y[1], Y[2], b0, z0)
    tx, ty, tz = Y[3], Y[4], Y[5]
    return np.stack([tx, ty, tz, kq * (ty * bz - tz * by), kq * (tz * bx - tx * bz),
                     kq * (tx * by - ty * bx)])


def _rk4(Y, h, kq, b0, z0):
    k1 = _deriv(Y, kq, b0, z0)
    k2 = _deriv(Y + 0.5 * h * k1, kq, b0, z0)
    k3 = _deriv(Y + 0.5 * h * k2, kq, b0, z0)
    k4 = _deriv(Y + h * k3, kq, b0, z0)
    return Y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


def to_state(Y, kq):
    """(position, direction) columns -> (x, y, z, c, phi, theta) rows."""
    tt = np.hypot(Y[3], Y[4])
    th = np.arctan2(tt, Y[5])
    return np.stack([Y[0], Y[1], Y[2], kq / KAPPA / np.sin(th), np.arctan2(Y[4], Y[3]), th],
                    axis=1)


def from_state(s):
    st = np.sin(s[:, 5])
    Y = np.stack([s[:, 0], s[:, 1], s[:, 2], st * np.cos(s[:, 4]), st * np.sin(s[:, 4]),
                  np.cos(s[:, 5])])
    return Y, KAPPA * s[:, 3] * st


def trace_to_radii(states, radii, zmax, b0=G.BZ_TESLA, z0=Z0_DEFAULT, step=0.05,
                   max_len=400.0):
    """Outward crossings of the cylinders `radii` (ascending) by tracks
    starting at `states` [n, 6].  Returns (crossing states [n, nl, 6] and a
    mask [n, nl]: crossed inside |z| <= zmax[l], before turning back)."""
    n, nl = states.shape[0], len(radii)
    Y, kq = from_state(states)
    out = np.zeros((n, nl, 6))
    hit = np.zeros((n, nl), bool)
    nxt = np.zeros(n, int)                  # next layer to cross
    alive = np.ones(n, bool)
    steps = int(max_len / step)
    for _ in range(steps):
        if not alive.any():
            break
        Yn = _rk4(Y, step, kq, b0, z0)
        r0, r1 = np.hypot(Y[0], Y[1]), np.hypot(Yn[0], Yn[1])
        # a track turning back inwards (away from the vertex region) or past
        # the last layer is done
        alive &= ~((r1 < r0 - 1e-9) & (r0 > 1.0))
        for _inner in range(3):                # at most a few layers per step
            idx = np.nonzero(alive & (nxt < nl))[0]
            if idx.size == 0:
                break
            rl = np.asarray(radii)[nxt[idx]]
            cross = (r0[idx] < rl) & (r1[idx] >= rl)
            if not cross.any():
                break
            ci = idx[cross]
            rc = rl[cross]
            # bisection on the step fraction, each trial a single RK4 sub-step
            lo, hi = np.zeros(ci.size), np.full(ci.size, step)
            for _b in range(40):
                mid = 0.5 * (lo + hi)
                Ym = _rk4(Y[:, ci], mid, kq[ci], b0, z0)
                inside = np.hypot(Ym[0], Ym[1]) < rc
                lo = np.where(inside, mid, lo)
                hi = np.where(inside, hi, mid)
            Yc = _rk4(Y[:, ci], 0.5 * (lo + hi), kq[ci], b0, z0)
            lay = nxt[ci]
            ok = np.abs(Yc[2]) <= np.asarray(zmax)[lay]
            out[ci, lay] = to_state(Yc, kq[ci])
            hit[ci, lay] = ok
            alive[ci[~ok]] = False
            nxt[ci] += 1
        alive &= nxt < nl
        Y = Yn
    return out, hit


def _vertex_states(rng, n):
    """pT U(0.5, 10) GeV, |eta| < 1, both charges, vertex sigma 0.01 cm."""
    pt = pt_uniform(0.5, 10.0)(rng, n)
    eta = rng.uniform(-1.0, 1.0, n)
    th = 2.0 * np.arctan(np.exp(-eta))
    phi = rng.uniform(-np.pi, np.pi, n)
    q = rng.choice([-1.0, 1.0], n)
    v = rng.normal(0.0, 0.01, (n, 3))
    return np.stack([v[:, 0], v[:, 1], v[:, 2], q / pt, phi, th], axis=1)


def field_sample(n_tracks=2000, seed=5, z0=Z0_DEFAULT, su=0.01, sv=0.05, step=0.05):
    """Fit workload in the parametrised field: pT U(0.5, 10) GeV, |eta| < 1,
    vertex sigma 0.01 cm, ten barrel layers, no material, hits smeared by
    (su, sv) on the surface.  Returns (geom, Event)."""
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=0.0, su=su, sv=sv)
    radii = [L["r_or_z"] for L in geom]
    zmax = [L["hi"] for L in geom]
    n = n_tracks
    st0 = _vertex_states(rng, n)
    cr, ok = trace_to_radii(st0, radii, zmax, z0=z0, step=step)
    # consecutive crossings from the first layer only
    nh = np.argmin(np.concatenate([ok, np.zeros((n, 1), bool)], axis=1), axis=1)
    xs, ys, zs, sus, svs, lay, sim = [], [], [], [], [], [], []
    seq_hit = np.full((n, len(geom)), -1, np.int32)
    seq_layer = np.full((n, len(geom)), -1, np.int32)
    truth_at = np.zeros((n, len(geom), 6))
    k = 0
    for t in range(n):
        for l in range(nh[t]):
            s = cr[t, l]
            r = np.hypot(s[0], s[1])
            ph = np.arctan2(s[1], s[0]) + rng.normal(0.0, su) / r
            xs.append(r * np.cos(ph))
            ys.append(r * np.sin(ph))
            zs.append(s[2] + rng.normal(0.0, sv))
            sus.append(su)
            svs.append(sv)
            lay.append(l)
            sim.append(t)
            seq_hit[t, l] = k
            seq_layer[t, l] = l
            truth_at[t, l] = s
            k += 1
    f32 = lambda a: np.asarray(a, np.float32)
    ev = Event(x=f32(xs), y=f32(ys), z=f32(zs), su=f32(sus), sv=f32(svs),
               layer=np.asarray(lay, np.int32), sim=np.asarray(sim, np.int32), truth0=st0,
               seq_hit=seq_hit, seq_layer=seq_layer, truth_at=truth_at, truth_out=truth_at.copy())
    return geom, ev


def field_pairs(n_tracks=100_000, seed=6, z0=Z0_DEFAULT, step=0.5):
    """Starting states and target layers for learning the propagation path
    length in the parametrised field: tracks of the field workload's
    distribution traced (RK4, `step` cm) through the ten barrel layers; every
    state a track passes through (its vertex and each crossing but the last)
    paired with the next layer, shuffled.  Returns (geom, state [n, 6]
    float64, target layer [n] int32)."""
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=0.0)
    radii = [L["r_or_z"] for L in geom]
    zmax = [L["hi"] for L in geom]
    st0 = _vertex_states(rng, n_tracks)
    cr, ok = trace_to_radii(st0, radii, zmax, z0=z0, step=step)
    nh = np.argmin(np.concatenate([ok, np.zeros((n_tracks, 1), bool)], axis=1), axis=1)
    states = [st0[nh > 0]]
    targets = [np.zeros(int((nh > 0).sum()), np.int32)]
    for k in range(1, len(geom)):
        m = nh > k
        states.append(cr[m, k - 1])
        targets.append(np.full(int(m.sum()), k, np.int32))
    st = np.concatenate(states)
    tg = np.concatenate(targets)
    sel = rng.permutation(st.shape[0])
    return geom, st[sel], tg[sel]


def field_find_events(n_events=3, n_tracks=600, n_noise=30_000, seed=25, z0=Z0_DEFAULT, step=0.2,
                      su=0.01, sv=0.05):
    """Finding workload in the parametrised field: per event n_tracks (an int,
    or one count per event) of the field workload's distribution traced (RK4,
    `step` cm, every event's tracks in one vectorised pass) through the ten
    barrels (no material), hits smeared by (su, sv), plus n_noise (an int, or
    one count per event) uniform noise hits spread over the layers; hits
    shuffled.  Returns (geom, events)."""
    from .generate import Event, _noise
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=0.0, su=su, sv=sv)
    nl = len(geom)
    radii = [L["r_or_z"] for L in geom]
    zmax = [L["hi"] for L in geom]
    nt = np.broadcast_to(np.asarray(n_tracks, np.int64), (n_events,))
    nn = np.broadcast_to(np.asarray(n_noise, np.int64), (n_events,))
    st_all = _vertex_states(rng, int(nt.sum()))
    cr_all, ok_all = trace_to_radii(st_all, radii, zmax, z0=z0, step=step)
    bounds = np.concatenate([[0], np.cumsum(nt)])
    evs = []
    for e in range(n_events):
        n = int(nt[e])
        st0 = st_all[bounds[e]:bounds[e + 1]]
        cr, ok = cr_all[bounds[e]:bounds[e + 1]], ok_all[bounds[e]:bounds[e + 1]]
        nh = np.argmin(np.concatenate([ok, np.zeros((n, 1), bool)], axis=1), axis=1)
        ti, si = np.nonzero(np.arange(nl)[None, :] < nh[:, None])
        s = cr[ti, si]
        r = np.hypot(s[:, 0], s[:, 1])
        ph = np.arctan2(s[:, 1], s[:, 0]) + rng.normal(0.0, su, ti.size) / r
        hx, hy = r * np.cos(ph), r * np.sin(ph)
        hz = s[:, 2] + rng.normal(0.0, sv, ti.size)
        nx, ny, nz, nlay, nsu, nsv = _noise(rng, geom, int(nn[e]) // nl)
        allx = np.concatenate([hx, nx])
        ally = np.concatenate([hy, ny])
        allz = np.concatenate([hz, nz])
        alll = np.concatenate([si, nlay])
        allsu = np.concatenate([np.full(ti.size, su), nsu])
        allsv = np.concatenate([np.full(ti.size, sv), nsv])
        sim = np.concatenate([ti, np.full(nx.shape[0], -1)])
        perm = rng.permutation(allx.shape[0])
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.shape[0])
        seq_hit = np.full((n, nl), -1, np.int32)
        seq_hit[ti, si] = inv[np.arange(ti.size)]
        seq_layer = np.where(seq_hit >= 0, np.arange(nl)[None, :], -1).astype(np.int32)
        truth_at = np.zeros((n, nl, 6))
        truth_at[ti, si] = s
        f32 = lambda a: np.asarray(a, np.float32)
        evs.append(Event(x=f32(allx[perm]), y=f32(ally[perm]), z=f32(allz[perm]),
                         su=f32(allsu[perm]), sv=f32(allsv[perm]),
                         layer=alll[perm].astype(np.int32), sim=sim[perm].astype(np.int32),
                         truth0=st0, seq_hit=seq_hit, seq_layer=seq_layer, truth_at=truth_at,
                         truth_out=truth_at.copy()))
    return geom, evs


def field_find_batch(n_events=16, seed=27):
    """The finding batch in the parametrised field: n_events events with
    N ~ Poisson(U(200, 4000)) tracks of the field workload's distribution and
    60 noise hits per track (the batched workload's multiplicity and noise
    recipe, on the ten barrels), traced in 0.5 cm steps.  Returns (geom,
    events)."""
    rng = np.random.default_rng(seed)
    nt = np.maximum(rng.poisson(rng.uniform(200, 4000, n_events)), 1)
    return field_find_events(n_events=n_events, n_tracks=nt, n_noise=60 * nt, seed=seed + 1, step=0.5)


DISK_AHEAD_EPS = 0.05    # cm: a disk counts as "ahead" if |dz| > eps in the direction of travel


def trace_surfaces(states, geom, b0=G.BZ_TESLA, z0=Z0_DEFAULT, step=0.1, max_steps=None,
                   max_len=600.0):
    """Walk tracks through barrels and disks in the parametrised field with a
    fine fixed-step RK4 (the generator's own integrator), surface by surface:
    from each surface the next one is the first crossed along the path among
    the next barrel outward (radius above rho + 0.05 cm, crossed inside its
    z extent) and any disk ahead (|dz| > 0.05 cm in the direction of travel,
    crossed inside its radial extent); a step ends the track once its
    transverse path exceeds half a turn of the curvature at the step's start.
    Crossings are found by secant iterations on a single RK4 sub-step's length.  Returns
    (layers [n, max_steps] int, -1 padded; crossing states [n, max_steps, 6])."""
    n, nl = states.shape[0], len(geom)
    max_steps = max_steps or nl
    kind = np.array([L["kind"] for L in geom])
    rz = np.array([L["r_or_z"] for L in geom], float)
    lo = np.array([L["lo"] for L in geom], float)
    hi = np.array([L["hi"] for L in geom], float)
    barrels = np.nonzero(kind == 0)[0]
    barrels = barrels[np.argsort(rz[barrels], kind="stable")]
    disks = np.nonzero(kind == 1)[0]
    dz_order = disks[np.argsort(rz[disks], kind="stable")]
    dz_sorted = rz[dz_order]
    Y, kq = from_state(states)
    out_l = np.full((n, max_steps), -1, np.int32)
    out_s = np.zeros((n, max_steps, 6))
    alive = np.ones(n, bool)
    k_out = np.zeros(n, int)
    total = np.zeros(n)

    def new_step(idx):
        """Surfaces and budgets of a navigation step starting at Y[:, idx]."""
        rho = np.hypot(Y[0, idx], Y[1, idx])
        j = np.searchsorted(rz[barrels], rho + 0.05, side="right")
        nb = np.where(j < barrels.size, barrels[np.minimum(j, barrels.size - 1)], -1)
        _, _, bz = field(Y[0, idx], Y[1, idx], Y[2, idx], b0, z0)
        c = kq[idx] / (KAPPA * np.sqrt(np.maximum(Y[3, idx] ** 2 + Y[4, idx] ** 2, 1e-300)))
        hh = np.abs(KAPPA * bz * c)
        smax = np.where(hh > 0, np.pi / np.maximum(hh, 1e-300), np.inf)
        return nb, smax

    nb = np.full(n, -1)
    smax = np.zeros(n)
    bvoid = np.zeros(n, bool)
    sturn = np.zeros(n)
    z_start = Y[2].copy()
    idx = np.arange(n)
    nb[idx], smax[idx] = new_step(idx)
    while alive.any():
        a = np.nonzero(alive)[0]
        Yn = _rk4(Y[:, a], step, kq[a], b0, z0)
        best_f = np.full(a.size, np.inf)
        best_l = np.full(a.size, -1)
        best_Y = np.zeros((6, a.size))
        # the next barrel outward
        hasb = (nb[a] >= 0) & ~bvoid[a]
        rb = np.where(hasb, rz[np.maximum(nb[a], 0)], np.inf)
        r0, r1 = np.hypot(Y[0, a], Y[1, a]), np.hypot(Yn[0], Yn[1])
        # a disk plane passed in this step (planes are far apart: at most one)
        zlo, zhi = np.minimum(Y[2, a], Yn[2]), np.maximum(Y[2, a], Yn[2])
        j = np.searchsorted(dz_sorted, zlo, side="left")
        jd = np.minimum(j, max(dz_sorted.size - 1, 0))
        dsel = dz_order[jd] if dz_sorted.size else np.zeros(a.size, int)
        crd = (j < dz_sorted.size) & (rz[dsel] <= zhi) & (Y[2, a] != rz[dsel]) \
            & ((rz[dsel] - z_start[a]) * np.sign(Y[5, a]) > DISK_AHEAD_EPS) if dz_sorted.size \
            else np.zeros(a.size, bool)
        for m, what in ((hasb & (r0 < rb) & (r1 >= rb), "b"), (crd, "d")):
            if not m.any():
                continue
            ci = np.nonzero(m)[0]
            g = a[ci]
            target = rb[ci] if what == "b" else rz[dsel[ci]]

            def gap(Ym):
                return np.hypot(Ym[0], Ym[1]) - target if what == "b" else Ym[2] - target
            # secant iterations on the single RK4 sub-step's length, from the
            # step's two ends (the surface lies between them)
            fa, fb = np.zeros(ci.size), np.full(ci.size, step)
            ga, gb = gap(Y[:, g]), gap(Yn[:, ci])
            f = fb
            for _it in range(8):
                den = np.where(gb != ga, gb - ga, 1.0)
                f = np.clip(fb - gb * (fb - fa) / den, 0.0, step)
                gf = gap(_rk4(Y[:, g], f, kq[g], b0, z0))
                fa, ga, fb, gb = fb, gb, f, gf
            Yc = _rk4(Y[:, g], f, kq[g], b0, z0)
            if what == "b":
                lay = nb[g]
                ok = np.abs(Yc[2]) <= hi[lay]
                # a barrel crossed outside its extent is void for this step
                bvoid[g[~ok]] = True
            else:
                lay = dsel[ci]
                rr = np.hypot(Yc[0], Yc[1])
                ok = (rr >= lo[lay]) & (rr <= hi[lay])
            better = ok & (f < best_f[ci])
            sel = ci[better]
            best_f[sel] = f[better]
            best_l[sel] = lay[better]
            best_Y[:, sel] = Yc[:, better]
        # advance: to the crossing if any, else the whole step
        got = best_l >= 0
        adv = np.where(got, best_f, step)
        sturn[a] += adv * np.hypot(Y[3, a], Y[4, a])
        total[a] += adv
        # no surface left: no barrel candidate and every disk behind
        dir_z = np.sign(Y[5, a])
        disk_ahead = ((rz[disks][None, :] - Y[2, a][:, None]) * dir_z[:, None] > 0).any(axis=1) \
            if disks.size else np.zeros(a.size, bool)
        none_left = ~got & ~((nb[a] >= 0) & ~bvoid[a]) & ~disk_ahead
        over = (sturn[a] > smax[a]) | (total[a] > max_len) | none_left
        rec = got & ~over
        Y[:, a] = np.where(got, best_Y, Yn)
        if rec.any():
            g = a[rec]
            out_l[g, k_out[g]] = best_l[rec]
            out_s[g, k_out[g]] = to_state(Y[:, g], kq[g])
            k_out[g] += 1
            sturn[g] = 0.0
            bvoid[g] = False
            z_start[g] = Y[2, g]
            nb[g], smax[g] = new_step(g)
        alive[a[over]] = False
        alive &= k_out < max_steps
    return out_l, out_s


def _vertex_states_eta(rng, n, eta_max):
    """pT U(0.5, 10) GeV, |eta| < eta_max, both charges, vertex sigma 0.01 cm."""
    pt = pt_uniform(0.5, 10.0)(rng, n)
    eta = rng.uniform(-eta_max, eta_max, n)
    th = 2.0 * np.arctan(np.exp(-eta))
    phi = rng.uniform(-np.pi, np.pi, n)
    q = rng.choice([-1.0, 1.0], n)
    v = rng.normal(0.0, 0.01, (n, 3))
    return np.stack([v[:, 0], v[:, 1], v[:, 2], q / pt, phi, th], axis=1)


def field_disk_events(n_events=2, n_tracks=500, n_noise=20_000, seed=30, z0=Z0_DEFAULT,
                      step=0.1, eta_max=2.5):
    """Barrel and endcap events in the parametrised field: per event
    n_tracks of pT U(0.5, 10) GeV over |eta| < eta_max traced by
    trace_surfaces through ten barrels and 2 x 7 disks (no material), hits
    smeared on their surfaces (barrel: r phi and z; disk: r phi and r, the
    layers' sigmas), plus n_noise uniform noise hits spread over the 24
    layers; hits shuffled.  n_noise = 0 gives a fit sample.  Returns (geom,
    events)."""
    from .generate import _noise
    rng = np.random.default_rng(seed)
    geom = G.barrel10_disks14(x0=0.0)
    nl = len(geom)
    kind = np.array([L["kind"] for L in geom])
    su_l = np.array([L["sig_u"] for L in geom])
    sv_l = np.array([L["sig_v"] for L in geom])
    st_all = _vertex_states_eta(rng, n_events * n_tracks, eta_max)
    lay_all, cr_all = trace_surfaces(st_all, geom, z0=z0, step=step)
    evs = []
    for e in range(n_events):
        sl = slice(e * n_tracks, (e + 1) * n_tracks)
        st0, lay, cr = st_all[sl], lay_all[sl], cr_all[sl]
        ti, si = np.nonzero(lay >= 0)
        ll = lay[ti, si]
        s = cr[ti, si]
        rt = np.hypot(s[:, 0], s[:, 1])
        du = rng.normal(0.0, 1.0, ti.size) * su_l[ll]
        dv = rng.normal(0.0, 1.0, ti.size) * sv_l[ll]
        ph = np.arctan2(s[:, 1], s[:, 0]) + du / rt
        barrel = kind[ll] == 0
        rh = np.where(barrel, rt, rt + dv)
        hx, hy = rh * np.cos(ph), rh * np.sin(ph)
        hz = np.where(barrel, s[:, 2] + dv, s[:, 2])
        nx, ny, nz, nlay, nsu, nsv = _noise(rng, geom, int(n_noise) // nl)
        allx = np.concatenate([hx, nx])
        ally = np.concatenate([hy, ny])
        allz = np.concatenate([hz, nz])
        alll = np.concatenate([ll, nlay])
        allsu = np.concatenate([su_l[ll], nsu])
        allsv = np.concatenate([sv_l[ll], nsv])
        sim = np.concatenate([ti, np.full(nx.shape[0], -1)])
        perm = rng.permutation(allx.shape[0])
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.shape[0])
        seq_hit = np.full((n_tracks, nl), -1, np.int32)
        seq_hit[ti, si] = inv[np.arange(ti.size)]
        seq_layer = np.where(seq_hit >= 0, lay, -1).astype(np.int32)
        truth_at = np.zeros((n_tracks, nl, 6))
        truth_at[ti, si] = s
        f32 = lambda a: np.asarray(a, np.float32)
        evs.append(Event(x=f32(allx[perm]), y=f32(ally[perm]), z=f32(allz[perm]),
                         su=f32(allsu[perm]), sv=f32(allsv[perm]),
                         layer=alll[perm].astype(np.int32), sim=sim[perm].astype(np.int32),
                         truth0=st0, seq_hit=seq_hit, seq_layer=seq_layer, truth_at=truth_at,
                         truth_out=truth_at.copy()))
    return geom, evs
