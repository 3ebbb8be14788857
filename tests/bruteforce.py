"""Independent brute-force references used to pin the oracle (numpy, float64).

Nothing here calls the oracle's arithmetic: the helix crossing is the
closed-form circle-circle intersection, derivatives are numerical, and the
fit is a Gauss-Newton weighted least-squares solve of all hits at once.
"""
import numpy as np

KAPPA = 0.00299792458


def wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def circle(p, bz):
    """Centre and signed curvature of the transverse track circle."""
    x, y, z, c, phi, th = p
    h = -KAPPA * bz * c
    return np.array([x - np.sin(phi) / h, y + np.cos(phi) / h]), h


def cf_barrel(p, r_l, bz, nearest=False):
    """Closed-form outward crossing of radius r_l.

    nearest=False: smallest positive arc length; nearest=True: smallest |s|
    (signed arc in (-pi/|h|, pi/|h|]).  Returns (state at crossing, s) or None.
    """
    x, y, z, c, phi, th = p
    C, h = circle(p, bz)
    R = 1.0 / abs(h)
    d = np.hypot(*C)
    a = (r_l * r_l - R * R + d * d) / (2 * d)
    disc = r_l * r_l - a * a
    if disc < 0:
        return None
    hh = np.sqrt(disc)
    u = C / d
    best = None
    for sg in (1.0, -1.0):
        P = a * u + sg * hh * np.array([-u[1], u[0]])
        v0 = np.array([x, y]) - C
        v1 = P - C
        ang = np.arctan2(v0[0] * v1[1] - v0[1] * v1[0], v0 @ v1)   # CCW angle v0 -> v1
        if nearest:
            s = ang / h                       # signed, |s| <= pi R
        else:
            s = np.mod(np.sign(h) * ang, 2 * np.pi) / abs(h)
        ph = phi + h * s
        if P[0] * np.cos(ph) + P[1] * np.sin(ph) <= 0:
            continue
        if best is None or (abs(s) < abs(best[1]) if nearest else s < best[1]):
            best = (np.array([P[0], P[1], z + s / np.tan(th), c, wrap(ph), th]), s)
    return best


def cf_disk(p, z_d, bz):
    x, y, z, c, phi, th = p
    s = (z_d - z) * np.tan(th)
    C, h = circle(p, bz)
    v0 = np.array([x, y]) - C
    a = h * s
    rot = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
    P = C + rot @ v0
    return np.array([P[0], P[1], z_d, c, wrap(phi + a), th]), s


def measure(q, hit, kind):
    """Local-frame residual of a hit (x, y, z, su, sv) w.r.t. state q."""
    rho = np.hypot(hit[0], hit[1])
    cp, sp = hit[0] / rho, hit[1] / rho
    ru = -sp * (hit[0] - q[0]) + cp * (hit[1] - q[1])
    if kind == 0:
        rv = hit[2] - q[2]
    else:
        rv = cp * (hit[0] - q[0]) + sp * (hit[1] - q[1])
    return np.array([ru, rv])


def wls_fit(p_seed, P0, hits, layers, geom, bz, iters=50, tol=1e-12):
    """Gauss-Newton minimisation of sum_i r_i^T V_i^-1 r_i + (p-p_seed)^T P0^-1 (p-p_seed)
    over the state at the seed point, each r_i from the exact crossing of layer i.
    Returns (p*, covariance of p*, chi2 of hits)."""
    P0i = np.linalg.inv(P0)

    def resid(p):
        out = []
        for hit, l in zip(hits, layers):
            L = geom[l]
            if L["kind"] == 0:
                q = cf_barrel(p, L["r_or_z"], bz, nearest=True)[0]
            else:
                q = cf_disk(p, L["r_or_z"], bz)[0]
            out.append(measure(q, hit, L["kind"]) / np.array([hit[3], hit[4]]))
        return np.concatenate(out)

    p = np.array(p_seed, float)
    steps = np.array([1e-6, 1e-6, 1e-6, 1e-8, 1e-8, 1e-8])
    for _ in range(iters):
        r = resid(p)
        J = np.zeros((r.size, 6))
        for j in range(6):
            e = np.zeros(6)
            e[j] = steps[j]
            J[:, j] = (resid(p + e) - resid(p - e)) / (2 * steps[j])
        # r(p + dp) ~ r - ... : residual = meas - pred, so d r/dp = -J_pred; J here is d r / dp
        A = J.T @ J + P0i
        g = J.T @ r + P0i @ (p - p_seed)
        dp = -np.linalg.solve(A, g)
        p = p + dp
        if np.linalg.norm(dp / np.array([1, 1, 1, 0.01, 0.01, 0.01])) < tol:
            break
    r = resid(p)
    J = np.zeros((r.size, 6))
    for j in range(6):
        e = np.zeros(6)
        e[j] = steps[j]
        J[:, j] = (resid(p + e) - resid(p - e)) / (2 * steps[j])
    cov = np.linalg.inv(J.T @ J + P0i)
    return p, cov, float(r @ r)


def propagate_cf(p, layer, geom, bz, nearest=False):
    L = geom[layer]
    if L["kind"] == 0:
        res = cf_barrel(p, L["r_or_z"], bz, nearest=nearest)
        return None if res is None else res[0]
    return cf_disk(p, L["r_or_z"], bz)[0]


def num_jacobian(fun, p, steps):
    p = np.asarray(p, float)
    out = []
    for j in range(6):
        e = np.zeros(6)
        e[j] = steps[j]
        a, b = fun(p + e), fun(p - e)
        d = (a - b)
        d[4] = wrap(d[4])
        out.append(d / (2 * steps[j]))
    return np.array(out).T
