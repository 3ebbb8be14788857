"""FP64 reference of the learned path-length guess: features, the 8-64-64-1
tanh network, its mean-squared-error gradient and the Adam update.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by the tests
and the CPU baseline, never by the product path, and sharing no code with
the HIP kernels.

The network is not part of the paper; it is the learned initial guess for
the iterative propagate-to-radius solve (the paper's Sec. 3.1 propagation to
the next layer).  Reading taken for the unstated details:
  * inputs (8): rho/100, sin psi, cos psi with psi = phi - atan2(y, x), the
    signed curvature h (in the field at the start point) times the target
    radius (barrel) or times 100 cm (disk), the target radius or disk z over
    100, the straight-line path length to the target over 100 (tangent-line
    intersection for a barrel, the exact (z_D - z) tan theta for a disk),
    cot theta, and z/100 (the parametrised field depends on z);
  * output: the transverse arc length to the target minus the straight-line
    one, in units of h s_line^2 (the leading order of that difference; the
    guess is s_line + h s_line^2 * output);
  * 8 -> 64 (tanh) -> 64 (tanh) -> 1 (linear), mean squared error, Adam.
Flat parameter order (4801 values): W1[64][8], b1[64], W2[64][64], b2[64],
w3[64], b3.
"""
import numpy as np

N_IN, N_H = 8, 64
SIZES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", ()))
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)
KAPPA = 0.00299792458      # GeV / (T cm)


def unpack(theta):
    """Flat parameter vector -> dict of views."""
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape) if shape else theta[o]
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1) for name, _ in SIZES])


def forward(theta, X):
    """X [n, 8] -> (y [n], cache).  Hidden layers tanh, output linear."""
    p = unpack(theta)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(a2)
    y = h2 @ p["w3"] + p["b3"]
    return y, (X, h1, h2)


def loss(theta, X, t):
    y, _ = forward(theta, X)
    return float(np.mean((y - t) ** 2))


def grad(theta, X, t):
    """Mean squared error over the batch and its gradient (flat, FP64) by
    the chain rule, layer by layer from the output back."""
    p = unpack(theta)
    y, (X, h1, h2) = forward(theta, X)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n                      # dL/dy
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = dy.sum()
    da2 = np.outer(dy, p["w3"]) * (1.0 - h2 ** 2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), pack(g)


def adam(theta, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step number
    `step` (1-based); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, t, perm, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Minibatch Adam over the rows perm[k*batch:(k+1)*batch] for every k
    (the shuffling is an input).  Returns (theta, losses per step)."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for k in range(len(perm) // batch):
        rows = perm[k * batch:(k + 1) * batch]
        L, g = grad(theta, X[rows], t[rows])
        losses.append(L)
        theta, m, v = adam(theta, m, v, g, k + 1, lr, beta1, beta2, eps)
    return theta, np.array(losses)


def features(state, kind, target, bz=3.8, field_z0=0.0):
    """Network inputs for propagating `state` [n, 6] = (x, y, z, c, phi,
    theta) to a barrel of radius `target` (kind 0) or a disk at z = `target`
    (kind 1); field_z0 > 0: the parametrised field Bz = bz / (1 + (z/z0)^2).
    Returns [n, 8] (FP64)."""
    s = np.atleast_2d(np.asarray(state, np.float64))
    kind = np.broadcast_to(np.asarray(kind), (s.shape[0],))
    target = np.broadcast_to(np.asarray(target, np.float64), (s.shape[0],))
    x, y, z, c, phi, th = s.T
    rho = np.hypot(x, y)
    alpha = np.arctan2(y, x)
    psi = phi - alpha
    sin_psi = np.where(rho > 0, np.sin(psi), 0.0)
    cos_psi = np.where(rho > 0, np.cos(psi), 1.0)
    bz_here = bz / (1.0 + (z / field_z0) ** 2) if field_z0 > 0 else bz
    h = -KAPPA * bz_here * c
    disk = kind == 1
    # tangent line from (x, y) along phi to the circle of radius target
    pu = x * np.cos(phi) + y * np.sin(phi)
    disc = pu * pu - rho * rho + target * target
    s_line_barrel = np.where(disc > 0, -pu + np.sqrt(np.maximum(disc, 0.0)), -pu)
    s_disk = (target - z) * np.tan(th)
    f = np.empty((s.shape[0], N_IN))
    f[:, 0] = rho / 100.0
    f[:, 1] = sin_psi
    f[:, 2] = cos_psi
    f[:, 3] = h * np.where(disk, 100.0, target)
    f[:, 4] = target / 100.0
    f[:, 5] = np.where(disk, s_disk, s_line_barrel) / 100.0
    f[:, 6] = np.cos(th) / np.sin(th)
    f[:, 7] = z / 100.0
    return f


def target(f, path):
    """Training target of one propagation with inputs f [n, 8] (features())
    and transverse path length `path` [n] [cm]: the output y for which the
    guess s_line + h s_line^2 y equals the path, written in the inputs'
    units (s_line = 100 f5, h s_line^2 = 100 f3 f5^2 / f4); 0 where that
    scale is at most 1e-9 (no curvature term)."""
    f = np.atleast_2d(np.asarray(f, np.float64))
    path = np.asarray(path, np.float64)
    k = np.where(f[:, 4] != 0, f[:, 3] * f[:, 5] ** 2 / np.where(f[:, 4] != 0, f[:, 4], 1.0), 0.0)
    big = np.abs(k) > 1e-9
    return np.where(big, (path / 100.0 - f[:, 5]) / np.where(big, k, 1.0), 0.0)


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even), returned
    as float64: the precision the network's weights and inputs take on the
    device."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isfinite(f), out, f).astype(np.float64)
