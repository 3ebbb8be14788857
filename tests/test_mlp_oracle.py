"""Pins of the FP64 network oracle (oracle/mlp.py) against facts that do not
come from its own code: central finite differences of the loss, a network
built to compute a known linear map, Adam's closed form under a constant
gradient, torch's bfloat16 rounding, and the propagation oracle's exact path
lengths for the straight-line feature."""
import numpy as np
import pytest

from oracle import mlp as M


def _rand_theta(rng, scale=0.5):
    return rng.normal(0.0, scale, M.N_PARAM)


def test_parameter_count_and_layout():
    assert M.N_PARAM == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4801
    th = np.arange(M.N_PARAM, dtype=np.float64)
    p = M.unpack(th)
    assert p["W1"][0, 1] == 1 and p["W1"][1, 0] == 8          # row-major [out][in]
    assert p["b1"][0] == 512 and p["W2"][0, 0] == 576 and p["W2"][2, 3] == 576 + 2 * 64 + 3
    assert p["b2"][0] == 576 + 4096 and p["w3"][0] == 576 + 4096 + 64 and p["b3"] == 4800
    assert np.array_equal(M.pack(p), th)


def test_gradient_matches_central_differences():
    """Every one of the 4801 partial derivatives against a central finite
    difference of the forward pass alone (FP64, step 1e-6)."""
    rng = np.random.default_rng(70)
    th = _rand_theta(rng, 0.3)
    X = rng.normal(0, 1, (12, 8))
    t = rng.normal(0, 1, 12)
    L, g = M.grad(th, X, t)
    assert L == pytest.approx(M.loss(th, X, t), rel=1e-14)
    eps = 1e-6
    fd = np.empty_like(th)
    for k in range(M.N_PARAM):
        a = th.copy()
        a[k] += eps
        b = th.copy()
        b[k] -= eps
        fd[k] = (M.loss(a, X, t) - M.loss(b, X, t)) / (2 * eps)
    err = np.abs(fd - g) / np.maximum(np.abs(g), 1e-3 * np.abs(g).max())
    assert err.max() < 1e-6, err.max()
    assert np.linalg.norm(fd - g) / np.linalg.norm(g) < 1e-8


def test_wiring_by_a_known_linear_map():
    """Small weights make tanh(u) = u + O(u^3): a network whose first layer
    routes input perm1[j] to hidden j and whose second layer routes hidden
    perm2[k] to hidden k computes y = sum_j w3[j] eps^2 x[perm1[perm2[j]]]
    + b3.  A transposed weight matrix or swapped layer routes other inputs."""
    rng = np.random.default_rng(71)
    e = 1e-4
    perm1 = np.array([(3 * j + 1) % 8 for j in range(64)])      # hidden j reads input perm1[j]
    perm2 = rng.permutation(64)                                   # hidden2 k reads hidden1 perm2[k]
    W1 = np.zeros((64, 8))
    W1[np.arange(64), perm1] = e
    W2 = np.zeros((64, 64))
    W2[np.arange(64), perm2] = e
    w3 = rng.normal(0, 1, 64) / e ** 2
    th = M.pack(dict(W1=W1, b1=np.zeros(64), W2=W2, b2=np.zeros(64), w3=w3, b3=0.25))
    X = rng.uniform(-1, 1, (50, 8))
    y, _ = M.forward(th, X)
    coef = np.zeros(8)
    for k in range(64):
        coef[perm1[perm2[k]]] += w3[k] * e ** 2
    assert np.allclose(y, X @ coef + 0.25, rtol=0, atol=1e-6 * np.abs(coef).sum())


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g both bias-corrected moments equal g and g^2
    exactly, so every step moves each parameter by lr * g / (|g| + eps)."""
    th0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -1e-3, 2.0, -7.0])
    th, m, v = th0.copy(), np.zeros(4), np.zeros(4)
    for step in range(1, 8):
        th, m, v = M.adam(th, m, v, g, step, lr=1e-2)
        want = th0 - step * 1e-2 * g / (np.abs(g) + 1e-8)
        assert np.allclose(th, want, rtol=0, atol=1e-13), step


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(72)
    X = rng.uniform(-1, 1, (4096, 8))
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 7]
    th = _rand_theta(rng, 0.2)
    L0 = M.loss(th, X, t)
    perm = np.concatenate([rng.permutation(4096) for _ in range(20)])
    th, losses = M.train(th, X, t, perm, 256, lr=3e-3)
    assert losses.shape == (320,)
    assert M.loss(th, X, t) < 0.05 * L0


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(73)
    a = np.concatenate([rng.normal(0, 1, 2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 65504.0, 1e-40]])
    want = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).float().double().numpy()
    assert np.array_equal(M.bf16_round(a), want)
    assert M.bf16_round(1 + 2 ** -8) == 1.0          # tie to even
    assert M.bf16_round(1 + 3 * 2 ** -9) == 1 + 2 ** -7


def test_features_radial_track_and_rotation_invariance():
    rng = np.random.default_rng(74)
    n = 200
    ang = rng.uniform(-np.pi, np.pi, n)
    r = rng.uniform(3, 90, n)
    st = np.stack([r * np.cos(ang), r * np.sin(ang), rng.uniform(-50, 50, n),
                   rng.uniform(-2, 2, n), ang, rng.uniform(0.3, 2.8, n)], axis=1)
    f = M.features(st, 0, 100.0)
    assert np.allclose(f[:, 1], 0, atol=1e-12) and np.allclose(f[:, 2], 1, atol=1e-12)
    # radial line from radius r reaches radius 100 after 100 - r
    assert np.allclose(f[:, 5] * 100, 100 - r, atol=1e-9)
    st[:, 4] = ang + rng.uniform(-1.5, 1.5, n)
    f = M.features(st, 0, 100.0)
    assert np.allclose(f[:, 1] ** 2 + f[:, 2] ** 2, 1, atol=1e-12)
    rot = st.copy()
    a = 0.7
    rot[:, 0] = st[:, 0] * np.cos(a) - st[:, 1] * np.sin(a)
    rot[:, 1] = st[:, 0] * np.sin(a) + st[:, 1] * np.cos(a)
    rot[:, 4] = st[:, 4] + a
    assert np.allclose(M.features(rot, 0, 100.0), f, atol=1e-12)


def test_features_path_lengths_against_propagation_oracle(orc):
    """For a disk the straight-line feature is the exact path length; for a
    barrel it is the exact one in the no-field limit.  Both checked against
    the propagation oracle (C, FP64)."""
    import eventgen as E
    rng = np.random.default_rng(75)
    geom = E.geometry.barrel10_disks14(x0=0.0)
    n = 100
    ang = rng.uniform(-np.pi, np.pi, n)
    st = np.stack([5 * np.cos(ang), 5 * np.sin(ang), rng.uniform(-5, 5, n),
                   rng.choice([-1, 1], n) * rng.uniform(0.5, 2, n), ang + rng.uniform(-0.3, 0.3, n),
                   rng.uniform(0.2, 0.45, n)], axis=1)
    disk = 10 + 4          # +z disk at |z| = 190
    zd = geom[disk]["r_or_z"]
    f = M.features(st, 1, zd)
    cfg = orc.Config(geom, material=False)
    P0 = np.zeros(21)

    def paths(states, layer):
        out = []
        for p in states:
            st, _, _, s, _ = orc.propagate(cfg, layer, p, P0, noise=False)
            out.append(s if st == 0 else np.nan)
        return np.array(out)

    sd = paths(st, disk)
    ok = np.isfinite(sd)
    assert ok.sum() > 50
    assert np.allclose(f[ok, 5] * 100, sd[ok], rtol=1e-12, atol=1e-9)
    # barrel: a nearly straight track (c = 1e-7 / GeV)
    st2 = st.copy()
    st2[:, 3] = 1e-7
    st2[:, 5] = np.pi / 2
    sb = paths(st2, 6)              # barrel r = 50
    f2 = M.features(st2, 0, 50.0)
    assert np.all(np.isfinite(sb))
    assert np.allclose(f2[:, 5] * 100, sb, rtol=1e-7)
