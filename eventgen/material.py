"""r-z material maps (synthetic) and the workloads that use them.  A map is a
grid over r in [0, r_max) and z in [z_min, z_max): each cell holds the
radiation-length fraction x0 and the areal density xi [g/cm^2] of the
surface crossing it, at normal incidence (zero where no surface passes).
Input generation only."""
import numpy as np

from . import geometry as G
from .generate import make_event, pt_uniform

X0_SI = 21.82          # g/cm^2, radiation length of silicon
# cell grid chosen so that no layer lies on a cell edge: barrel radii fall at
# least 0.08 of a cell inside, disk planes half a cell or a third inside
R_MAX, N_R = 120.0, 250
Z_MIN, Z_MAX, N_Z = -300.0, 300.0, 250


def material_map(geom, base=0.02, seed=21):
    """Each barrel's cells along z and each disk's cells along r carry a
    smoothly varying thickness: base x (1 + 0.6 (u)^2 + 0.2 sin(3 u + phase))
    with u the position along the surface scaled to [-1, 1], so that
    neighbouring cells differ by about a percent; xi = x0 * X0(Si)."""
    rng = np.random.default_rng(seed)
    x0 = np.zeros((N_R, N_Z), np.float32)
    dr, dz = R_MAX / N_R, (Z_MAX - Z_MIN) / N_Z
    zc = Z_MIN + (np.arange(N_Z) + 0.5) * dz
    rc = (np.arange(N_R) + 0.5) * dr
    for L in geom:
        ph = rng.uniform(0, 2 * np.pi)
        if L["kind"] == 0:
            ir = int(np.floor(L["r_or_z"] / dr))
            u = np.clip(zc / max(abs(L["lo"]), abs(L["hi"])), -1, 1)
            x0[ir, :] = base * (1 + 0.6 * u ** 2 + 0.2 * np.sin(3 * u + ph))
        else:
            iz = int(np.floor((L["r_or_z"] - Z_MIN) / dz))
            u = np.clip((rc - L["lo"]) / (L["hi"] - L["lo"]) * 2 - 1, -1, 1)
            x0[:, iz] = base * (1 + 0.6 * u ** 2 + 0.2 * np.sin(3 * u + ph))
    return dict(r_max=R_MAX, z_min=Z_MIN, z_max=Z_MAX, x0=x0, xi=(x0 * X0_SI).astype(np.float32))


def eloss_sample(n_tracks=3000, seed=22, base=0.05, pt=(0.5, 1.0)):
    """Fit workload with energy loss: ten barrels (no per-layer x0: all
    material from the map), map thickness around `base` X0, pT U(pt) GeV,
    |eta| < 1, both charges.  Returns (geom, map, Event)."""
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=0.0)
    mat = material_map(geom, base=base, seed=seed)
    ev = make_event(rng, geom, n_tracks, pt_uniform(*pt), 1.0, material=mat)
    return geom, mat, ev


def eloss_find_events(n_events=3, n_tracks=800, n_noise=50_000, seed=23, base=0.03):
    """The finding workload's shape (ten barrels, pT^-2 on 0.5-50 GeV, |eta|
    < 1, uniform noise) with all material from an r-z map around `base` X0,
    tracks simulated with scattering and energy loss.  Returns (geom, map,
    events)."""
    from .generate import pt_power2
    rng = np.random.default_rng(seed)
    geom = G.barrel10(x0=0.0)
    mat = material_map(geom, base=base, seed=seed)
    per_layer = n_noise // len(geom)
    evs = [make_event(rng, geom, n_tracks, pt_power2(0.5, 50.0), 1.0, per_layer, material=mat)
           for _ in range(n_events)]
    return geom, mat, evs


def eloss_batch(seed=2, base=0.02, noise_per_track=60, lam_lo=200.0, lam_hi=4000.0,
                n_events=64):
    """The uneven-multiplicity batch's shape (64 events, N ~ Poisson(U(200,
    4000)), 60 noise hits per track, ten barrels + 2 x 7 disks, |eta| < 2.5)
    with all material from an r-z map around `base` X0 and tracks simulated
    with scattering and energy loss.  Returns (geom, map, events)."""
    from .generate import pt_power2
    rng = np.random.default_rng(seed)
    geom = G.barrel10_disks14(x0=0.0)
    mat = material_map(geom, base=base, seed=seed)
    evs = []
    for _ in range(n_events):
        lam = rng.uniform(lam_lo, lam_hi)
        n = max(1, int(rng.poisson(lam)))
        per_layer = noise_per_track * n // len(geom)
        evs.append(make_event(rng, geom, n, pt_power2(0.5, 50.0), 2.5, per_layer, material=mat))
    return geom, mat, evs


__all__ = ["material_map", "eloss_sample", "eloss_find_events", "eloss_batch", "X0_SI"]
