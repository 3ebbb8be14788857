"""Shared helpers for the parity tests: input marshalling and the comparison
rules (tolerances stated once, here)."""
import numpy as np

# Parameter parity: |d| <= REL * max(|p_oracle|, floor); phi compared modulo 2 pi.
REL = 1e-4
FLOORS = np.array([1.0, 1.0, 1.0, 0.01, 1.0, 1.0])     # cm, cm, cm, 1/GeV, rad, rad
CHI2_REL = 1e-3                                        # |dchi2| <= 1e-3 * max(chi2, ndf, 1)


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def par_error(gpu_par, orc_par):
    """Relative parameter error in units of the parity scale (1 = at tolerance)."""
    d = gpu_par - orc_par
    d[:, 4] = wrap(d[:, 4])
    scale = np.maximum(np.abs(orc_par), FLOORS)
    return np.abs(d) / scale


def chi2_error(gpu_chi2, orc_chi2, ndf):
    return np.abs(gpu_chi2 - orc_chi2) / np.maximum(np.maximum(np.abs(orc_chi2), ndf), 1.0)


def seed_hits(ev):
    """[n_trk, 3] first three hits in crossing order (tracks with >= 3 hits)."""
    return ev.seq_hit[:, :3]


def ld_of(n):
    return max(64, (n + 63) // 64 * 64)


def soa_int(a, ld, fill=-1):
    """[n, k] int array -> [k, ld] int32 (SoA) padded with `fill`."""
    n, k = a.shape
    out = np.full((k, ld), fill, np.int32)
    out[:, :n] = a.T
    return out
