"""Detector descriptions used by the synthetic workloads.

A geometry is a list of layer descriptions (the paper's geometry section
describes the detector as a vector of per-layer records holding the layer's
dimensions, its hit-search windows and flags).  Here a record is a plain dict:

    kind      0 = barrel cylinder at radius ``r_or_z``; 1 = disk at z = ``r_or_z``
    r_or_z    cylinder radius or disk z position                      [cm]
    lo, hi    barrel: z extent [-Z, Z]; disk: radial extent [r_in, r_out] [cm]
    x0        material thickness in radiation lengths at normal incidence
    nbin_phi  number of phi bins over [-pi, pi)
    nbin_2    number of bins in z (barrel) or r (disk) over [lo, hi]
    win_su    largest hit sigma along r*phi on the layer (window sizing)  [cm]
    win_sv    largest hit sigma along z (barrel) or r (disk)            [cm]
    sig_u, sig_v  sigma used to smear hits on this layer                 [cm]

This module holds data only, no arithmetic of the filter.
"""
import math

BZ_TESLA = 3.8
BARREL_R = (4.0, 7.0, 11.0, 16.0, 25.0, 34.0, 50.0, 65.0, 80.0, 100.0)
DISK_Z = (30.0, 70.0, 110.0, 150.0, 190.0, 230.0, 270.0)

NBIN_PHI = 128
NBIN_2 = 32


def _barrel(r, x0, su, sv):
    half = r * math.sinh(1.0) + 2.0
    return dict(kind=0, r_or_z=r, lo=-half, hi=half, x0=x0,
                nbin_phi=NBIN_PHI, nbin_2=NBIN_2,
                win_su=su, win_sv=sv, sig_u=su, sig_v=sv)


def _disk(z, x0, su=0.01, sv=0.05):
    az = abs(z)
    return dict(kind=1, r_or_z=z, lo=az / math.sinh(2.5),
                hi=min(100.0, az / math.sinh(1.0)), x0=x0,
                nbin_phi=NBIN_PHI, nbin_2=NBIN_2,
                win_su=su, win_sv=sv, sig_u=su, sig_v=sv)


def barrel10(x0=0.0, su=0.01, sv=0.05):
    """Ten barrel cylinders, r = 4 ... 100 cm."""
    return [_barrel(r, x0, su, sv) for r in BARREL_R]


def barrel10_disks14(x0=0.02, su=0.01, sv=0.05):
    """Ten barrel cylinders plus seven disks on each side (|z| = 30 ... 270 cm).

    Layer order: barrels 0-9, +z disks 10-16, -z disks 17-23.
    """
    layers = [_barrel(r, x0, su, sv) for r in BARREL_R]
    layers += [_disk(z, x0) for z in DISK_Z]
    layers += [_disk(-z, x0) for z in DISK_Z]
    return layers


LAYER_FIELDS = ("kind", "r_or_z", "lo", "hi", "x0", "nbin_phi", "nbin_2",
                "win_su", "win_sv")


def steering_plans(geom, edges=(0.8, 1.6, 2.5), n_eta=41):
    """Tracking regions and their layer plans: five regions in eta (barrel
    |eta| < edges[0], transitions up to edges[1], endcaps up to edges[2], both
    signs).  A region's plan lists every layer a straight line from the origin
    crosses (inside the layer's extent) for some eta sampled in the region,
    ordered by the median path length to it over those etas.  Returns a list
    of dict(eta_lo, eta_hi, layers)."""
    import numpy as np
    e0, e1, e2 = edges
    bounds = [(-e2, -e1), (-e1, -e0), (-e0, e0), (e0, e1), (e1, e2)]
    out = []
    for lo, hi in bounds:
        etas = np.linspace(lo, hi, n_eta)[1:-1]
        paths = {}
        for eta in etas:
            sh, ch = np.sinh(eta), np.cosh(eta)
            for i, L in enumerate(geom):
                if L["kind"] == 0:
                    z = L["r_or_z"] * sh
                    if L["lo"] <= z <= L["hi"]:
                        paths.setdefault(i, []).append(L["r_or_z"] * ch)
                elif sh != 0 and np.sign(L["r_or_z"]) == np.sign(sh):
                    r = L["r_or_z"] / sh
                    if L["lo"] <= r <= L["hi"]:
                        paths.setdefault(i, []).append(abs(L["r_or_z"]) * ch / abs(sh))
        plan = sorted(paths, key=lambda i: float(np.median(paths[i])))
        out.append(dict(eta_lo=float(lo), eta_hi=float(hi), layers=[int(i) for i in plan]))
    return out
