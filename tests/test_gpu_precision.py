"""Precision variants on the ill-conditioned fit workload: 200,000 tracks
mixing 0.3 GeV loopers and 100 GeV stiff tracks, hit sigma_u log-uniform in
[0.002, 0.01] cm, sigma_v = 5 sigma_u, no material.  Each GPU variant (all
FP32; mixed = FP32 state/transport with FP64 covariance and update; all
FP64) is compared with the FP64 oracle; max and RMS relative error per
parameter are printed, and the bars are:
  FP64   max relative error < 1e-9 (same algorithm, rounding order only)
  mixed  max relative error < 2e-4 and RMS < 2e-5 per parameter, chi2 < 1e-3
         (FP32 state transport: on 100 GeV tracks with 0.002 cm hits the
         curvature tail reaches ~1.2e-4 relative, about 1% of its sigma)
  FP32   reported; must stay finite for >= 99% of tracks
"""
import numpy as np
import pytest

import eventgen as E
from tests import common as CM
from tests.test_gpu_fit import K, _gpu_fit, _oracle_fit  # noqa: F401

pytestmark = pytest.mark.gpu

NAMES = ("x", "y", "z", "c", "phi", "theta")


@pytest.fixture(scope="module")
def cfg3(orc):
    geom, ev = E.precision_sample()
    return geom, ev, _oracle_fit(orc, geom, ev)


def _report(label, g, o):
    ok = (o["status"] == 0) & (g["status"] == 0)
    err = CM.par_error(g["par"][ok], o["par"][ok])
    cerr = CM.chi2_error(g["chi2"][ok], o["chi2"][ok], o["ndf"][ok])
    line = " ".join(f"{n}:max={err[:, i].max():.1e},rms={np.sqrt((err[:, i]**2).mean()):.1e}"
                    for i, n in enumerate(NAMES))
    print(f"{label}: ok={ok.mean():.4f} {line} chi2:max={cerr.max():.1e}")
    return ok, err, cerr


def test_precision_fp64(K, cfg3):
    geom, ev, o = cfg3
    g = _gpu_fit(K, geom, ev, flags=K.PREC_FP64)
    ok, err, cerr = _report("fp64", g, o)
    assert np.array_equal(g["status"], o["status"])
    assert err.max() < 1e-9 and cerr.max() < 1e-9


def test_precision_mixed(K, cfg3):
    geom, ev, o = cfg3
    g = _gpu_fit(K, geom, ev, flags=K.PREC_MIXED)
    ok, err, cerr = _report("mixed", g, o)
    assert np.array_equal(g["status"], o["status"])
    assert err.max() < 2 * CM.REL and cerr.max() < CM.CHI2_REL
    assert np.sqrt((err ** 2).mean(axis=0)).max() < 0.2 * CM.REL


def test_precision_fp32(K, cfg3):
    geom, ev, o = cfg3
    g = _gpu_fit(K, geom, ev, flags=K.PREC_FP32)
    ok, err, cerr = _report("fp32", g, o)
    assert ok.mean() > 0.99
