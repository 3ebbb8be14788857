"""GPU parity of the batched finding workload: 64 events with track counts
~ Poisson(lambda), lambda ~ U(200, 4000), 60 noise hits per track, barrel
plus 2 x 7 disks, |eta| < 2.5, 0.02 X0 per layer (the full-size batch, all
seeds compared with the FP64 oracle)."""
import numpy as np
import pytest

import eventgen as E
from tests import common as CM
from tests.test_gpu_find import K, _gpu_find, _check_parity  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg2():
    geom, evs = E.batch_events()
    return geom, evs, E.find_inputs(evs)


def test_batch_parity_full(K, orc, cfg2):
    geom, evs, inp = cfg2
    g = _gpu_find(K, geom, inp)
    o = CM.oracle_find_events(orc, geom, evs, inp)
    _check_parity(g, o, "batch", outlier_frac=1e-4)
    assert abs(int(g["counters"][0]) - o["n_prop"]) <= 0.01 * o["n_prop"]


def test_batch_widths_identical(K, cfg2):
    geom, evs, inp = cfg2
    ref = _gpu_find(K, geom, inp, 256, True)
    for w, lf in ((64, False), (128, True)):
        r = _gpu_find(K, geom, inp, w, lf)
        for k in ("hits", "par", "chi2", "ndf", "status"):
            assert np.array_equal(r[k], ref[k]), (w, lf, k)
