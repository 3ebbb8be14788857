"""GPU parity of steered finding (tracking regions in eta with layer plans,
Sec. 3.1) against the FP64 oracle under the finding tests' tie rules (a
seed whose eta lies within 1e-3 of a region edge counts as a tie), plus the
equivalences that pin the GPU path to its own dynamic navigation."""
import numpy as np
import pytest

import eventgen as E
from tests import common as CM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_02253_amd as K
    from paper_1906_02253_amd import pipeline
    K.pipeline = pipeline
    return K


def _events(seed=41, n_events=3, n_tracks=600):
    rng = np.random.default_rng(seed)
    geom = E.geometry.barrel10_disks14(x0=0.02)
    evs = [E.make_event(rng, geom, n_tracks, E.pt_power2(0.5, 50.0), 2.5, 3000)
           for _ in range(n_events)]
    return geom, evs


def _run(K, geom, inp, steering=None, batched=False, width=64):
    import torch
    ctx = K.Context(geom)
    ctx.set_find_config(width, False)
    if steering is not None:
        ctx.set_steering(steering)
    fp = K.pipeline.FindProblem(ctx, inp)
    if batched:
        fp.run_batched()
        fp.run_batched()
    else:
        fp.run()
    torch.cuda.synchronize()
    return fp.results()


@pytest.mark.parametrize("batched", [False, True])
def test_steered_find_matches_oracle(K, orc, batched):
    """Three events of 600 tracks over |eta| < 2.5 (ten barrels + 2 x 7
    disks, 0.02 X0, 3,000 noise hits per layer), five-region plans."""
    geom, evs = _events()
    inp = E.find_inputs(evs)
    plans = E.geometry.steering_plans(geom)
    g = _run(K, geom, inp, plans, batched=batched)
    o = CM.oracle_find_events(orc, geom, evs, inp, steering=plans)
    n_same, n_exc, bad = CM.compare_find(g, o)
    ns = g["hits"].shape[0]
    print(f"steered find: {n_same}/{ns} identical, {n_exc} excused, {bad.size} unexplained")
    assert bad.size == 0
    assert n_same > 0.95 * ns
    assert np.array_equal(g["status"][o["tie"] < 0] & ~K.ST_FALLBACK, o["status"][o["tie"] < 0])
    assert n_exc <= CM.MAX_EXCUSED_FRAC * max(g["hits"].shape[0], 1000)
    CM.check_find_params(g, o, "params", lambda s: CM.oracle_sensitivity(
        orc, geom, evs, inp, s, steering=plans))


def test_barrel_plan_equals_dynamic(K):
    """Ten barrels and one region whose plan is 0..9: bit-identical to the
    dynamic navigation on the GPU; removing the steering restores it."""
    import torch
    geom, evs = E.find_events(n_events=2, n_tracks=400, n_noise=20_000, seed=42)
    inp = E.find_inputs(evs)
    a = _run(K, geom, inp)
    b = _run(K, geom, inp, [dict(eta_lo=-10.0, eta_hi=10.0, layers=list(range(10)))])
    for k in ("hits", "par", "chi2", "ndf", "status"):
        assert np.array_equal(a[k], b[k]), k
    ctx = K.Context(geom)
    ctx.set_steering([dict(eta_lo=-10.0, eta_hi=10.0, layers=[5, 6, 7, 8, 9])])
    ctx.set_steering(None)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run()
    torch.cuda.synchronize()
    c = fp.results()
    for k in ("hits", "par", "status"):
        assert np.array_equal(a[k], c[k]), k


def test_unreachable_seeds_and_validation(K):
    """Seeds outside every region, or whose layers the plan lacks, are not
    searched (UNREACHABLE, seed hits only); bad plans and steering with the
    learned guess are refused."""
    geom, evs = E.find_events(n_events=1, n_tracks=200, n_noise=0, seed=43)
    inp = E.find_inputs(evs)
    out = _run(K, geom, inp, [dict(eta_lo=5.0, eta_hi=6.0, layers=list(range(10)))])
    assert (out["status"] & K.ST_UNREACHABLE).all()
    assert (out["hits"][:, 3:] < 0).all()
    lack = _run(K, geom, inp, [dict(eta_lo=-10.0, eta_hi=10.0, layers=[5, 6, 7, 8, 9])])
    assert (lack["status"] & K.ST_UNREACHABLE).all()
    ctx = K.Context(geom)
    for bad in ([dict(eta_lo=0.0, eta_hi=1.0, layers=[1, 1])],
                [dict(eta_lo=0.0, eta_hi=1.0, layers=[99])],
                [dict(eta_lo=1.0, eta_hi=0.0, layers=[1])],
                [dict(eta_lo=0.0, eta_hi=1.0, layers=[1])] * 9):
        with pytest.raises(K.KFError):
            ctx.set_steering(bad)
    ctx.set_steering([dict(eta_lo=-10.0, eta_hi=10.0, layers=list(range(10)))])
    ctx.mlp_load(E.mlp_init(1))
    fp = K.pipeline.FindProblem(ctx, inp)
    with pytest.raises(K.KFError, match="exclude"):
        fp.run(K.INIT_MLP)


def test_steered_find_with_material_map(K, orc):
    """Steered finding with the r-z material map (its own kernel instance):
    the five-region plans on two barrel + endcap events, scattering and mean
    energy loss from a map around 0.02 X0, against the FP64 oracle with the
    same plans and map."""
    import torch
    import eventgen.material as EM
    geom, evs = _events(seed=42, n_events=2, n_tracks=500)
    inp = E.find_inputs(evs)
    plans = E.geometry.steering_plans(geom)
    mat = EM.material_map(geom, base=0.02, seed=21)
    ctx = K.Context(geom)
    ctx.set_find_config(64, False)
    ctx.set_steering(plans)
    ctx.set_material(mat)
    fp = K.pipeline.FindProblem(ctx, inp)
    fp.run()
    torch.cuda.synchronize()
    g = fp.results()
    o = CM.oracle_find_events(orc, geom, evs, inp, steering=plans, material_map=mat)
    n_same, n_exc, bad = CM.compare_find(g, o)
    ns = g["hits"].shape[0]
    print(f"steered find with map: {n_same}/{ns} identical, {n_exc} excused, {bad.size} unexplained")
    assert bad.size == 0
    assert n_same > 0.95 * ns
    assert n_exc <= CM.MAX_EXCUSED_FRAC * max(g["hits"].shape[0], 1000)
    CM.check_find_params(g, o, "params", lambda s: CM.oracle_sensitivity(
        orc, geom, evs, inp, s, steering=plans, material_map=mat))
