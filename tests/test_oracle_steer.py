"""Pins of the oracle's steering (Sec. 3.1: tracking regions in eta, each
with the list of layers its track finding traverses): equivalence with the
dynamic next-surface navigation where the plan is the crossing order, plans
that omit or reorder layers by construction, seeds outside every region or
whose layers the plan lacks, and the finding efficiency of the generated
five-region plans on barrel + endcap events."""
import numpy as np

import eventgen as E
from tests import common as CM


def _find(orc, geom, evs, inp, **kw):
    return CM.oracle_find_events(orc, geom, evs, inp, **kw)


def test_barrel_plan_equals_dynamic_navigation(orc):
    """Ten barrels, one region over all eta with the plan 0..9: the steered
    finder returns exactly the dynamic navigation's hit lists and states."""
    geom, evs = E.find_events(n_events=2, n_tracks=300, n_noise=20_000, seed=31)
    inp = E.find_inputs(evs)
    a = _find(orc, geom, evs, inp)
    b = _find(orc, geom, evs, inp, steering=[dict(eta_lo=-10.0, eta_hi=10.0, layers=list(range(10)))])
    assert np.array_equal(a["hits"], b["hits"])
    assert np.array_equal(a["status"], b["status"])
    assert np.allclose(a["par"], b["par"], rtol=0, atol=0)


def test_plans_by_construction(orc):
    """A plan without layer 5 finds no hit there and the same hits elsewhere
    as far as the candidates agree; a reversed plan leaves nothing after the
    seed layers; seeds outside every region or whose layers the plan lacks
    are unreachable and keep their seed hits only."""
    geom, evs = E.find_events(n_events=1, n_tracks=300, n_noise=0, seed=32)
    inp = E.find_inputs(evs)
    full = _find(orc, geom, evs, inp)
    no5 = _find(orc, geom, evs, inp,
                steering=[dict(eta_lo=-10.0, eta_hi=10.0, layers=[0, 1, 2, 3, 4, 6, 7, 8, 9])])
    assert (no5["hits"][:, 5] < 0).all()
    assert (full["hits"][:, 5] >= 0).mean() > 0.9
    agree = (no5["hits"][:, :5] == full["hits"][:, :5]).all(axis=1)
    assert agree.mean() > 0.95
    rev = _find(orc, geom, evs, inp,
                steering=[dict(eta_lo=-10.0, eta_hi=10.0, layers=list(range(9, -1, -1)))])
    assert (rev["hits"][:, 3:] < 0).all()
    assert (rev["hits"][:, :3] >= 0).all()
    out = _find(orc, geom, evs, inp, steering=[dict(eta_lo=5.0, eta_hi=6.0, layers=list(range(10)))])
    assert (out["status"] & orc.ST_UNREACHABLE).all()
    lack = _find(orc, geom, evs, inp,
                 steering=[dict(eta_lo=-10.0, eta_hi=10.0, layers=[5, 6, 7, 8, 9])])
    assert (lack["status"] & orc.ST_UNREACHABLE).all()
    assert (lack["hits"][:, 3:] < 0).all()


def _efficiency(evs, inp, r):
    """Fraction of the seeded tracks' true hits (beyond the seed) found."""
    found = tot = 0
    for s in range(inp["seed_hits"].shape[0]):
        e = inp["seed_event"][s]
        t = inp["seed_track"][s]
        ev = evs[e]
        off = inp["event_off"][e]
        true = set((ev.seq_hit[t][ev.seq_hit[t] >= 0][3:] + off).tolist())
        got = set(r["hits"][s][r["hits"][s] >= 0].tolist())
        found += len(true & got)
        tot += len(true)
    return found / max(tot, 1)


def test_five_region_plans_keep_efficiency(orc):
    """Barrel + 2 x 7 disk events over |eta| < 2.5: finding that follows the
    generated five-region plans recovers about as many true hits as the
    dynamic navigation (fixed plans miss a few crossings whose order differs
    from the region's typical order)."""
    rng = np.random.default_rng(33)
    geom = E.geometry.barrel10_disks14(x0=0.02)
    evs = [E.make_event(rng, geom, 400, E.pt_power2(0.5, 50.0), 2.5, 2000) for _ in range(2)]
    inp = E.find_inputs(evs)
    dyn = _find(orc, geom, evs, inp)
    st = _find(orc, geom, evs, inp, steering=E.geometry.steering_plans(geom))
    e_dyn, e_st = _efficiency(evs, inp, dyn), _efficiency(evs, inp, st)
    print(f"hit efficiency: dynamic {e_dyn:.4f}, five-region plans {e_st:.4f}")
    assert e_dyn > 0.95
    assert e_st > e_dyn - 0.02
    same = (dyn["hits"] == st["hits"]).all(axis=1).mean()
    print(f"identical hit lists: {same:.3f}")
    assert same > 0.8


def test_field_steering_uniform_limit(orc):
    """Steering in the parametrised field with Z0 = 1e9 cm (Runge-Kutta solves
    of the plan's barrels and disks) reproduces the closed-form helix
    steering on uniform-field barrel + endcap events hit for hit."""
    rng = np.random.default_rng(34)
    geom = E.geometry.barrel10_disks14(x0=0.0)
    evs = [E.make_event(rng, geom, 300, E.pt_power2(0.5, 50.0), 2.5, 1000) for _ in range(2)]
    inp = E.find_inputs(evs)
    plans = E.geometry.steering_plans(geom)
    u = _find(orc, geom, evs, inp, steering=plans)
    f = _find(orc, geom, evs, inp, steering=plans, field_z0=1e9, field_step=0.5)
    kinds = np.array([L["kind"] for L in geom])
    assert (u["hits"][:, kinds == 1] >= 0).sum() > 500
    same = (u["hits"] == f["hits"]).all(axis=1)
    print(f"identical: {same.mean():.4f}")
    assert same.mean() > 0.995
    ok = same & (u["status"] == 0)
    assert CM.par_error(f["par"][ok], u["par"][ok]).max() < 1e-8


def test_field_steering_keeps_efficiency(orc):
    """Tracks traced through the field over barrels and disks: finding that
    follows the five-region plans in the field recovers about as many true
    hits as the field's dynamic navigation, and most hit lists agree."""
    import eventgen.field as EF
    geom, evs = EF.field_disk_events(n_events=2, n_tracks=400, n_noise=24_000, seed=32)
    inp = E.find_inputs(evs)
    kw = dict(field_z0=300.0, field_step=2.0)
    dyn = _find(orc, geom, evs, inp, **kw)
    st = _find(orc, geom, evs, inp, steering=E.geometry.steering_plans(geom), **kw)
    e_dyn, e_st = _efficiency(evs, inp, dyn), _efficiency(evs, inp, st)
    same = (dyn["hits"] == st["hits"]).all(axis=1).mean()
    print(f"field: hit efficiency dynamic {e_dyn:.4f}, plans {e_st:.4f}; identical {same:.3f}")
    assert e_dyn > 0.95
    assert e_st > e_dyn - 0.02
    assert same > 0.8
