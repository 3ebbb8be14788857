"""Pins of the oracle's seed cleaning (Sec. 3.2: duplicate seeds removed before
finding, by hit identity and the seeds' pT, eta and phi) against answers
fixed by construction, invariants any correct implementation of the rule
must satisfy, its relation to the serial greedy cleaning, and the physics of
module-overlap duplicates."""
import numpy as np
import pytest

import eventgen.overlap as EO

DETA, DPHI, DC = 0.01, 0.01, 0.05


def _seeds(rng, n, eta=None, phi=None, c=None):
    eta = rng.uniform(-2, 2, n) if eta is None else np.asarray(eta, float)
    phi = rng.uniform(-np.pi, np.pi, n) if phi is None else np.asarray(phi, float)
    c = rng.uniform(-2, 2, n) if c is None else np.asarray(c, float)
    par = np.zeros((n, 6))
    par[:, 3] = c
    par[:, 4] = phi
    par[:, 5] = 2 * np.arctan(np.exp(-eta))
    return par


def _clean(orc, par, chi2, hits=None, event=None, status=None, **kw):
    n = par.shape[0]
    hits = np.arange(3 * n).reshape(n, 3) if hits is None else hits
    event = np.zeros(n, int) if event is None else event
    status = np.zeros(n, int) if status is None else status
    return orc.clean_seeds(par, chi2, status, event, hits, **kw)


def _dup_matrix(par, hits, event, deta=DETA, dphi=DPHI, dc=DC):
    """Duplicate relation evaluated pair by pair with numpy broadcasting."""
    eta = -np.log(np.tan(par[:, 5] / 2))
    d_eta = np.abs(eta[:, None] - eta[None, :])
    d_phi = np.abs(np.angle(np.exp(1j * (par[:, 4][:, None] - par[:, 4][None, :]))))
    d_c = np.abs(par[:, 3][:, None] - par[:, 3][None, :])
    share = (hits[:, None, :, None] == hits[None, :, None, :]).any(axis=(2, 3))
    D = (share | ((d_eta < deta) & (d_phi < dphi) & (d_c < dc))) & (event[:, None] == event[None, :])
    np.fill_diagonal(D, False)
    return D


def test_groups_keep_their_best(orc):
    """Groups of identical-parameter seeds far from each other: exactly the
    lowest-chi2 seed of each group survives; equal chi2 goes to the lower
    index."""
    rng = np.random.default_rng(1)
    g = 40
    centres = _seeds(rng, g, eta=np.linspace(-2, 2, g), phi=np.linspace(-3, 3, g),
                     c=np.linspace(-1.5, 1.5, g))
    sizes = rng.integers(1, 6, g)
    par = np.repeat(centres, sizes, axis=0)
    grp = np.repeat(np.arange(g), sizes)
    chi2 = rng.uniform(0, 10, par.shape[0])
    perm = rng.permutation(par.shape[0])
    par, grp, chi2 = par[perm], grp[perm], chi2[perm]
    keep, tie = _clean(orc, par, chi2)
    # groups lie far apart in every parameter: only close chi2 values mark ties
    assert tie.mean() < 0.1
    for k in range(g):
        m = np.nonzero(grp == k)[0]
        assert keep[m].sum() == 1
        assert keep[m[np.argmin(chi2[m])]]
    # equal chi2: the lower index wins
    par2 = np.repeat(centres[:1], 3, axis=0)
    keep2, _ = _clean(orc, par2, np.array([2.0, 2.0, 2.0]))
    assert keep2.tolist() == [True, False, False]


def test_shared_hit_alone_makes_duplicates(orc):
    rng = np.random.default_rng(2)
    par = _seeds(rng, 3, eta=[-1, 0, 1], phi=[-2, 0, 2], c=[-1, 0.5, 1.5])
    hits = np.array([[0, 1, 2], [3, 2, 4], [5, 6, 7]])
    keep, _ = _clean(orc, par, np.array([1.0, 0.5, 0.1]), hits=hits)
    assert keep.tolist() == [False, True, True]
    # no hit shared (-1 entries never match each other)
    hits = np.array([[0, 1, -1], [3, -1, 4], [5, 6, 7]])
    keep, _ = _clean(orc, par, np.array([1.0, 0.5, 0.1]), hits=hits)
    assert keep.all()


@pytest.mark.parametrize("which", ["eta", "phi", "c"])
def test_thresholds_apply_to_their_own_parameter(orc, which):
    """Distinct thresholds (0.01, 0.02, 0.012): a difference of 0.015 is a
    duplicate only in phi, and each threshold is strict."""
    base = dict(eta=[0.5, 0.5], phi=[1.0, 1.0], c=[0.8, 0.8])
    thr = dict(eta=0.01, phi=0.02, c=0.012)[which]
    kw = dict(deta=0.01, dphi=0.02, dc=0.012)
    rng = np.random.default_rng(3)
    for d, want_dup in ((0.015, which == "phi"), (thr * 0.999, True), (thr * 1.001, False)):
        v = dict(base)
        v[which] = [base[which][0], base[which][0] + d]
        keep, _ = _clean(orc, _seeds(rng, 2, **v), np.array([1.0, 2.0]), **kw)
        assert keep.tolist() == [True, not want_dup], (which, d)


def test_phi_wraps(orc):
    rng = np.random.default_rng(4)
    par = _seeds(rng, 2, eta=[0.3, 0.3], phi=[np.pi - 0.002, -np.pi + 0.002], c=[1.0, 1.0])
    keep, _ = _clean(orc, par, np.array([1.0, 2.0]))
    assert keep.tolist() == [True, False]


def test_events_and_status_are_respected(orc):
    rng = np.random.default_rng(5)
    par = np.repeat(_seeds(rng, 1), 4, axis=0)
    keep, _ = _clean(orc, par, np.array([1.0, 2.0, 3.0, 4.0]), event=np.array([0, 1, 0, 1]))
    assert keep.tolist() == [True, True, False, False]
    # a failed seed neither removes nor is removed
    keep, _ = _clean(orc, par, np.array([1.0, 2.0, 3.0, 4.0]), status=np.array([2, 0, 0, 8]))
    assert keep.tolist() == [True, True, False, True]


def test_chi2_compared_in_float(orc):
    """Two values equal in float but not in double tie, and the lower index
    wins even though it has the larger double value."""
    rng = np.random.default_rng(6)
    par = np.repeat(_seeds(rng, 1), 2, axis=0)
    a = 3.0
    b = a - 1e-12
    assert np.float32(a) == np.float32(b) and b < a
    keep, tie = _clean(orc, par, np.array([a, b]))
    assert keep.tolist() == [True, False] and tie.all()


def test_invariants_on_dense_random_sets(orc):
    """Dense random seeds (many chains of duplicates): no two kept seeds are
    duplicates; a removed seed always has a better duplicate; the best seed of
    every connected group is kept; the result does not depend on the seeds'
    order beyond the index tie-break; the kept set lies inside the serial
    greedy cleaning's kept set."""
    rng = np.random.default_rng(7)
    n = 600
    par = _seeds(rng, n, eta=rng.uniform(0, 0.08, n), phi=rng.uniform(0, 0.08, n),
                 c=rng.uniform(0, 0.4, n))
    hits = rng.integers(0, 4000, (n, 3))
    event = rng.integers(0, 2, n)
    chi2 = rng.uniform(0, 20, n)
    keep, _ = _clean(orc, par, chi2, hits=hits, event=event)
    D = _dup_matrix(par, hits, event)
    assert D.sum() > n                    # chains, not just pairs
    k = np.nonzero(keep)[0]
    assert not D[np.ix_(k, k)].any()
    order = np.lexsort((np.arange(n), chi2.astype(np.float32)))
    rank = np.empty(n, int)
    rank[order] = np.arange(n)
    for j in np.nonzero(~keep)[0]:
        assert (D[:, j] & (rank < rank[j])).any()
    # connected groups
    lab = np.arange(n)
    changed = True
    while changed:
        nl = np.where(D, lab[None, :], n).min(axis=1)
        nl = np.minimum(nl, lab)
        changed = (nl != lab).any()
        lab = nl
    for g in np.unique(lab):
        m = np.nonzero(lab == g)[0]
        assert keep[m[np.argmin(rank[m])]]
    # order independence
    perm = rng.permutation(n)
    keep_p, _ = _clean(orc, par[perm], chi2[perm], hits=hits[perm], event=event[perm])
    assert np.array_equal(keep_p, keep[perm])
    # serial greedy in rank order
    greedy = np.zeros(n, bool)
    for j in order:
        greedy[j] = not (D[j] & greedy).any()
    assert not (keep & ~greedy).any()
    assert greedy.sum() > keep.sum()      # the chains make the two differ here


def test_cliques_match_serial_greedy(orc):
    """When the duplicate relation is an equivalence (separated clusters of
    mutually close seeds), the order-free rule and the serial greedy
    cleaning keep the same seeds: one per cluster."""
    rng = np.random.default_rng(8)
    cl = 30
    centre = _seeds(rng, cl, eta=np.linspace(-2, 2, cl), phi=np.linspace(-3, 3, cl),
                    c=np.linspace(-1, 1, cl))
    par = np.repeat(centre, 4, axis=0)
    par[:, 4] += rng.uniform(-0.002, 0.002, par.shape[0])
    par[:, 3] += rng.uniform(-0.01, 0.01, par.shape[0])
    chi2 = rng.uniform(0, 5, par.shape[0])
    keep, _ = _clean(orc, par, chi2)
    assert keep.sum() == cl
    for k in range(cl):
        m = np.arange(4 * k, 4 * k + 4)
        assert keep[m[np.argmin(chi2[m])]]


def test_overlap_duplicates_cleaned(orc):
    """Module-overlap events: one particle gives up to eight seeds (about 2.2
    on average at 30% overlap per layer); after cleaning almost every particle
    keeps exactly one, and hardly any particle loses all of its seeds."""
    geom, evs, ovls = EO.overlap_find_events(n_events=2, n_tracks=800, n_noise=0)
    inp = EO.overlap_inputs(evs, ovls)
    ns = inp["seed_hits"].shape[0]
    cfg = orc.Config(geom)
    par, chi2, st = np.zeros((ns, 6)), np.zeros(ns), np.zeros(ns, np.int32)
    for e, ev in enumerate(evs):
        m = np.nonzero(inp["seed_event"] == e)[0]
        shl = inp["seed_hits_local"][m]
        p0, c0 = np.zeros((m.size, 6)), np.zeros((m.size, 21))
        for k in range(m.size):
            p0[k], c0[k] = orc.seed(*[np.array([ev.x[h], ev.y[h], ev.z[h]]) for h in shl[k]])
        r = orc.fit(cfg, dict(x=ev.x, y=ev.y, z=ev.z, su=ev.su, sv=ev.sv), inp["seed_layers"][m],
                    shl, p0, c0, n_threads=8)
        par[m], chi2[m], st[m] = r["par"], r["chi2"], r["status"]
    keep, _ = orc.clean_seeds(par, chi2, st, inp["seed_event"], inp["seed_hits"])
    key = inp["seed_event"].astype(np.int64) * 100_000 + inp["seed_track"]
    _, inv = np.unique(key, return_inverse=True)
    per = np.bincount(inv)
    kept = np.bincount(inv, weights=keep)
    assert per.mean() > 2.0
    assert (kept >= 1).mean() > 0.995
    assert kept.mean() < 1.01
