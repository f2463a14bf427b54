"""Pins of the oracle's other two forms of the generator factor of Sec. VI.

Sec. VI lets a generator run once every f_g occasions instead of with probability 1/f_g,
and, in reverse, run N_g times at every occasion with the products' weight divided by N_g.
The readings (the event still acts on its parent every time it fires, as in the random
form):
* deterministic form: a parent's events are numbered by its event count; with F = f_g the
  children of event e are made iff (e + phi) mod F == 0 for a phase phi fixed over the
  parent's life, drawn from its id;
* reverse mode for emission: every run that fires makes a photon of weight w / N_g from the
  momentum the lepton had before the sub-step's events, and the lepton recoils by the sum
  of those momenta over N_g;
* reverse mode for pairs: the photon stands for N_g copies of weight w / N_g, each run that
  fires makes a pair of that weight, the photon keeps the weight of the copies left, and is
  removed when all of them decay.
What the paper and the arithmetic fix, and what these tests check: run 0 is the ordinary
draw; the runs are independent; weighted numbers, energies and momenta are unbiased; the
weighted momentum (emission) and weight (pairs) are conserved event by event; a parent
with n events makes floor(n / F) or ceil(n / F) children, at event numbers one phase
explains over all steps; and every event is sampled with probability 1/F."""
import math

import numpy as np
import pytest

from paper_1412_6426_amd import workloads as W

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)


def _stores(orc, init, caps):
    st = [orc.Store(caps[0]), orc.Store(caps[1]), orc.Store(caps[2], with_events=False)]
    for s, cols in zip(st, init):
        s.load(cols)
    return st


def _electrons(orc, n=20_000, dt_frac=0.001, steps=1, **kw):
    """Electrons at chi = 1 in a uniform B, one sub-step per step (a tenth of a percent of
    the gyro period), emission only; returns the stores and the per-step records."""
    w = W.uniform_b(n=n, steps=steps, dt_frac=dt_frac, photon_capacity=16 * n * steps)
    st = _stores(orc, W.uniform_b_initial(w), w.capacity)
    fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=w.field.b0)
    par = orc.Params(dt=w.dt, eps_r=w.eps_r, pairs=0, push_photons=0, seed=9,
                     forced_substeps=1, **kw)
    out = orc.run(st, fld, par, steps)
    return st, out, w


def _photons(n=20_000, k=1000.0, seed=1):
    rng = np.random.default_rng(seed)
    zero = np.zeros(n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    cols = W._seed_columns(zero, zero, zero, k * np.cos(phi), k * np.sin(phi), zero)
    cols["w"] = rng.uniform(0.5, 2.0, n)
    return cols


def _pair_step(orc, cols, dt=3e5, **kw):
    """One step of photons with chi_gamma = 2 (k = 1000 perpendicular to B = 0.002 E_S)."""
    n = len(cols["x"])
    st = [orc.Store(16 * n), orc.Store(16 * n), orc.Store(n, with_events=False)]
    st[0].load(W.empty_columns())
    st[1].load(W.empty_columns())
    st[2].load(cols)
    fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=(0, 0, 0.002))
    par = orc.Params(dt=dt, eps_r=1.0, seed=3, emission=0, **kw)
    out = orc.run(st, fld, par, 1)
    return st, out[0]


def _by_id(v):
    o = np.argsort(v["id"])
    return {k: a[o] for k, a in v.items()}


def _children_of(parents, children):
    """Children per parent (parents in store order)."""
    order = np.argsort(parents)
    pos = np.searchsorted(parents[order], children)
    assert np.array_equal(parents[order][pos], children)
    cnt = np.bincount(order[pos], minlength=len(parents))
    return cnt


# ---------------------------------------------------------------------------------------
# reverse mode, emission
# ---------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def emission_runs(orc):
    return (_electrons(orc), _electrons(orc, runs_photon=4), _electrons(orc, emission=0))


def test_reverse_emission_run_zero_is_the_ordinary_draw(emission_runs):
    (a, out_a, _), (b, out_b, _), _ = emission_runs
    ga, gb = _by_id(a[2].view()), _by_id(b[2].view())
    assert len(ga["id"]) == out_a[0]["emitted"] > 500
    assert len(gb["id"]) == out_b[0]["emitted"]
    pos = np.searchsorted(gb["id"], ga["id"])
    assert np.array_equal(gb["id"][pos], ga["id"])  # run 0 makes the photons of N_g = 1
    for c in ("x", "y", "z", "px", "py", "pz", "parent", "birth"):
        assert np.array_equal(gb[c][pos], ga[c]), c
    assert np.array_equal(gb["w"][pos], ga["w"] / 4.0)
    assert len(np.unique(gb["id"])) == len(gb["id"])


def test_reverse_emission_conserves_the_weighted_momentum(emission_runs):
    _, (b, _, _), (c, _, _) = emission_runs
    e, push = b[0].view(), c[0].view()  # the electrons after the events, and without them
    assert np.array_equal(e["id"], push["id"])
    g = b[2].view()
    order = np.argsort(e["id"])
    idx = order[np.searchsorted(e["id"][order], g["parent"])]
    for d in ("px", "py", "pz"):
        k_sum = np.bincount(idx, weights=g["w"] * g[d], minlength=len(e["id"]))
        lhs = e["w"] * e[d] + k_sum
        rhs = push["w"] * push[d]
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * 1000.0), d
    fired = np.bincount(idx, minlength=len(e["id"])) > 0
    assert fired.sum() > 1000
    assert not np.array_equal(e["px"][fired], push["px"][fired])  # they did recoil


def test_reverse_emission_runs_are_independent_and_unbiased(emission_runs):
    (a, _, _), (b, _, _), _ = emission_runs
    n = len(a[0].view()["id"])
    k1 = _children_of(a[0].view()["id"], a[2].view()["parent"])
    k4 = _children_of(b[0].view()["id"], b[2].view()["parent"])
    p = k1.mean()  # every electron has the same chi and gamma: one probability per run
    assert 0.02 < p < 0.3
    sd = math.sqrt(4 * p * (1 - p) / n)
    assert abs(k4.mean() - 4 * p) < 5 * sd + 4 * math.sqrt(p * (1 - p) / n)
    # firings per electron are binomial(4, p): runs that shared a draw would all fire at once
    for m in range(5):
        q = math.comb(4, m) * p ** m * (1 - p) ** (4 - m)
        got = np.count_nonzero(k4 == m)
        assert abs(got - n * q) < 5 * math.sqrt(n * q * (1 - q)) + 0.02 * n * q, m
    # the weighted photon energy is unbiased
    ga, gb = a[2].view(), b[2].view()
    ea = ga["w"] * np.sqrt(ga["px"] ** 2 + ga["py"] ** 2 + ga["pz"] ** 2)
    eb = gb["w"] * np.sqrt(gb["px"] ** 2 + gb["py"] ** 2 + gb["pz"] ** 2)
    sd = math.sqrt(float((ea ** 2).sum()) + float((eb ** 2).sum()))
    assert abs(float(eb.sum()) - float(ea.sum())) < 5 * sd


def test_reverse_emission_stats(emission_runs):
    (_, _, _), (b, out_b, _), _ = emission_runs
    g = b[2].view()
    s = out_b[0]
    assert s["emitted"] == len(g["id"])
    eps = np.sqrt(g["px"] ** 2 + g["py"] ** 2 + g["pz"] ** 2)
    assert s["photon_energy"] == pytest.approx(float((g["w"] * eps).sum()), rel=1e-12)
    b = np.floor(10.0 * (np.log10(eps) + 8.0))
    b = b[(b >= 0) & (b < len(s["photon_hist"]))].astype(int)
    want = np.bincount(b, minlength=len(s["photon_hist"]))
    assert np.abs(np.array(s["photon_hist"]) - want).sum() <= 2  # a log10 ulp at a bin edge


# ---------------------------------------------------------------------------------------
# reverse mode, pairs
# ---------------------------------------------------------------------------------------
def _row_of(ids, parents):
    """Row of each parent id among `ids`."""
    order = np.argsort(ids)
    pos = np.searchsorted(ids[order], parents)
    assert np.array_equal(ids[order][pos], parents)
    return order[pos]


def test_reverse_pairs_conserve_the_photon_weight(orc):
    """One sub-step of chi_gamma = 2 photons in which about a fifth of the copies decay."""
    cols = _photons()
    b, sb = _pair_step(orc, cols, runs_pair=3)
    ph = b[2].view()
    e, p = b[0].view(), b[1].view()
    assert len(e["id"]) == len(p["id"]) == sb["pairs"] > 1000
    idx = _row_of(cols["id"], e["parent"])
    w_pairs = np.bincount(idx, weights=e["w"], minlength=len(cols["id"]))
    w_left = np.where(ph["id"] == DEAD, 0.0, ph["w"])
    assert np.allclose(w_left + w_pairs, cols["w"], rtol=1e-14, atol=0)
    # an electron and a positron per firing (stored in the same order), with the same
    # weight, sharing k
    assert np.array_equal(e["parent"], p["parent"])
    assert np.array_equal(e["birth"], p["birth"])
    assert np.array_equal(e["w"], p["w"])
    for c in ("px", "py", "pz"):
        assert np.allclose(e[c] + p[c], cols[c][idx], rtol=0, atol=1e-12 * 1000.0)
    dead = ph["id"] == DEAD
    partial = (~dead) & (ph["w"] != cols["w"])
    assert dead.sum() > 50 and partial.sum() > 1000  # whole and partial decays both happen
    assert np.all(np.bincount(idx, minlength=len(cols["id"]))[dead] >= 3)
    assert np.all(ph["w"][partial] < cols["w"][partial])


def test_reverse_pairs_run_zero_and_unbiased(orc):
    cols = _photons(seed=5)
    a, sa = _pair_step(orc, cols, forced_substeps=1)
    b, sb = _pair_step(orc, cols, forced_substeps=1, runs_pair=3)
    dead_a = a[2].view()["id"] == DEAD
    n, p = len(cols["id"]), float(dead_a.mean())
    assert 0.05 < p < 0.5
    # run 0 makes the pairs of N_g = 1
    for sp in (0, 1):
        va, vb = _by_id(a[sp].view()), _by_id(b[sp].view())
        pos = np.searchsorted(vb["id"], va["id"])
        assert np.array_equal(vb["id"][pos], va["id"])
        for c in ("x", "y", "z", "px", "py", "pz", "parent", "birth"):
            assert np.array_equal(vb[c][pos], va[c]), c
        assert np.allclose(vb["w"][pos], va["w"] / 3.0, rtol=1e-15, atol=0)
    # one sub-step: the copies decay independently, so a photon is removed with
    # probability p^3 and the pair weight made is unbiased
    dead_b = b[2].view()["id"] == DEAD
    q = p ** 3
    assert abs(dead_b.sum() - n * q) < 5 * math.sqrt(n * q * (1 - q)) + 0.02 * n * q
    e = b[0].view()
    m = _children_of(cols["id"], e["parent"])
    for j in range(4):
        qj = math.comb(3, j) * p ** j * (1 - p) ** (3 - j)
        assert abs(np.count_nonzero(m == j) - n * qj) < 5 * math.sqrt(n * qj) + 0.02 * n * qj
    w_made = float(e["w"].sum())
    w_dec = float(cols["w"][dead_a].sum())
    sd = math.sqrt(float((cols["w"] ** 2).sum()) * p * (1 - p) * (1 + 1 / 3))
    assert abs(w_made - w_dec) < 5 * sd
    assert sb["pairs"] == len(e["id"])


# ---------------------------------------------------------------------------------------
# deterministic form
# ---------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def every_runs(orc):
    """12 steps of 3000 electrons at chi = 1 (about 8 sub-steps a step), f_g = 4 every
    fourth event and f_g = 1, step by step with the event counts and children of each."""
    out = {}
    for f, every in ((1.0, 0), (4.0, 1)):
        w = W.uniform_b(n=3000, steps=12)
        st = _stores(orc, W.uniform_b_initial(w), w.capacity)
        fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=w.field.b0)
        par = orc.Params(dt=w.dt, eps_r=w.eps_r, pairs=0, push_photons=0, seed=4,
                         f_photon=f, f_every=every)
        ids = st[0].view()["id"].copy()
        nev = [st[0].view()["n_events"].astype(np.int64)]
        kids = []
        seen = 0
        for n in range(12):
            orc.run(st, fld, par, 1, first_step=n)
            v = st[0].view()
            assert np.array_equal(v["id"], ids)
            nev.append(v["n_events"].astype(np.int64))
            g = st[2].view()
            kids.append(_children_of(ids, g["parent"][seen:]))
            seen = len(g["id"])
        out[every] = (st, np.array(nev), np.array(kids))
    return out


def test_deterministic_parents_evolve_as_without_the_factor(every_runs):
    a, b = every_runs[0][0][0].view(), every_runs[1][0][0].view()
    for c in a:
        assert np.array_equal(a[c], b[c]), c
    ga, gb = _by_id(every_runs[0][0][2].view()), _by_id(every_runs[1][0][2].view())
    pos = np.searchsorted(ga["id"], gb["id"])
    assert np.array_equal(ga["id"][pos], gb["id"])
    for c in ("x", "y", "z", "px", "py", "pz", "parent", "birth"):
        assert np.array_equal(ga[c][pos], gb[c]), c
    assert np.array_equal(gb["w"], 4.0 * ga["w"][pos])


def test_deterministic_every_fourth_event_with_one_phase(every_runs):
    _, nev, kids = every_runs[1]
    F = 4
    ev = nev[1:] - nev[:-1]  # events per step and electron
    total = nev[-1] - nev[0]
    made = kids.sum(0)
    assert total.sum() > 10_000
    assert np.all((made == total // F) | (made == -(-total // F)))
    # one phase per electron explains every step: children at step s are the event
    # numbers e in [nev_s, nev_s+1) with (e + phi) mod F == 0
    fits = np.zeros((F, len(made)), bool)
    for phi in range(F):
        ok = np.ones(len(made), bool)
        for s in range(ev.shape[0]):
            lo, hi = nev[s], nev[s + 1]
            want = (hi + phi + F - 1) // F - (lo + phi + F - 1) // F  # multiples in range
            ok &= kids[s] == want
        fits[phi] = ok
    assert np.all(fits.any(0))
    # where the counts leave one phase, the phases are uniform over 0..F-1
    unique = fits.sum(0) == 1
    cnt = np.bincount(np.argmax(fits[:, unique], 0), minlength=F)
    m = cnt.sum()
    assert m > 1000
    assert np.all(np.abs(cnt - m / F) < 5 * math.sqrt(m / F))


def test_deterministic_factor_is_unbiased(every_runs):
    _, nev, kids = every_runs[1]
    total = (nev[-1] - nev[0]).astype(float)
    made = kids.sum(0).astype(float)
    # E[made] = total / F for every electron: the deviations average out
    dev = made - total / 4.0
    assert abs(dev.mean()) < 5 * math.sqrt(0.25 / len(dev))


def test_deterministic_pairs_with_probability_one_over_f(orc):
    cols = _photons(seed=7)
    a, sa = _pair_step(orc, cols)
    b, sb = _pair_step(orc, cols, f_pair=3.0, f_every=1)
    pa, pb = a[2].view(), b[2].view()
    assert np.array_equal(pa["id"] == DEAD, pb["id"] == DEAD)  # the same photons decay
    events = int((pa["id"] == DEAD).sum())
    va, vb = _by_id(a[0].view()), _by_id(b[0].view())
    pos = np.searchsorted(va["id"], vb["id"])
    assert np.array_equal(va["id"][pos], vb["id"])
    assert np.array_equal(vb["w"], 3.0 * va["w"][pos])
    m, q = sb["pairs"], 1.0 / 3.0
    assert abs(m - events * q) < 4.0 * math.sqrt(events * q * (1 - q))


def test_forms_that_do_not_combine_are_refused(orc):
    cols = _photons(n=100)
    for kw in (dict(f_pair=2.0, runs_pair=2), dict(f_pair=2.5, f_every=1),
               dict(runs_pair=65)):
        with pytest.raises(RuntimeError):
            _pair_step(orc, cols, **kw)
    with pytest.raises(RuntimeError):
        _electrons(orc, n=100, f_photon=3.0, runs_photon=3)


def test_one_run_is_the_ordinary_generator(orc):
    a, out_a, _ = _electrons(orc, n=2000, steps=3)
    b, out_b, _ = _electrons(orc, n=2000, steps=3, runs_photon=1, runs_pair=0)
    for s1, s2 in zip(a, b):
        v1, v2 = s1.view(), s2.view()
        for c in v1:
            assert np.array_equal(v1[c], v2[c]), c
