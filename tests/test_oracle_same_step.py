"""Pins of the oracle's same-step processing of children (Sec. IV.H: the adaptive generator
accounts for several events within one iteration; Sec. VII checks that large and small time
steps give the same cascade).

A child born at sub-step k of a parent advanced through T in n_sub sub-steps has
tau = (n_sub - k - 1) T / n_sub of the step left; it is advanced through tau with the
parent's frozen fields and its own sub-steps, and its own children likewise, up to G
generations.  What fixes the result, and what these tests check:
* with one sub-step per particle every child is born at the end of the step (tau = 0), so
  nothing changes;
* a photon child moves exactly tau along its k in its birth step;
* a lepton child in a pure magnetic field turns through the Boris angle of its sub-steps
  over tau, in the sense its charge gives, with |p| unchanged;
* generations: children of generation G + 1 are counted as deferred, and advancing one more
  generation advances exactly those;
* the shower cascade of Sec. VII (gamma_0 = 2e5 electrons across H_0 = 0.2 E_S): particle
  counts above 1e-3 of the initial energy at a time step of 400 single-sub-step intervals
  agree with one sub-step per interval, and differ when children wait for the next step."""
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


def _by_id(v):
    o = np.argsort(v["id"])
    return {k: a[o] for k, a in v.items()}


def test_one_substep_means_nothing_is_left_of_the_step(orc):
    w = W.rotating_e(n=300, periods=0.5, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=2)
    fld = orc.Field(kind=orc.FIELD_ROTATING_E, amp=w.field.amp)
    runs = []
    for G in (0, 4):
        st = _stores(orc, init, w.capacity)
        par = orc.Params(dt=w.dt, eps_r=w.eps_r, seed=7, forced_substeps=1,
                         same_step_generations=G)
        out = orc.run(st, fld, par, w.n_steps)
        runs.append((st, out))
    (a, oa), (b, ob) = runs
    assert sum(s["emitted"] for s in oa) > 1000
    assert sum(s["children_advanced"] for s in ob) == 0
    for s1, s2 in zip(a, b):
        v1, v2 = s1.view(), s2.view()
        for c in v1:
            assert np.array_equal(v1[c], v2[c]), c


def test_photon_children_move_through_the_rest_of_the_step(orc):
    """Uniform B with chi = 1: every electron takes 8 sub-steps of dt / 8.  A photon born at
    sub-step k ends the step tau = (7 - k) dt / 8 further along its k than where it was
    born (its position without same-step processing)."""
    w = W.uniform_b(n=4000, steps=1)
    init = W.uniform_b_initial(w)
    fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=w.field.b0)
    runs = []
    for G in (0, 1):
        st = _stores(orc, init, w.capacity)
        par = orc.Params(dt=w.dt, eps_r=w.eps_r, pairs=0, push_photons=1, seed=4,
                         same_step_generations=G)
        out = orc.run(st, fld, par, 1)
        runs.append((st, out[0]))
    (a, sa), (b, sb) = runs
    # the parents do not see it
    va, vb = a[0].view(), b[0].view()
    for c in va:
        assert np.array_equal(va[c], vb[c]), c
    ga, gb = _by_id(a[2].view()), _by_id(b[2].view())
    assert np.array_equal(ga["id"], gb["id"]) and len(ga["id"]) > 1000
    k = (ga["birth"] & 0x3FFF).astype(np.float64)
    assert k.max() == 7
    tau = (8.0 - k - 1.0) * (w.dt / 8.0)
    kv = np.stack([ga["px"], ga["py"], ga["pz"]], 1)
    khat = kv / np.linalg.norm(kv, axis=1, keepdims=True)
    moved = np.stack([gb["x"] - ga["x"], gb["y"] - ga["y"], gb["z"] - ga["z"]], 1)
    np.testing.assert_allclose(moved, tau[:, None] * khat, rtol=0, atol=1e-12 * w.dt)
    for c in ("px", "py", "pz", "w", "parent", "birth"):
        assert np.array_equal(ga[c], gb[c]), c
    # every photon born before the last sub-step was advanced
    assert sb["children_advanced"] == int((k < 7).sum())
    assert sb["deferred"] == 0  # photons without pairs have no children


def _photon_state(n=20_000, k=1000.0, seed=1):
    rng = np.random.default_rng(seed)
    zero = np.zeros(n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    return W._seed_columns(zero, zero, zero, k * np.cos(phi), k * np.sin(phi), zero)


def test_pair_leptons_turn_through_the_rest_of_the_step(orc):
    """Photons (k = 1000 across B = 0.002 E_S, chi_gamma = 2) decay over one step of four
    forced sub-steps; emission off.  A lepton born at sub-step k turns in its birth step
    through 4 Boris rotations of h = tau / 4, tau = (3 - k) dt / 4, each by
    2 atan(B h / (2 gamma)): counter-clockwise about B for the electron, clockwise for the
    positron, |p| unchanged."""
    B, dt = 0.002, 3e5
    cols = _photon_state()
    runs = []
    for G in (0, 1):
        st = [orc.Store(80_000), orc.Store(80_000), orc.Store(20_000, with_events=False)]
        st[0].load(W.empty_columns())
        st[1].load(W.empty_columns())
        st[2].load(cols)
        fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=(0, 0, B))
        par = orc.Params(dt=dt, eps_r=1.0, seed=3, emission=0, forced_substeps=4,
                         same_step_generations=G)
        out = orc.run(st, fld, par, 1)
        runs.append((st, out[0]))
    (a, sa), (b, sb) = runs
    assert sa["pairs"] == sb["pairs"] > 1000
    for sp, sense in ((0, 1.0), (1, -1.0)):
        va, vb = _by_id(a[sp].view()), _by_id(b[sp].view())
        assert np.array_equal(va["id"], vb["id"])
        pa = np.stack([va["px"], va["py"]], 1)
        pb = np.stack([vb["px"], vb["py"]], 1)
        na, nb = np.linalg.norm(pa, axis=1), np.linalg.norm(pb, axis=1)
        np.testing.assert_allclose(nb, na, rtol=1e-12)
        assert np.all(vb["pz"] == 0.0)
        k = (va["birth"] & 0x3FFF).astype(np.float64)
        tau = (4.0 - k - 1.0) * (dt / 4.0)
        gam = np.sqrt(1.0 + na * na)
        want = 4.0 * 2.0 * np.arctan(B * (tau / 4.0) / (2.0 * gam))
        got = np.arctan2(pa[:, 0] * pb[:, 1] - pa[:, 1] * pb[:, 0],
                         (pa * pb).sum(1))
        # slow leptons turn by more than pi: compare modulo 2 pi
        diff = np.angle(np.exp(1j * (got - sense * want)))
        np.testing.assert_allclose(diff, 0.0, rtol=0, atol=1e-10)
        assert np.any(want > 0.01)  # turned by a visible angle
    assert sb["children_advanced"] == 2 * int(((a[0].view()["birth"] & 0x3FFF) < 3).sum())


def test_each_generation_advances_what_the_last_one_deferred(orc):
    """One large step of the shower below, from the state after a first one: G = 1 leaves
    grandchildren with time left for the next step (deferred); G = 2 advances exactly those
    as well, and so on, until nothing is deferred."""
    zero = np.zeros(50)
    cols = W._seed_columns(zero, zero, zero, np.full(50, math.sqrt(G0 * G0 - 1)), zero, zero)
    caps = (100_000, 100_000, 2_000_000)
    st = _stores(orc, [cols, W.empty_columns(), W.empty_columns()], caps)
    fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=(0, 0, B0))
    orc.run(st, fld, orc.Params(dt=LARGE_DT, eps_r=1.0, seed=5, kappa=0.25,
                                same_step_generations=64), 1)
    state = [s.view() for s in st]
    got = {}
    for G in (1, 2, 3, 64):
        s2 = _stores(orc, state, caps)
        par = orc.Params(dt=LARGE_DT, eps_r=1.0, seed=5, kappa=0.25, same_step_generations=G)
        got[G] = orc.run(s2, fld, par, 1, first_step=1)[0]
    assert got[1]["deferred"] > 0 and got[2]["deferred"] > 0
    for G in (1, 2):
        assert got[G + 1]["children_advanced"] == got[G]["children_advanced"] + got[G]["deferred"]
    assert got[64]["deferred"] == 0


G0, B0 = 2e5, 0.2  # Sec. VII cascade development: gamma_0, H_0 / E_S
LARGE_DT = 25_000.0


def _shower(orc, dt, steps_per_sample, G, kappa, seed, n_seed=50, samples=3):
    zero = np.zeros(n_seed)
    cols = W._seed_columns(zero, zero, zero, np.full(n_seed, math.sqrt(G0 * G0 - 1)), zero, zero)
    st = _stores(orc, [cols, W.empty_columns(), W.empty_columns()],
                 (2000 * n_seed, 2000 * n_seed, 40_000 * n_seed))
    fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=(0, 0, B0))
    par = orc.Params(dt=dt, eps_r=1.0, seed=seed, same_step_generations=G, kappa=kappa)
    thr = 1e-3 * G0
    out, n = [], 0
    for _ in range(samples):
        r = orc.run(st, fld, par, steps_per_sample, first_step=n)
        assert all(s["dropped"] == 0 for s in r)
        n += steps_per_sample
        e, p, g = (s.view() for s in st)
        live = g["id"] != DEAD
        out.append([int((np.sqrt(1 + e["px"] ** 2 + e["py"] ** 2) > thr).sum()),
                    int((np.sqrt(1 + p["px"] ** 2 + p["py"] ** 2) > thr).sum()),
                    int((np.hypot(g["px"], g["py"])[live] > thr).sum())])
    return np.array(out, dtype=np.float64)


def test_shower_cascade_is_invariant_to_the_time_step(orc):
    """Eight batches of 50 seeds, counts of e-, e+ and photons above 200 m c^2 at t = 25k,
    50k and 75k hbar / m c^2 (t_rad = 9.0e4).  Reference: dt = 62.5, every particle one
    sub-step (so children have nothing left of their step).  Large: dt = 25k, about 400
    lepton sub-steps a step at kappa = 0.25 (per-sub-step probabilities stay below 0.25; at
    kappa = 1 they approach 1 and single-event sub-steps undercount hard photons).  With
    children advanced in their birth step the two agree within 4 standard errors; with
    children left for the next step the large step lags by far more."""
    batches = range(8)
    ref = np.array([_shower(orc, 62.5, 400, 0, 1.0, 100 + b) for b in batches])
    big = np.array([_shower(orc, LARGE_DT, 1, 64, 0.25, 100 + b) for b in batches])
    lag = np.array([_shower(orc, LARGE_DT, 1, 0, 0.25, 100 + b) for b in batches])

    def z(x):
        se = np.sqrt(x.var(0, ddof=1) / len(x) + ref.var(0, ddof=1) / len(ref))
        return (x.mean(0) - ref.mean(0)) / se

    assert ref.mean(0)[-1].min() > 150  # a developed cascade
    assert np.abs(z(big)).max() < 4.0, z(big)
    assert np.abs(z(lag)).max() > 8.0, z(lag)
