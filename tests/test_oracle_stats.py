"""Pins of the oracle's per-step record and of its sub-step refinement, against what the
stores themselves hold and against rates recomputed from the oracle's own scalar functions:
the photon-energy histogram and the radiated energy against the emitted photons, the live
and advanced counts against the store counts, the largest pair probability against the
probabilities of the pairs that were made, and the refinement of Sec. IV.H's sub-steps for a
lepton the field slows down within the step."""
import math

import numpy as np

from paper_1412_6426_amd import workloads as W

ALPHA = 7.2973525693e-3
EPS_R = W.eps_r_for_wavelength(0.8e-6)
DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)


def _stores(orc, init, caps):
    st = [orc.Store(caps[0]), orc.Store(caps[1]), orc.Store(caps[2], with_events=False)]
    for s, cols in zip(st, init):
        s.load(cols)
    return st


def test_photon_histogram_and_energy_match_the_emitted_photons(orc):
    """Uniform B, emission only, photons recorded where they are born and not advanced: each
    photon's |k| is its energy, so the steps' histograms add up to the histogram of the photon
    store (bin floor(10 (log10 eps + 8))), the radiated energy to sum w |k|, and the counts
    to the store's."""
    w = W.uniform_b(n=300, steps=6)
    st = _stores(orc, W.uniform_b_initial(w), w.capacity)
    fld = orc.Field(kind=orc.FIELD_UNIFORM, b0=w.field.b0)
    par = orc.Params(dt=w.dt, eps_r=w.eps_r, pairs=0, push_photons=0, seed=5)
    out = []
    for n in range(w.n_steps):
        before = [s.count for s in st]
        par.step = n
        out.append(orc.step(st, fld, par))
        assert out[-1]["n_start"] == before
        assert out[-1]["advanced"] == [300, 0, 0]  # photons are neither pushed nor decayed
        assert out[-1]["emitted"] == st[2].count - before[2]
    g = st[2].view()
    eps = np.sqrt(g["px"] ** 2 + g["py"] ** 2 + g["pz"] ** 2)
    assert len(eps) > 500
    bins = np.floor(10.0 * (np.log10(eps) + 8.0)).astype(int)
    want = np.bincount(bins[(bins >= 0) & (bins < 130)], minlength=130)
    got = np.sum([s["photon_hist"] for s in out], axis=0)
    assert np.array_equal(got, want)
    assert sum(s["photon_energy"] for s in out) == \
        __import__("pytest").approx(float((g["w"] * eps).sum()), rel=1e-12)


def test_largest_pair_probability_is_that_of_a_pair_made(orc):
    """Photons of random energy and direction in a uniform field strong enough for pairs,
    one step: every pair's probability is recomputed from its children (r1 = |p_e| / |k|,
    k = p_e + p_e+) with the oracle's rate and sub-step functions; the record's largest pair
    probability is the largest of these, and lies below the largest over all the step's
    decisions (recomputed from the photons' own draws)."""
    rng = np.random.default_rng(7)
    n = 4000
    kdir = rng.normal(size=(3, n))
    kdir /= np.linalg.norm(kdir, axis=0)
    kabs = 10.0 ** rng.uniform(1.0, 3.5, n)
    k = kdir * kabs
    zero = np.zeros(n)
    cols = W._seed_columns(zero, zero, zero, k[0], k[1], k[2], first_id=1000)
    init = [W.empty_columns(), W.empty_columns(), cols]
    E0, B0, dt = (0.3, 0.0, 0.0), (0.0, 0.2, 0.1), 500.0
    st = _stores(orc, init, (20000, 20000, 20000))
    fld = orc.Field(kind=orc.FIELD_UNIFORM, e0=E0, b0=B0)
    par = orc.Params(dt=dt, eps_r=1.0, emission=0, seed=11)
    s0 = orc.step(st, fld, par)
    assert s0["n_start"] == [0, 0, n] and s0["advanced"] == [0, 0, n]
    e, p = st[0].view(), st[1].view()
    assert s0["pairs"] == len(e["id"]) == len(p["id"]) > 100
    P = []
    for i in range(len(e["id"])):
        kk = np.array([e["px"][i] + p["px"][i], e["py"][i] + p["py"][i],
                       e["pz"][i] + p["pz"][i]])
        ka = float(np.linalg.norm(kk))
        r1 = float(np.linalg.norm([e["px"][i], e["py"][i], e["pz"][i]])) / ka
        chi = orc.chi_photon(kk, E0, B0, 1.0)
        nsub = orc.substeps(dt, orc.dtq_photon(chi, ka, 1.0))[0]
        P.append(orc.rate_pair(r1, chi, ka, dt / nsub * ALPHA))
    assert s0["max_p_pair"] == __import__("pytest").approx(max(P), rel=1e-12)
    # every decision of the step (sub-step 0 of each photon, from its own draw)
    Pall = []
    for i in range(n):
        ka = float(kabs[i])
        chi = orc.chi_photon(k[:, i], E0, B0, 1.0)
        nsub = orc.substeps(dt, orc.dtq_photon(chi, ka, 1.0))[0]
        o = orc.philox((0, 0, 11, 0), (1000 + i, 0))
        Pall.append(orc.rate_pair(orc.uniform(o[0], o[1]), chi, ka, dt / nsub * ALPHA))
    assert max(Pall) > max(P) * 1.01
    # next step: the removed photons keep their slots and are not advanced
    par.step = 1
    s1 = orc.step(st, fld, par)
    assert s1["n_start"] == [s0["pairs"], s0["pairs"], n]
    assert s1["advanced"] == [s0["pairs"], s0["pairs"], n - s0["pairs"]]


def test_slowed_leptons_refine_their_substeps(orc):
    """Positrons moving against a uniform E (a0 = 1000 at 0.8 um, dt = T/200) with |p| = 30
    m c < |E| dt = 31.4 m c: at the step start they need one sub-step (H_eff = |E| / gamma),
    but the field stops them within it, where H_eff = |E| and Eq. (29) asks for three.  The
    step refines their sub-steps, so no emission probability reaches 1, and the refinement
    takes exactly dt in all: a positron that emitted nothing ends at p = p0 + |E| dt."""
    n = 3000
    a0 = 1000.0
    dt = 2.0 * math.pi / 200.0
    zero = np.zeros(n)
    cols = W._seed_columns(zero, zero, zero, np.full(n, -30.0), zero, zero)
    init = [W.empty_columns(), cols, W.empty_columns()]
    st = _stores(orc, init, (10, 10 * n, 10 * n))
    fld = orc.Field(kind=orc.FIELD_UNIFORM, e0=(a0, 0.0, 0.0))
    par = orc.Params(dt=dt, eps_r=EPS_R, pairs=0, push_photons=0, seed=2)
    s = orc.step(st, fld, par)
    assert s["nsub_hist"][1] == n
    assert s["nsub_refined"] >= n
    assert s["saturated"] == 0 and s["max_p_emit"] < 1.0
    assert s["emitted"] > 100
    v = st[1].view()
    quiet = v["n_events"] == 0
    assert quiet.sum() > 100
    np.testing.assert_allclose(v["px"][quiet], -30.0 + a0 * dt, rtol=0, atol=1e-12)
    assert np.all(v["py"] == 0.0) and np.all(v["pz"] == 0.0)
