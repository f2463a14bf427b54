"""Pins of the oracle's thinning by global even redistribution (Sec. VI).

What the method fixes: the total statistical weight of a store is unchanged (the removed
weight f_r goes to the survivors by the factor sum f / (sum f - f_r)); survivors are a
subset of the particles with every other column untouched; each live particle survives
independently with probability target / live, whatever its weight; nothing happens at or
below the trigger; removed photons (dead ids) neither count as live nor survive."""
import math

import numpy as np
import pytest

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)


def _store(orc, n, seed, dead_every=0, photon=False):
    rng = np.random.default_rng(seed)
    cols = {c: rng.normal(size=n) for c in ("x", "y", "z", "px", "py", "pz")}
    cols["w"] = rng.uniform(0.5, 2.0, n)
    cols["id"] = (np.arange(n, dtype=np.uint64) * np.uint64(2654435761)) | np.uint64(1 << 63)
    if dead_every:
        cols["id"][::dead_every] = DEAD
    cols["parent"] = rng.integers(0, 1 << 62, n, dtype=np.int64).astype(np.uint64)
    cols["birth"] = rng.integers(0, 1 << 20, n, dtype=np.int64).astype(np.uint32)
    if not photon:
        cols["n_events"] = rng.integers(0, 9, n, dtype=np.int64).astype(np.uint32)
    st = orc.Store(n, with_events=not photon)
    st.load(cols)
    return st, cols


def test_weight_conserved_and_survivors_untouched(orc):
    st, cols = _store(orc, 20_000, 1)
    rec = orc.thin(st, trigger=10_000, target=5_000, seed=11, step=42)
    assert rec["thinned"] and rec["live_before"] == 20_000
    assert rec["weight_after"] == pytest.approx(rec["weight_before"], rel=1e-12)
    v = st.view()
    assert len(v["id"]) == rec["kept"]
    pos = {int(i): k for k, i in enumerate(cols["id"])}
    idx = np.array([pos[int(i)] for i in v["id"]])
    assert np.all(np.diff(idx) > 0)  # a subset, in the original order
    for c in ("x", "y", "z", "px", "py", "pz", "parent", "birth", "n_events"):
        assert np.array_equal(v[c], cols[c][idx]), c
    np.testing.assert_allclose(v["w"], cols["w"][idx] * rec["factor"], rtol=1e-15)
    # factor = sum f / (sum f - f_r)
    f_r = cols["w"].sum() - cols["w"][idx].sum()
    assert rec["factor"] == pytest.approx(cols["w"].sum() / (cols["w"].sum() - f_r), rel=1e-12)


@pytest.mark.parametrize("q", [0.1, 0.5, 0.9])
def test_survival_is_binomial_and_blind_to_weight(orc, q):
    n = 100_000
    st, cols = _store(orc, n, 2)
    target = int(q * n)
    rec = orc.thin(st, trigger=0, target=target, seed=3, step=1)
    p = target / n
    assert abs(rec["kept"] - n * p) < 4.0 * math.sqrt(n * p * (1 - p))
    # the survivors' weights before the rescale have the population's mean
    v = st.view()
    w0 = v["w"] / rec["factor"]
    se = cols["w"].std() / math.sqrt(len(w0))
    assert abs(w0.mean() - cols["w"].mean()) < 4.0 * se


def test_draws_are_independent_across_steps(orc):
    n = 50_000
    a, _ = _store(orc, n, 4)
    b, _ = _store(orc, n, 4)
    orc.thin(a, trigger=0, target=n // 2, seed=9, step=10)
    orc.thin(b, trigger=0, target=n // 2, seed=9, step=11)
    ia, ib = set(a.view()["id"].tolist()), set(b.view()["id"].tolist())
    both = len(ia & ib)
    # independent halves overlap in about a quarter of the particles
    assert abs(both - n / 4) < 4.0 * math.sqrt(n * 0.25 * 0.75)
    c, _ = _store(orc, n, 4)
    orc.thin(c, trigger=0, target=n // 2, seed=9, step=10)
    assert set(c.view()["id"].tolist()) == ia  # same key, same survivors


def test_no_change_at_or_below_trigger(orc):
    st, cols = _store(orc, 1000, 5)
    for trig, tgt in ((1000, 10), (5000, 10)):  # not examined
        rec = orc.thin(st, trigger=trig, target=tgt, seed=1, step=1)
        assert not rec["thinned"] and rec["live_before"] == 0 and rec["factor"] == 1.0
    rec = orc.thin(st, trigger=10, target=2000, seed=1, step=1)  # examined, target above live
    assert not rec["thinned"] and rec["live_before"] == rec["kept"] == 1000
    assert rec["factor"] == 1.0
    v = st.view()
    for c in cols:
        assert np.array_equal(v[c], cols[c])


def test_dead_photons_are_not_live_and_do_not_survive(orc):
    n = 30_000
    st, cols = _store(orc, n, 6, dead_every=3, photon=True)
    live = int((cols["id"] != DEAD).sum())
    w_live = cols["w"][cols["id"] != DEAD].sum()
    rec = orc.thin(st, trigger=live - 1, target=live // 2, seed=2, step=7)
    assert rec["live_before"] == live
    assert rec["weight_before"] == pytest.approx(w_live, rel=1e-12)
    v = st.view()
    assert not np.any(v["id"] == DEAD)
    assert v["w"].sum() == pytest.approx(w_live, rel=1e-12)
