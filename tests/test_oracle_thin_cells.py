"""Pins of the oracle's thinning per cell (Sec. VI's redistribution applied within each block
of grid cells; Sec. VII's thinning that caps how many particles a cell holds).

What the method fixes: every group keeps its statistical weight (the removed weight goes to
the group's survivors by sum f / (sum f - f_r)); a group at or below the cap is untouched;
in a larger group each particle survives independently with probability cap / n, whatever
its weight, and at least one survives; survivors are a subset of the particles with every
other column untouched; removed photons go.  The groups here are cells of a grid small
enough that a block is one cell, and are recomputed on the host from the positions."""
import math

import numpy as np
import pytest

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)
N_GRID = (16, 8, 4)
DX = (0.5, 0.25, 1.0)
ORIGIN = (-4.0, -1.0, -2.0)


def _cells(cols):
    """Cell index per particle (x fastest), -1 for a non-finite coordinate."""
    idx = np.zeros(len(cols["x"]), dtype=np.int64)
    ok = np.ones(len(cols["x"]), dtype=bool)
    mul = 1
    for d, c in enumerate(("x", "y", "z")):
        with np.errstate(invalid="ignore"):
            fl = np.floor((cols[c] - ORIGIN[d]) / DX[d])
        good = np.isfinite(fl)
        ok &= good
        i = np.zeros(len(fl), dtype=np.int64)
        i[good] = np.mod(fl[good].astype(np.int64), N_GRID[d])
        idx += mul * i
        mul *= N_GRID[d]
    return np.where(ok, idx, -1)


def _store(orc, n, seed, spread=1.0, photon=False, dead_every=0, nonfinite=0):
    rng = np.random.default_rng(seed)
    span = np.array(N_GRID) * np.array(DX)
    cols = {}
    for d, c in enumerate(("x", "y", "z")):
        # concentrated near one corner so that cells hold very different counts, with some
        # positions outside the box (periodic wrap)
        cols[c] = ORIGIN[d] + span[d] * rng.beta(1.0, 3.0, n) * spread
        cols[c][rng.random(n) < 0.05] += span[d] * rng.integers(-2, 3)
    for c in ("px", "py", "pz"):
        cols[c] = rng.normal(size=n)
    cols["w"] = rng.uniform(0.5, 2.0, n)
    cols["id"] = (np.arange(n, dtype=np.uint64) * np.uint64(2654435761)) | np.uint64(1 << 63)
    if dead_every:
        cols["id"][::dead_every] = DEAD
    if nonfinite:
        cols["y"][1:nonfinite * 7:7] = np.nan
    cols["parent"] = rng.integers(0, 1 << 62, n, dtype=np.int64).astype(np.uint64)
    cols["birth"] = rng.integers(0, 1 << 20, n, dtype=np.int64).astype(np.uint32)
    if not photon:
        cols["n_events"] = rng.integers(0, 9, n, dtype=np.int64).astype(np.uint32)
    st = orc.Store(n, with_events=not photon)
    st.load(cols)
    return st, cols


def _thin(orc, st, cap, photon=False, seed=5, step=9):
    return orc.thin_cells(st, photon, N_GRID, DX, ORIGIN, cap, seed, step)


def test_groups_keep_their_weight_and_small_groups_are_untouched(orc):
    st, cols = _store(orc, 30_000, 1)
    cap = 40
    rec = _thin(orc, st, cap)
    v = st.view()
    cell_in = _cells(cols)
    pos = {int(i): k for k, i in enumerate(cols["id"])}
    src = np.array([pos[int(i)] for i in v["id"]])
    assert len(np.unique(src)) == len(src) == rec["kept"]
    # every column but the weight is the input's
    for c in ("x", "y", "z", "px", "py", "pz", "parent", "birth", "n_events"):
        assert np.array_equal(v[c], cols[c][src], equal_nan=True), c
    groups = np.unique(cell_in)
    assert rec["groups"] == len(groups)
    thinned = 0
    for g in groups:
        members = np.flatnonzero(cell_in == g)
        kept = src[cell_in[src] == g]
        w_in = cols["w"][members].sum()
        w_out = v["w"][cell_in[src] == g].sum()
        assert w_out == pytest.approx(w_in, rel=1e-12), g
        assert len(kept) >= 1
        if len(members) <= cap:
            assert np.array_equal(np.sort(kept), members)
            assert np.array_equal(v["w"][cell_in[src] == g], cols["w"][kept])
        else:
            thinned += 1
            # one factor per group, W / K
            ratio = v["w"][cell_in[src] == g] / cols["w"][kept]
            assert np.allclose(ratio, ratio[0], rtol=1e-14, atol=0)
    assert thinned == rec["groups_thinned"] > 10
    assert rec["weight_after"] == pytest.approx(rec["weight_before"], rel=1e-12)
    assert rec["weight_before"] == pytest.approx(cols["w"].sum(), rel=1e-12)


def test_survivors_come_in_cell_order_then_store_order(orc):
    st, cols = _store(orc, 10_000, 2, nonfinite=20)
    _thin(orc, st, 15)
    v = st.view()
    cells = _cells(v)
    key = np.where(cells < 0, np.iinfo(np.int64).max, cells)  # non-finite group last
    assert np.all(np.diff(key) >= 0)
    pos = {int(i): k for k, i in enumerate(cols["id"])}
    src = np.array([pos[int(i)] for i in v["id"]])
    same = np.diff(key) == 0
    assert np.all(np.diff(src)[same] > 0)
    assert np.count_nonzero(cells < 0) >= 1  # the non-finite ones form a group of their own


def test_survival_is_binomial_and_blind_to_weight(orc):
    """Cells of at least 400 particles with cap 20: kept counts average 20 with the binomial spread,
    and survival does not depend on the particle's weight."""
    kept, frac_heavy, frac_light = [], [], []
    for seed in range(6):
        st, cols = _store(orc, 40_000, 100 + seed, spread=0.3)  # tens of crowded cells
        cells_in = _cells(cols)
        _thin(orc, st, 20, seed=seed, step=3)
        v = st.view()
        pos = {int(i): k for k, i in enumerate(cols["id"])}
        src = np.array([pos[int(i)] for i in v["id"]])
        for g in np.unique(cells_in):
            m = np.count_nonzero(cells_in == g)
            if m < 400:
                continue
            k = np.count_nonzero(cells_in[src] == g)
            kept.append((k - 20) / math.sqrt(20 * (1 - 20 / m)))
        heavy = cols["w"] > 1.25
        surv = np.zeros(len(cols["w"]), bool)
        surv[src] = True
        crowded = np.isin(cells_in, [g for g in np.unique(cells_in)
                                     if np.count_nonzero(cells_in == g) >= 400])
        frac_heavy.append(surv[crowded & heavy].mean())
        frac_light.append(surv[crowded & ~heavy].mean())
    z = np.array(kept)
    assert len(z) >= 10
    assert abs(z.mean()) < 4.0 / math.sqrt(len(z))
    assert 0.5 < z.std() < 1.6
    assert abs(np.mean(frac_heavy) - np.mean(frac_light)) < 0.1 * np.mean(frac_light)


def test_survivors_are_the_draws_below_the_cap(orc):
    """Brute force on one crowded cell: the survivors are the particles whose Philox draw,
    keyed by the id with counter (step, 11 << 16, seed lo, seed hi), is below cap / n."""
    n, cap, seed, step = 500, 37, 0x1234_5678_9ABC, 77
    rng = np.random.default_rng(9)
    cols = {"x": np.full(n, 0.1), "y": np.full(n, 0.1), "z": np.full(n, 0.1)}
    for c in ("px", "py", "pz"):
        cols[c] = rng.normal(size=n)
    cols["w"] = rng.uniform(0.5, 2.0, n)
    cols["id"] = rng.integers(1, 1 << 62, n, dtype=np.int64).astype(np.uint64)
    cols["parent"] = np.zeros(n, np.uint64)
    cols["birth"] = np.zeros(n, np.uint32)
    cols["n_events"] = np.zeros(n, np.uint32)
    st = orc.Store(n)
    st.load(cols)
    rec = orc.thin_cells(st, False, N_GRID, DX, ORIGIN, cap, seed, step)
    q = cap / n
    want = []
    for i in range(n):
        idv = int(cols["id"][i])
        o = orc.philox([step, 11 << 16, seed & 0xFFFFFFFF, seed >> 32],
                       [idv & 0xFFFFFFFF, idv >> 32])
        if orc.uniform(o[0], o[1]) < q:
            want.append(idv)
    got = st.view()["id"]
    assert [int(i) for i in got] == want  # in store order
    w_in = cols["w"].sum()
    w_kept = sum(float(cols["w"][i]) for i in range(n) if int(cols["id"][i]) in set(want))
    assert np.allclose(st.view()["w"],
                       [cols["w"][list(cols["id"]).index(i)] * (w_in / w_kept) for i in got],
                       rtol=1e-15, atol=0)
    assert rec["groups"] == 1 and rec["groups_thinned"] == 1


def test_a_group_that_draws_no_survivor_keeps_its_smallest_draw(orc):
    """Cap 1 on cells of 2 to 6 particles: no draw falls below q in about a third of them,
    and then the particle with the smallest draw survives with the whole weight."""
    n_cells, seen_empty = 400, 0
    rng = np.random.default_rng(4)
    xs, ids = [], []
    for c in range(n_cells):
        m = 2 + c % 5
        cx = ORIGIN[0] + (c % N_GRID[0] + 0.5) * DX[0]
        cy = ORIGIN[1] + ((c // N_GRID[0]) % N_GRID[1] + 0.5) * DX[1]
        cz = ORIGIN[2] + ((c // (N_GRID[0] * N_GRID[1])) % N_GRID[2] + 0.5) * DX[2]
        xs += [(cx, cy, cz)] * m
    n = len(xs)
    cols = {"x": np.array([p[0] for p in xs]), "y": np.array([p[1] for p in xs]),
            "z": np.array([p[2] for p in xs])}
    for c in ("px", "py", "pz"):
        cols[c] = rng.normal(size=n)
    cols["w"] = rng.uniform(0.5, 2.0, n)
    cols["id"] = np.arange(1, n + 1, dtype=np.uint64)
    cols["parent"] = np.zeros(n, np.uint64)
    cols["birth"] = np.zeros(n, np.uint32)
    cols["n_events"] = np.zeros(n, np.uint32)
    st = orc.Store(n)
    st.load(cols)
    orc.thin_cells(st, False, N_GRID, DX, ORIGIN, 1, 3, 1)
    v = st.view()
    cells_in = _cells(cols)
    cells_out = _cells(v)
    for g in np.unique(cells_in):
        members = np.flatnonzero(cells_in == g)
        out = np.flatnonzero(cells_out == g)
        assert len(out) >= 1
        assert v["w"][out].sum() == pytest.approx(cols["w"][members].sum(), rel=1e-13)
        u = []
        for i in members:
            o = orc.philox([1, 11 << 16, 3, 0], [int(cols["id"][i]), 0])
            u.append(orc.uniform(o[0], o[1]))
        u = np.array(u)
        if not np.any(u < 1.0 / len(members)):
            seen_empty += 1
            assert len(out) == 1 and int(v["id"][out[0]]) == int(cols["id"][members[np.argmin(u)]])
    assert seen_empty > 50


def test_removed_photons_go_and_nothing_else_changes_below_the_cap(orc):
    st, cols = _store(orc, 5_000, 3, photon=True, dead_every=7)
    rec = _thin(orc, st, 10**9, photon=True)
    live = cols["id"] != DEAD
    assert rec["live_before"] == rec["kept"] == int(live.sum())
    assert rec["groups_thinned"] == 0 and not rec["thinned"]
    v = st.view()
    assert np.all(v["id"] != DEAD)
    assert sorted(int(i) for i in v["id"]) == sorted(int(i) for i in cols["id"][live])
    assert rec["weight_before"] == pytest.approx(cols["w"][live].sum(), rel=1e-12)


def test_deterministic_and_keyed_by_step(orc):
    a, _ = _store(orc, 8_000, 6)
    b, _ = _store(orc, 8_000, 6)
    c, _ = _store(orc, 8_000, 6)
    _thin(orc, a, 12, step=4)
    _thin(orc, b, 12, step=4)
    _thin(orc, c, 12, step=5)
    va, vb, vc = a.view(), b.view(), c.view()
    for k in va:
        if va[k] is not None:
            assert np.array_equal(va[k], vb[k], equal_nan=True)
    assert set(int(i) for i in va["id"]) != set(int(i) for i in vc["id"])


def test_empty_store(orc):
    st = orc.Store(4)
    rec = _thin(orc, st, 3)
    assert rec["live_before"] == rec["kept"] == rec["groups"] == 0 and st.count == 0
