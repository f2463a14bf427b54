"""Pins of the oracle's cap on the children one particle generates in one iteration (Sec. VII:
the thinning that restricts the super-particles generated from a single particle or photon
during one iteration).

What the method and the arithmetic fix: only the children born in the last step take part
(birth code (step + 1) << 14 | sub-step, against the step counter after the step), grouped
by the parent that made them; every group keeps its weight (the children of one parent in
one step share one weight, so the survivors take n / K of it); a group at or below the cap
is untouched; in a larger group each child survives independently with probability cap / n,
and at least one does; every other particle, removed photons included, is untouched and
keeps its place in the store order."""
import math

import numpy as np
import pytest

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)
STEP = 12  # the step counter after the step that made the children


def _store(orc, rng, sizes, photon=False, old=300, dead_every=0, equal_w=True):
    """Children of parents 1000 + j (sizes[j] each, born in step STEP - 1), `old` particles
    born earlier, shuffled together; parents' weights uniform in [0.5, 2)."""
    parents, births, w = [], [], []
    for j, m in enumerate(sizes):
        wp = rng.uniform(0.5, 2.0)
        parents += [1000 + j] * m
        births += [(STEP << 14) | int(k) for k in rng.integers(0, 16, m)]
        w += list(np.full(m, wp) if equal_w else rng.uniform(0.5, 2.0, m))
    parents += list(rng.integers(1000, 1000 + len(sizes) + 5, old))
    births += [(int(s) << 14) | 3 for s in rng.integers(0, STEP, old)]  # earlier steps
    w += list(rng.uniform(0.5, 2.0, old))
    n = len(parents)
    order = rng.permutation(n)
    cols = {c: rng.normal(size=n) for c in ("x", "y", "z", "px", "py", "pz")}
    cols["w"] = np.array(w)[order]
    cols["id"] = rng.choice(np.arange(1 << 40, (1 << 40) + 50 * n, dtype=np.uint64), n,
                            replace=False)
    cols["parent"] = np.array(parents, dtype=np.uint64)[order]
    cols["birth"] = np.array(births, dtype=np.uint32)[order]
    cols["n_events"] = rng.integers(0, 9, n, dtype=np.uint32)
    if dead_every:
        cols["id"][::dead_every] = DEAD
    st = orc.Store(n, with_events=not photon)
    st.load({k: v for k, v in cols.items() if not photon or k != "n_events"})
    return st, cols


def _thin(orc, st, cap, photon=False, seed=5, step=STEP):
    return orc.thin_children(st, photon, cap, seed, step)


def _is_child(cols, step=STEP, photon=False):
    c = (cols["birth"] >> 14) == step
    if photon:
        c &= cols["id"] != DEAD
    return c


def test_groups_keep_their_weight_and_nothing_else_changes(orc):
    rng = np.random.default_rng(1)
    sizes = list(rng.integers(1, 120, 300))
    st, cols = _store(orc, rng, sizes)
    rec = _thin(orc, st, 10)
    v = st.view()
    child = _is_child(cols)
    assert rec["children"] == int(child.sum())
    assert rec["groups"] == len(sizes)
    assert rec["groups_thinned"] == sum(m > 10 for m in sizes)
    # every particle that is no child of the last step, in its order and unchanged
    others = ~child
    vo = ~_is_child(v)
    for c in cols:
        if cols[c] is not None:
            assert np.array_equal(v[c][vo], cols[c][others]), c
    # the survivors: a subset of the children, each group's weight kept
    pos = {int(i): k for k, i in enumerate(cols["id"])}
    src = np.array([pos[int(i)] for i in v["id"]])
    assert np.all(np.diff(src) > 0)  # store order kept
    for c in ("x", "y", "z", "px", "py", "pz", "parent", "birth", "n_events"):
        assert np.array_equal(v[c], cols[c][src]), c
    for j, m in enumerate(sizes):
        g_in = child & (cols["parent"] == 1000 + j)
        g_out = _is_child(v) & (v["parent"] == 1000 + j)
        k = int(g_out.sum())
        assert 1 <= k <= m and (m > 10 or k == m)
        assert v["w"][g_out].sum() == pytest.approx(cols["w"][g_in].sum(), rel=1e-13)
        if m <= 10:
            assert np.array_equal(v["w"][g_out], cols["w"][g_in])
        else:
            assert np.allclose(v["w"][g_out], cols["w"][g_in][0] * m / k, rtol=1e-15, atol=0)
    assert rec["kept"] == int(_is_child(v).sum())
    assert rec["weight_before"] == pytest.approx(cols["w"][child].sum(), rel=1e-13)
    assert rec["weight_after"] == pytest.approx(rec["weight_before"], rel=1e-12)


def test_survival_is_binomial(orc):
    rng = np.random.default_rng(2)
    sizes = [200] * 400
    st, cols = _store(orc, rng, sizes, old=0)
    _thin(orc, st, 20)
    v = st.view()
    kept = np.array([int(np.count_nonzero(v["parent"] == 1000 + j)) for j in range(len(sizes))])
    q = 20 / 200
    # the mean survivors per group (at least one survives, which the cap of 20 never needs)
    assert abs(kept.mean() - 20) < 5 * math.sqrt(200 * q * (1 - q) / len(sizes))
    assert abs(kept.var() - 200 * q * (1 - q)) < 0.25 * 200 * q * (1 - q)


def test_survivors_are_the_draws_below_the_cap(orc):
    """Brute force on one parent's 300 children: the survivors are those whose Philox draw,
    keyed by the id with counter (step, 13 << 16, seed lo, seed hi), is below cap / n."""
    rng = np.random.default_rng(3)
    seed, cap = 0x1234_5678_9ABC, 29
    st, cols = _store(orc, rng, [300], old=50)
    _thin(orc, st, cap, seed=seed)
    q = cap / 300
    want = []
    for i in range(len(cols["id"])):
        idv = int(cols["id"][i])
        if (int(cols["birth"][i]) >> 14) != STEP:
            want.append(idv)
            continue
        o = orc.philox([STEP, 13 << 16, seed & 0xFFFFFFFF, seed >> 32],
                       [idv & 0xFFFFFFFF, idv >> 32])
        if orc.uniform(o[0], o[1]) < q:
            want.append(idv)
    assert [int(i) for i in st.view()["id"]] == want  # in store order


def test_a_group_that_draws_no_survivor_keeps_its_smallest_draw(orc):
    """Cap 1 on groups of 2 to 6 children: no draw falls below 1 / n in about a third of
    them, and then the child with the smallest draw survives with the group's weight."""
    rng = np.random.default_rng(4)
    sizes = [2 + j % 5 for j in range(400)]
    st, cols = _store(orc, rng, sizes, old=0)
    _thin(orc, st, 1, seed=3)
    v = st.view()
    seen_empty = 0
    for j, m in enumerate(sizes):
        members = np.flatnonzero(cols["parent"] == 1000 + j)
        out = np.flatnonzero(v["parent"] == 1000 + j)
        assert len(out) >= 1
        assert v["w"][out].sum() == pytest.approx(cols["w"][members].sum(), rel=1e-13)
        u = []
        for i in members:
            idv = int(cols["id"][i])
            o = orc.philox([STEP, 13 << 16, 3, 0], [idv & 0xFFFFFFFF, idv >> 32])
            u.append(orc.uniform(o[0], o[1]))
        u = np.array(u)
        if not np.any(u < 1.0 / m):
            seen_empty += 1
            assert len(out) == 1
            assert int(v["id"][out[0]]) == int(cols["id"][members[np.argmin(u)]])
    assert seen_empty > 50


def test_removed_photons_stay_and_other_steps_are_not_children(orc):
    rng = np.random.default_rng(5)
    st, cols = _store(orc, rng, [50, 80, 3], photon=True, old=400, dead_every=7)
    rec = _thin(orc, st, 4, photon=True)
    v = st.view()
    child = _is_child(cols, photon=True)
    assert rec["children"] == int(child.sum())
    # removed photons stay, in order, among the particles that are not live children
    assert int((v["id"] == DEAD).sum()) == int((cols["id"] == DEAD).sum())
    keep_src = ~child
    assert np.array_equal(v["id"][~_is_child(v, photon=True)], cols["id"][keep_src])
    # a step counter one off selects other children
    st2, _ = _store(orc, np.random.default_rng(5), [50, 80, 3], photon=True, old=400,
                    dead_every=7)
    rec2 = _thin(orc, st2, 4, photon=True, step=STEP + 1)
    assert rec2["children"] == 0 and st2.count == len(cols["id"])


def test_pairs_without_a_parent_are_no_group(orc):
    """Schwinger pairs of the last step carry no parent: however many, they stay."""
    rng = np.random.default_rng(10)
    st, cols = _store(orc, rng, [60, 5], old=100)
    orphans = np.flatnonzero((cols["parent"] == 1000) & ((cols["birth"] >> 14) == STEP))
    assert len(orphans) == 60  # the children of the first parent lose it
    cols["parent"][orphans] = np.uint64(0xFFFFFFFFFFFFFFFF)
    st = orc.Store(len(cols["id"]))
    st.load(cols)
    rec = _thin(orc, st, 4)
    assert rec["children"] == 5 and rec["groups"] == 1 and rec["groups_thinned"] == 1
    v = st.view()
    none = np.uint64(0xFFFFFFFFFFFFFFFF)
    assert np.array_equal(v["id"][v["parent"] == none], cols["id"][cols["parent"] == none])


def test_unequal_weights_are_kept_in_expectation(orc):
    """Children of one parent with different weights (the pairs of one photon in the reverse
    mode): the survivors take n / K of their own weight, so the group keeps its weight on
    average over the draws."""
    rng = np.random.default_rng(6)
    sizes = [40] * 500
    st, cols = _store(orc, rng, sizes, old=0, equal_w=False)
    rec = _thin(orc, st, 8)
    v = st.view()
    pos = {int(i): k for k, i in enumerate(cols["id"])}
    for j in range(len(sizes)):
        out = np.flatnonzero(v["parent"] == 1000 + j)
        k = len(out)
        src = [pos[int(i)] for i in v["id"][out]]
        assert np.allclose(v["w"][out], cols["w"][src] * 40 / k, rtol=1e-15, atol=0)
    # the total over 500 groups: mean of sum (n / K) w_i 1[kept] is sum w_i
    per_group = np.array([v["w"][v["parent"] == 1000 + j].sum() for j in range(len(sizes))])
    before = np.array([cols["w"][cols["parent"] == 1000 + j].sum() for j in range(len(sizes))])
    rel = per_group / before - 1.0
    assert abs(rel.mean()) < 5 * rel.std() / math.sqrt(len(sizes))
    assert rec["weight_after"] != pytest.approx(rec["weight_before"], rel=1e-12)


def test_deterministic_and_keyed_by_seed(orc):
    out = []
    for seed in (7, 7, 8):
        st, _ = _store(orc, np.random.default_rng(8), [90] * 40)
        _thin(orc, st, 9, seed=seed)
        out.append(st.view())
    for k in out[0]:
        if out[0][k] is not None:
            assert np.array_equal(out[0][k], out[1][k], equal_nan=True)
    assert set(int(i) for i in out[0]["id"]) != set(int(i) for i in out[2]["id"])


def test_empty_store_and_no_children(orc):
    st = orc.Store(4)
    rec = _thin(orc, st, 3)
    assert rec["children"] == rec["kept"] == rec["groups"] == 0 and st.count == 0
    st, cols = _store(orc, np.random.default_rng(9), [], old=100)
    rec = _thin(orc, st, 1)
    assert rec["children"] == 0 and st.count == 100 and not rec["thinned"]
