"""qed_thin_children (the cap on the children one particle generates in one step, Sec. VII)
through the C ABI against the oracle: the stores after the call equal the oracle's row for
row (same order, every column, weights bit-identical: both sides scale a survivor by the
same n / K), counts and records equal (the records' weight sums to 1e-12: they are summed
in another order), frozen instances untouched; and a rotating-E cascade whose photons and
pair leptons are capped per parent after every step equals the oracle run with the same
cap."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import compare_all, compare_stats, oracle_field, oracle_params, oracle_stores

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import qed as Q  # noqa: E402
from paper_1412_6426_amd import runner as R  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402
from paper_1412_6426_amd.engine import Engine  # noqa: E402

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)
COLS = ("x", "y", "z", "px", "py", "pz", "w", "id", "parent", "birth")
STEP = 9  # the step counter after the step that made the children


def _note(msg):
    print(msg, flush=True)


def _columns(rng, sizes, old, photon, first_id):
    """Children of parents first_id + 7 j (sizes[j] each, born in step STEP - 1, sharing the
    parent's weight), `old` particles of earlier steps, some children without a parent,
    shuffled; removed photons among them."""
    parents, births, w = [], [], []
    for j, m in enumerate(sizes):
        parents += [first_id + 7 * j] * m
        births += [(STEP << 14) | int(k) for k in rng.integers(0, 40, m)]
        w += [rng.uniform(0.5, 2.0)] * m
    parents += list(first_id + 7 * rng.integers(0, len(sizes) + 3, old))
    births += [(int(s) << 14) | 1 for s in rng.integers(0, STEP, old)]
    w += list(rng.uniform(0.5, 2.0, old))
    n = len(parents)
    order = rng.permutation(n)
    cols = W._seed_columns(*[rng.normal(size=n) for _ in range(6)], first_id=first_id * 1000)
    cols["w"] = np.array(w)[order]
    cols["parent"] = np.array(parents, dtype=np.uint64)[order]
    cols["birth"] = np.array(births, dtype=np.uint32)[order]
    cols["n_events"] = rng.integers(0, 9, n, dtype=np.uint32)
    if n:
        orphan = rng.random(n) < 0.03
        cols["parent"][orphan] = np.uint64(0xFFFFFFFFFFFFFFFF)  # Schwinger pairs
        if photon:
            cols["id"][rng.random(n) < 0.06] = DEAD
    return cols


def test_thin_children_matches_oracle(orc):
    """Four instances (one without children, one frozen), every species; caps 1, 4, 25."""
    rng = np.random.default_rng(5)
    plans = [([rng.integers(1, 200) for _ in range(300)], 2000),
             ([], 500),
             ([rng.integers(1, 9) for _ in range(4000)], 100),
             ([50] * 20, 30)]
    caps = []
    init = []
    seeds = [21, 22, 23, 24]
    for i, (sizes, old) in enumerate(plans):
        per = [_columns(rng, sizes, old, sp == 2, 10_000 * (i + 1)) for sp in range(3)]
        init.append(per)
        caps.append(tuple(len(c["id"]) + 17 for c in per))
    e = Engine(caps, seeds)
    for i in range(len(plans)):
        for sp in range(3):
            e.load(i, sp, init[i][sp])
    e.set_frozen(3)
    e.set_step(STEP)
    seen = 0
    for sp, cap in ((0, 1), (1, 4), (2, 25)):
        _note(f"thin children: species {sp}, cap {cap}")
        before3 = e.read(3, sp)
        e.thin_children(sp, cap)
        torch.cuda.synchronize()
        recs = e.thin_children_records()
        for i in range(len(plans)):
            got = e.read(i, sp)
            if i == 3:
                for c in COLS:
                    assert np.array_equal(got[c], before3[c], equal_nan=True), c
                assert all(v == 0 for v in recs[i].values())
                continue
            st = orc.Store(caps[i][sp], with_events=sp != 2)
            st.load({k: v for k, v in init[i][sp].items() if sp != 2 or k != "n_events"})
            orec = orc.thin_children(st, sp == 2, cap, seeds[i], STEP)
            want = st.view()
            assert e.counts()[i, sp] == st.count == len(got["id"]), (i, sp)
            for c in COLS:
                assert np.array_equal(got[c], want[c], equal_nan=True), (i, sp, c)
            if sp != 2:
                assert np.array_equal(got["n_events"], want["n_events"])
            for k in ("children", "groups", "groups_thinned", "kept"):
                assert recs[i][k] == orec[k], (i, sp, k)
            for k in ("weight_before", "weight_after"):
                assert recs[i][k] == pytest.approx(orec[k], rel=1e-12, abs=1e-300), (i, sp, k)
            seen += orec["groups_thinned"]
    assert seen > 1000


def test_rotating_cascade_capped_per_parent_matches_oracle(orc):
    """The rotating-E cascade in the reverse mode for pairs (two runs, so a photon can make
    two pairs in a step), with at most one photon per lepton and one lepton of each charge
    per photon kept after every step, on both sides."""
    w = W.rotating_e(n=300, periods=1.0, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    over = dict(runs_pair=2)
    _note(f"capped cascade: {w.description}")
    e = R.engine_single(w, init)
    f = R.field_of(w)
    p = R.params_of(w, **over)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w, **over)
    fo = oracle_field(orc, w)
    e.set_step(0)
    st, ost, thinned = [], [], 0
    for n in range(w.n_steps):
        e.step(f, p)
        op.step = n
        ost.append(orc.step(os_, fo, op))
        torch.cuda.synchronize()
        st.append(e.stats())
        for sp in range(3):
            e.thin_children(sp, 1)
            torch.cuda.synchronize()
            g = e.thin_children_records()[0]
            o = orc.thin_children(os_[sp], sp == 2, 1, w.seed, n + 1)
            for k in ("children", "groups", "groups_thinned", "kept"):
                assert g[k] == o[k], (n, sp, k)
            thinned += o["groups_thinned"]
    assert thinned > 100
    assert sum(s["pairs"] for s in ost) > 5
    compare_stats(st, ost, label="capped")
    compare_all(e, os_, label="capped")


def test_refused_arguments():
    w = W.rotating_e(n=10, periods=0.05, capacity=1000, lepton_capacity=100)
    e = R.engine_single(w, W.rotating_e_initial(10, seed=1))
    with pytest.raises(Q.QedError, match="argument"):
        e.thin_children(0, 0)
