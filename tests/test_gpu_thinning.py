"""GPU thinning (qed_thin, global even redistribution of Sec. VI) against the oracle.

The survivors are decided by per-particle draws on both sides, so the set of survivors,
their ids and every column but the weight are bit-exact; the weight factor is the live
weight over the surviving weight, sums that the two sides take in different orders, so
weights agree within 1e-10 relative (the rounding of a sum of N positive terms in any
order is below (N-1) 2^-53 of it: 1e-10 covers N up to 10^6).  The store order differs
(the GPU fills holes from the tail); multisets are compared."""
import math

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import (compare_all, compare_species, oracle_field, oracle_params,
                               oracle_stores)

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import qed as Q  # noqa: E402
from paper_1412_6426_amd import runner as R  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402
from paper_1412_6426_amd.engine import Engine  # noqa: E402

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)
WTOL = 1e-10


def _note(msg):
    print(msg, flush=True)


def _columns(n, seed, dead_every=0, photon=False):
    rng = np.random.default_rng(seed)
    cols = {c: rng.normal(size=n) for c in ("x", "y", "z", "px", "py", "pz")}
    cols["w"] = rng.uniform(0.5, 2.0, n)
    cols["id"] = (np.arange(n, dtype=np.uint64) * np.uint64(2654435761) + np.uint64(seed)) \
        | np.uint64(1 << 63)
    if dead_every:
        cols["id"][::dead_every] = DEAD
    cols["parent"] = rng.integers(0, 1 << 62, n, dtype=np.int64).astype(np.uint64)
    cols["birth"] = rng.integers(0, 1 << 20, n, dtype=np.int64).astype(np.uint32)
    if not photon:
        cols["n_events"] = rng.integers(0, 9, n, dtype=np.int64).astype(np.uint32)
    return cols


@pytest.mark.parametrize("species", [0, 2])
def test_thin_matches_oracle(orc, species):
    """Four instances: three above the trigger (thinned to the same target from different
    sizes) and one below it; each segment is cut into 24 ranges with ragged ends."""
    photon = species == 2
    sizes = [300_001, 257_777, 90_000, 120_000]
    caps = [(n, n, n) for n in sizes]
    e = Engine(caps, seeds=[5, 6, 7, 8])
    ocols = []
    for i, n in enumerate(sizes):
        cols = _columns(n, 10 + i, dead_every=7 if photon else 0, photon=photon)
        full = dict(cols)
        if photon:
            full["n_events"] = np.zeros(n, np.uint32)
        e.load(i, species, full)
        ocols.append(cols)
    step = 123
    e.set_step(step)
    trigger, target = 100_000, 60_000
    _note(f"thinning species {species}")
    e.thin(species, trigger, target)
    torch.cuda.synchronize()
    recs = e.thin_records()
    for i, n in enumerate(sizes):
        st = orc.Store(n, with_events=not photon)
        st.load(ocols[i])
        orec = orc.thin(st, trigger, target, seed=5 + i, step=step)
        r = recs[i]
        assert r["thinned"] == int(orec["thinned"]), i
        assert r["live_before"] == orec["live_before"] and r["kept"] == orec["kept"], i
        assert r["factor"] == pytest.approx(orec["factor"], rel=WTOL)
        assert r["weight_before"] == pytest.approx(orec["weight_before"], rel=WTOL)
        got = e.read(i, species)
        assert len(got["id"]) == orec["kept"] if orec["thinned"] else len(got["id"]) == n
        want = st.view()
        if photon:
            got.pop("n_events")
            want.pop("n_events", None)
        compare_species(got, want, species, rtol=0.0, label=f"instance {i}", wtol=WTOL)
        if orec["thinned"]:
            assert not np.any(got["id"] == DEAD)
            assert got["w"].sum() == pytest.approx(orec["weight_before"], rel=1e-12)
    assert [r["thinned"] for r in recs] == [1, 1, 0, 1]


@pytest.mark.parametrize("n", [3_000_017, 16_789_561])
def test_thin_large_segment(orc, n):
    """One instance whose segment is cut into 367 ranges (two per thread of the plan
    kernels, the last thread's group short) or into the maximum of 2048 ranges of 8198
    slots (the last one short)."""
    cols = _columns(n, 21, dead_every=5, photon=True)
    full = dict(cols)
    full["n_events"] = np.zeros(n, np.uint32)
    e = Engine([(1, 1, n)], seeds=[17])
    e.load(0, 2, full)
    del full
    e.set_step(77)
    _note(f"thinning one segment of {n} photons")
    e.thin(2, 0, n // 3)
    torch.cuda.synchronize()
    r = e.thin_records()[0]
    st = orc.Store(n, with_events=False)
    st.load(cols)
    orec = orc.thin(st, 0, n // 3, seed=17, step=77)
    assert r["thinned"] == 1 and orec["thinned"]
    assert r["live_before"] == orec["live_before"] and r["kept"] == orec["kept"]
    assert r["factor"] == pytest.approx(orec["factor"], rel=WTOL)
    got = e.read(0, 2)
    got.pop("n_events")
    compare_species(got, st.view(), 2, rtol=0.0, label=f"{n} photons", wtol=WTOL)


def test_thin_small_and_degenerate_stores(orc):
    """Fewer slots than ranges, a target of one, and a store of removed photons only."""
    e = Engine([(1, 1, 40), (1, 1, 1000), (1, 1, 50)], seeds=[1, 2, 3])
    c0 = _columns(40, 1, photon=True)
    c1 = _columns(1000, 2, photon=True)
    c2 = _columns(50, 3, photon=True)
    c2["id"][:] = DEAD
    for i, c in enumerate((c0, c1, c2)):
        full = dict(c)
        full["n_events"] = np.zeros(len(c["x"]), np.uint32)
        e.load(i, 2, full)
    e.set_step(9)
    e.thin(2, 10, 1)
    torch.cuda.synchronize()
    recs = e.thin_records()
    for i, c in enumerate((c0, c1, c2)):
        st = orc.Store(len(c["x"]), with_events=False)
        st.load(c)
        orec = orc.thin(st, 10, 1, seed=i + 1, step=9)
        assert recs[i]["kept"] == orec["kept"] and recs[i]["thinned"] == int(orec["thinned"])
        got = e.read(i, 2)
        got.pop("n_events")
        compare_species(got, st.view(), 2, rtol=0.0, label=f"store {i}", wtol=WTOL)
    assert recs[2]["thinned"] == 0 and recs[2]["live_before"] == 0


def test_cascade_with_thinning_matches_oracle(orc):
    """The rotating-field cascade kept under a small photon capacity by thinning after every
    step (trigger 3/4 of the capacity, target 3/8): never a drop, and every store equals the
    oracle's run with the same thinning."""
    cap = 20_000
    w = W.rotating_e(n=300, periods=1.5, capacity=cap, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    e = R.engine_single(w, init)
    f, p = R.field_of(w), R.params_of(w)
    os_ = oracle_stores(orc, init, w.capacity)
    of, op = oracle_field(orc, w), oracle_params(orc, w)
    trigger, target = 3 * cap // 4, 3 * cap // 8
    thinned = 0
    e.set_step(0)
    for n in range(w.n_steps):
        e.step(f, p)
        e.thin(2, trigger, target)
        torch.cuda.synchronize()
        op.step = n
        s = orc.step(os_, of, op)
        r = orc.thin(os_[2], trigger, target, seed=w.seed, step=n + 1)
        g = e.thin_records()[0]
        assert g["kept"] == r["kept"] and g["thinned"] == int(r["thinned"]), n
        assert s["dropped"] == 0 and e.stats()["dropped"] == 0
        thinned += int(r["thinned"])
    assert thinned >= 3
    compare_all(e, os_, label="thinned cascade", wtol=WTOL)
