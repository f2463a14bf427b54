"""qed_sort_cells through the C ABI: the order of every instance's segment after the sort
equals a stable sort, on the host, of the cell-block keys computed with the same arithmetic
(cell = floor((x - origin) / dx) per axis, periodic; blocks of 2^s cells per axis, s the
smallest that leaves at most 2^24 - 2 blocks; removed photons last, non-finite positions
just before them), column for column; and a grid cascade whose stores are sorted every other step
still equals the oracle in every store and every step's record (the sort moves slots only)."""
import math

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


def _note(msg):
    print(msg, flush=True)


def host_keys(cols, n, dx, origin, dead):
    s = 0
    while math.prod((v + (1 << s) - 1) >> s for v in n) > (1 << 24) - 2:
        s += 1
    nb = [(v + (1 << s) - 1) >> s for v in n]
    # keys of 8, 16 or 24 bits: the fewest that hold every block and the two reserved keys
    passes = next(p for p in (1, 2, 3) if math.prod(nb) <= (1 << (8 * p)) - 2 or p == 3)
    top = (1 << (8 * passes)) - 1
    cell = []
    for d, c in enumerate(("x", "y", "z")):
        v = (cols[c] - origin[d]) / dx[d]
        with np.errstate(invalid="ignore"):
            fl = np.floor(v)
        ok = np.isfinite(fl)
        i = np.zeros(len(v), dtype=np.int64)
        i[ok] = np.mod(fl[ok].astype(np.int64), n[d])
        cell.append((i, ok))
    (ix, okx), (iy, oky), (iz, okz) = cell
    key = ((iz >> s) * nb[1] + (iy >> s)) * nb[0] + (ix >> s)
    key = np.where(okx & oky & okz, key, top - 1)
    return np.where(dead, top, key)


@pytest.mark.parametrize("n", [(7, 5, 4), (256, 256, 256), (300, 2, 9), (40, 40, 40),
                               (300, 300, 300)])
def test_sort_order_matches_a_stable_host_sort(n):
    rng = np.random.default_rng(sum(n))
    dx, origin = (0.7, 1.1, 0.45), (-2.0, 3.0, 0.5)
    caps = [(9000, 700, 30000), (10, 10, 10), (5000, 900, 12000), (300, 300, 300)]
    counts = [(8000, 650, 25000), (0, 0, 0), (4096, 1, 4097), (290, 280, 270)]
    e = Engine(caps, [1, 2, 3, 4])
    for i, cnt in enumerate(counts):
        for sp in range(3):
            m = cnt[sp]
            span = np.array(n) * np.array(dx)
            pos = [origin[d] - span[d] + 3 * span[d] * rng.random(m) for d in range(3)]
            cols = W._seed_columns(*pos, rng.normal(size=m), rng.normal(size=m),
                                   rng.normal(size=m), first_id=1000 * i)
            cols["parent"] = rng.integers(0, 2 ** 63, m, dtype=np.uint64)
            cols["birth"] = rng.integers(0, 2 ** 31, m, dtype=np.uint32)
            cols["w"] = rng.random(m)
            if sp == 2 and m:
                cols["id"][rng.random(m) < 0.1] = DEAD
                cols["x"][: m // 50] = np.nan
            cols["n_events"] = rng.integers(0, 9, m, dtype=np.uint32)
            e.load(i, sp, cols)
    e.set_frozen(3)  # a frozen instance is not sorted
    before = [[e.read(i, sp) for sp in range(3)] for i in range(len(caps))]
    f = Engine.make_field(Q.QED_FIELD_YEE, grid=[torch.zeros(1, device="cuda")] * 6, n=n,
                          dx=dx, origin=origin)
    for sp in range(3):
        e.sort_cells(sp, f)
    torch.cuda.synchronize()
    for i in range(len(caps)):
        assert e.counts()[i].tolist() == list(counts[i])
        for sp in range(3):
            b = before[i][sp]
            dead = (b["id"] == DEAD) if sp == 2 else np.zeros(len(b["id"]), bool)
            order = np.argsort(host_keys(b, n, dx, origin, dead), kind="stable")
            if i == 3:
                order = np.arange(len(order))
            got = e.read(i, sp)
            for c, v in b.items():
                assert np.array_equal(got[c], v[order], equal_nan=True), (n, i, sp, c)


def test_sorted_grid_cascade_matches_oracle(orc):
    """The 32^3 Yee-grid cascade with all three stores sorted by cell after every other step
    (the sort is part of the run, between steps): every store and record equals the
    oracle's, which never sorts."""
    w = W.standing_wave_grid(n=300, cells=32, capacity=200_000, lepton_capacity=20_000,
                             steps=40, a0=2000.0)
    init = W.standing_wave_initial(300, seed=2)
    _note(f"sorted yee grid: {w.description}")
    e = R.engine_single(w, init)
    grid = R.YeeGrid(w)
    f = R.field_of(w, grid=grid.g)
    p = R.params_of(w)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w)
    e.set_step(0)
    st, ost = [], []
    for n in range(w.n_steps):
        vals = W.standing_wave_grid_values(w.field, w.t0 + n * w.dt)
        grid.load_numpy(vals)
        if n % 2 == 1:
            for sp in range(3):
                e.sort_cells(sp, f)
        e.step(f, p)
        torch.cuda.synchronize()
        st.append(e.stats())
        op.step = n
        ost.append(orc.step(os_, oracle_field(orc, w, grids=vals), op))
    assert e.stats()["n_start"][2] > 100
    compare_stats(st, ost, label="sorted yee")
    compare_all(e, os_, label="sorted yee")


def test_full_size_lepton_store_sort_properties():
    """The grid cascade's electron store at its full size (2.5*10^7 slots, all live), sorted
    once on the 256^3 grid as the bench sorts it: checked by properties that hold at any
    size.  The host recomputes every key from the sorted columns: the keys do not decrease;
    the ids are a permutation of the input's; every row carries the columns of the input row
    with its id; and among equal keys the input order is kept (stability)."""
    n = 25_000_000
    rng = np.random.default_rng(7)
    cells, dxv = 256, 2.0 * np.pi / 32.0
    dx, origin = (dxv, dxv, dxv), (-128 * dxv, -128 * dxv, -128 * dxv)
    # most particles in a Gaussian cloud about the focus, the rest anywhere in and around
    # the box (periodic wrap), a few non-finite
    pos = []
    for d in range(3):
        v = rng.normal(0.0, 3.0 * dxv, n)
        far = rng.random(n) < 0.2
        v[far] = origin[d] + rng.uniform(-0.5, 1.5, int(far.sum())) * cells * dxv
        pos.append(v)
    pos[1][rng.random(n) < 1e-5] = np.inf
    cols = W._seed_columns(*pos, rng.normal(size=n), rng.normal(size=n), rng.normal(size=n),
                           first_id=1)
    cols["w"] = rng.random(n)
    cols["n_events"] = rng.integers(0, 50, n, dtype=np.uint32)
    _note("full-size sort: loading 2.5e7 electrons")
    e = Engine([(n, 10, 10)], [5])
    e.load(0, 0, cols)
    f = Engine.make_field(Q.QED_FIELD_YEE, grid=[torch.zeros(1, device="cuda")] * 6,
                          n=(cells, cells, cells), dx=dx, origin=origin)
    _note("full-size sort: sorting")
    e.sort_cells(0, f)
    torch.cuda.synchronize()
    got = e.read(0, 0)
    del e
    torch.cuda.empty_cache()
    assert int(len(got["id"])) == n
    keys = host_keys(got, (cells, cells, cells), dx, origin, np.zeros(n, bool))
    assert np.all(np.diff(keys) >= 0), "keys decrease"
    src = (got["id"] - np.uint64(1)).astype(np.int64)  # the input row of each output row
    assert np.array_equal(np.sort(src), np.arange(n)), "ids are not a permutation"
    for c in ("x", "y", "z", "px", "py", "pz", "w", "parent", "birth", "n_events"):
        assert np.array_equal(got[c], cols[c][src], equal_nan=True), c
    same = np.diff(keys) == 0
    assert np.all(np.diff(src)[same] > 0), "equal keys lost their order"
    # the sort did move rows (a trivial identity would pass the checks above)
    assert np.count_nonzero(src != np.arange(n)) > n // 2
