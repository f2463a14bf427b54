"""GPU Schwinger pair production (qed_schwinger, Sec. V.B) against the oracle.

The decisions and positions come from per-cell Philox draws on both sides, so the pairs,
their ids, births and weights are bit-exact; positions agree within 1e-12 (the two sides
may contract origin + (i + u) dx differently); the expected count (a sum of per-cell
probabilities taken in different orders) within 1e-12 relative on the small grids, and
within (n + 2) 2^-53 relative for the n = 1.7e7 cells of the full grid (the bound for
summing n positive terms in any order, plus an ulp of exp per term on each side).  The store order follows
the GPU's reservations; multisets are compared."""
import math

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import compare_species

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import qed as Q  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402
from paper_1412_6426_amd.engine import Engine  # noqa: E402

N = (24, 20, 16)
DX = 0.5


def _note(msg):
    print(msg, flush=True)


def _grids(seed, n=N, widths=(6.0, 5.0, 4.0)):
    """A field blob up to |E| = 4 E_S (eps_r = 1) with random directions, and a random B."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (((i - nx / 2) / widths[0]) ** 2 + ((j - ny / 2) / widths[1]) ** 2 +
          ((k - nz / 2) / widths[2]) ** 2)
    mag = 4.0 * np.exp(-r2)
    out = []
    for d in (0.48, 0.6, 0.64):  # a unit direction, with 10% noise per sample
        out.append((mag * d * (1.0 + 0.1 * rng.normal(size=mag.shape))).astype(np.float32))
    for _ in range(3):
        out.append(rng.normal(size=mag.shape).astype(np.float32))
    return [np.ascontiguousarray(a) for a in out]


def _oracle_stores(orc, cap):
    st = [orc.Store(cap), orc.Store(cap), orc.Store(16, with_events=False)]
    for s in st:
        s.load(W.empty_columns())
    return st


def _engine(caps, seeds):
    e = Engine([(c, c, 16) for c in caps], seeds=seeds)
    return e


def _field(grids, n=N):
    dev = [torch.from_numpy(g).to("cuda") for g in grids]
    f = Engine.make_field(Q.QED_FIELD_YEE, grid=dev, n=n, dx=(DX, DX, DX), origin=(-1.0, 0.5, 2.0))
    return f, dev


def test_schwinger_matches_oracle(orc):
    grids = _grids(1)
    f, keep = _field(grids)
    ofld = orc.Field(kind=orc.FIELD_YEE, grid=grids, dx=(DX, DX, DX), origin=(-1.0, 0.5, 2.0))
    dt = 400.0
    e = _engine([200_000], [7])
    ost = _oracle_stores(orc, 200_000)
    for step in range(4):
        _note(f"schwinger step {step}")
        e.set_step(step)
        e.schwinger(f, dt, 1.0, weight=1.5)
        torch.cuda.synchronize()
        r = e.schwinger_record()
        o = orc.schwinger(ost, ofld, dt, 1.0, 1.5, seed=7, step=step)
        for c in ("cells", "pairs", "dropped", "saturated"):
            assert r[c] == o[c], (step, c)
        assert r["expected"] == pytest.approx(o["expected"], rel=1e-12)
    assert r["pairs"] > 100 and r["saturated"] > 0
    for s in range(2):
        compare_species(e.read(0, s), ost[s].view(), s, rtol=1e-12, label=f"species {s}")


def test_schwinger_instances_draw_their_own_pairs(orc):
    """Three instances (seeds 2, 4, 3) on the same grid; the second has room for only ten
    pairs (drops counted, its counts brought back to its capacity, so the instance after it
    keeps its segment), the third is frozen."""
    grids = _grids(2)
    f, keep = _field(grids)
    ofld = orc.Field(kind=orc.FIELD_YEE, grid=grids, dx=(DX, DX, DX), origin=(-1.0, 0.5, 2.0))
    dt = 400.0
    e = _engine([100_000, 10, 100_000], [2, 4, 3])
    e.set_frozen(2)
    e.set_step(5)
    e.schwinger(f, dt, 1.0)
    torch.cuda.synchronize()
    r = e.schwinger_record()
    inst = e.instances()
    want_pairs = want_drop = want_cells = 0
    assert inst[1]["count"][:2] == [10, 10]  # clamped to the capacity after the drops
    for i, (seed, cap) in enumerate(((2, 100_000), (4, 10), (3, 100_000))):
        if i == 2:
            assert inst[2]["count"][:2] == [0, 0]
            continue
        ost = _oracle_stores(orc, cap)
        o = orc.schwinger(ost, ofld, dt, 1.0, 1.0, seed=seed, step=5)
        want_pairs += o["pairs"]
        want_drop += o["dropped"]
        want_cells += o["cells"]
        for s in range(2):
            got = e.read(i, s)
            if i == 1:
                # the store keeps 10 of the instance's pairs (which ones depends on the order
                # of the reservations; the oracle keeps the first 10 in cell order): they are
                # a subset of all the pairs the oracle makes with room for them, field for field
                assert len(got["id"]) == 10
                full = _oracle_stores(orc, 100_000)
                orc.schwinger(full, ofld, dt, 1.0, 1.0, seed=seed, step=5)
                want = full[s].view()
                at = {int(v): q for q, v in enumerate(want["id"])}
                rows = [at[int(v)] for v in got["id"]]
                for c in ("parent", "birth", "w", "px", "py", "pz"):
                    assert np.array_equal(got[c], want[c][rows]), c
                for c in ("x", "y", "z"):
                    np.testing.assert_allclose(got[c], want[c][rows], rtol=1e-12, atol=1e-12)
                continue
            compare_species(got, ost[s].view(), s, rtol=1e-12, label=f"instance {i} sp {s}")
        assert inst[i]["dropped"] == o["dropped"]
    assert r["pairs"] == want_pairs and r["dropped"] == want_drop and r["cells"] == want_cells
    assert want_drop > 0


def test_schwinger_rows_of_several_pieces(orc):
    """150 x 12 x 10 cells: each row is two full 64-cell pieces and a ragged 22-cell tail,
    the pieces split unevenly over the workgroups, and the drawing cells of the blob fill the
    per-wavefront draw queues several times over, with a partial queue left at the end."""
    n = (150, 12, 10)
    grids = _grids(3, n=n, widths=(40.0, 4.0, 3.5))
    f, keep = _field(grids, n=n)
    ofld = orc.Field(kind=orc.FIELD_YEE, grid=grids, dx=(DX, DX, DX), origin=(-1.0, 0.5, 2.0))
    dt = 400.0
    e = _engine([400_000], [11])
    ost = _oracle_stores(orc, 400_000)
    for step in range(3):
        _note(f"schwinger rows step {step}")
        e.set_step(step)
        e.schwinger(f, dt, 1.0, weight=0.5)
        torch.cuda.synchronize()
        r = e.schwinger_record()
        o = orc.schwinger(ost, ofld, dt, 1.0, 0.5, seed=11, step=step)
        for c in ("cells", "pairs", "dropped", "saturated"):
            assert r[c] == o[c], (step, c)
        assert r["expected"] == pytest.approx(o["expected"], rel=1e-12)
    assert r["pairs"] > 1000
    for s in range(2):
        compare_species(e.read(0, s), ost[s].view(), s, rtol=1e-12, label=f"species {s}")


def test_schwinger_without_field_makes_nothing(orc):
    grids = [np.zeros(N[::-1], np.float32) for _ in range(6)]
    f, keep = _field(grids)
    e = _engine([1000], [1])
    e.set_step(0)
    e.schwinger(f, 400.0, 1.0)
    torch.cuda.synchronize()
    r = e.schwinger_record()
    assert r["cells"] == N[0] * N[1] * N[2]
    assert r["pairs"] == 0 and r["expected"] == 0.0 and r["saturated"] == 0
    assert e.instances()[0]["count"][:2] == [0, 0]


def test_schwinger_full_grid_parity(orc):
    """The bench's Schwinger workload at full size, in the launch configuration it times: the
    256^3 standing-wave grid (cells of lambda/32, dt = T/100) with the wave raised so that
    the antinodes reach 0.075 E_S.  Two steps, each against the oracle over the whole grid
    (about 260 pairs a step out of 1.7e7 cells, 42% of which draw)."""
    w = W.standing_wave_grid(n=1)
    w.field.grid_wave_amp = 0.075 / (2.0 * w.eps_r)
    fs = w.field
    e = _engine([100_000], [0])
    ost = _oracle_stores(orc, 100_000)
    for step in range(2):
        t = w.t0 + step * w.dt
        _note(f"schwinger full grid step {step}")
        grids = [np.ascontiguousarray(g) for g in W.standing_wave_grid_values(fs, t)]
        dev = [torch.from_numpy(g).to("cuda") for g in grids]
        f = Engine.make_field(Q.QED_FIELD_YEE, grid=dev, n=fs.grid_n, dx=fs.grid_dx,
                              origin=fs.grid_origin)
        e.set_step(step)
        e.schwinger(f, w.dt, w.eps_r, weight=1.0)
        torch.cuda.synchronize()
        r = e.schwinger_record()
        ofld = orc.Field(kind=orc.FIELD_YEE, grid=grids, dx=fs.grid_dx, origin=fs.grid_origin)
        o = orc.schwinger(ost, ofld, w.dt, w.eps_r, 1.0, seed=0, step=step)
        for c in ("cells", "pairs", "dropped", "saturated"):
            assert r[c] == o[c], (step, c)
        # a sum of 1.7e7 positive terms in two orders: within (n - 1) u of each other, plus
        # the per-term ulp of exp on each side
        assert r["expected"] == pytest.approx(o["expected"], rel=(r["cells"] + 2) * 2.0 ** -53)
        assert r["pairs"] > 100
        del dev, grids
    for s in range(2):
        compare_species(e.read(0, s), ost[s].view(), s, rtol=1e-12, label=f"species {s}")
