"""The deterministic generator factor and the reverse mode N_g of Sec. VI through the C ABI
against the oracle, to the bar of the other cascade tests: ids, parents, births, event
counts and weights bit-exact (w / N_g, the weight the copies left keep after a partial
decay, f_g times the parent's), momenta within 1e-12 of each particle's own |p|, positions
within 1e-12, every field of every step's record.  The rotating-E cascade in the three
append modes of the other parity tests, with same-step children (both generation kernels),
and on a Yee grid (fields at the particle and a B field)."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import compare_all, compare_stats, oracle_field, oracle_params, oracle_stores

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import runner as R  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)
ARENA_MODES = {"arena": None, "tiny_arena": 5000, "no_arena": 0}
FORMS = {
    "reverse": dict(runs_photon=3, runs_pair=2),
    "every": dict(f_every=1, f_photon=4.0, f_pair=2.0),
}
# the reverse mode multiplies the particles: shorter runs keep the stores from filling
PERIODS = {"reverse": 1.0, "every": 1.5}
YEE_STEPS = {"reverse": 24, "every": 40}
COUNTERS = ("emitted", "pairs", "dropped", "children_advanced", "deferred")


def _note(msg):
    print(msg, flush=True)


def _rotating(orc, over, periods, arena=None, same_step=False):
    """The rotating-E cascade (300 seeds, steps of T/200) on both sides."""
    w = W.rotating_e(n=300, periods=periods, capacity=600_000, lepton_capacity=60_000)
    init = W.rotating_e_initial(300, seed=3)
    e = R.engine_single(w, init, arena_records=arena, same_step=same_step)
    stats = R.run(e, R.field_of(w), R.params_of(w, **over), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, **over), w.n_steps)
    assert len(stats) == len(ostats) == w.n_steps
    for c in COUNTERS:
        assert [s[c] for s in stats] == [s[c] for s in ostats], c
    compare_stats(stats, ostats, label=str(over))
    compare_all(e, os_, label=str(over))
    assert sum(s["pairs"] for s in stats) > 5
    assert sum(s["dropped"] for s in stats) == 0
    return e, stats


def _check_form(e, form):
    g = e.read(0, 2)
    seeds = g["parent"] < np.uint64(300)  # photons of the seeds, whose weight is 1
    assert seeds.sum() > 100
    if form == "reverse":
        # a third of the seed's weight, halved by every sub-step in which one of the two
        # copies decayed
        ws = g["w"][seeds & (g["id"] != DEAD)]
        j = np.round(-np.log2(3.0 * ws))
        assert np.all((j >= 0) & (ws == (1.0 / 3.0) * np.exp2(-j)))
        assert np.any(j > 0) and np.any(j == 0)
        lep = e.read(0, 0)
        kids = lep["birth"] > 0  # electrons of pairs
        assert kids.sum() > 0 and np.all(lep["w"][kids] < 1.0)
    else:
        assert np.all(g["w"][seeds] == 4.0)
        lep = [e.read(0, s) for s in (0, 1)]
        events = int(sum(v["n_events"].sum() for v in lep))
        assert len(g["id"]) < events


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("arena", list(ARENA_MODES))
def test_rotating_cascade(orc, form, arena):
    _note(f"rotating cascade, {FORMS[form]}, {arena}")
    e, _ = _rotating(orc, FORMS[form], PERIODS[form], ARENA_MODES[arena])
    _check_form(e, form)


@pytest.mark.parametrize("form", list(FORMS))
def test_rotating_cascade_same_step_children(orc, form):
    """Children advanced through the rest of their birth step, two generations: the
    generation kernels take the same forms."""
    over = dict(FORMS[form], same_step_generations=2)
    _note(f"rotating cascade, {over}")
    e, stats = _rotating(orc, over, PERIODS[form], same_step=True)
    assert sum(s["children_advanced"] for s in stats) > 1000
    _check_form(e, form)


@pytest.mark.parametrize("form", list(FORMS))
def test_yee_grid(orc, form):
    """The standing-wave cascade on a 32^3 Yee grid, 24 or 40 steps."""
    over = FORMS[form]
    w = W.standing_wave_grid(n=300, cells=32, capacity=300_000, lepton_capacity=30_000,
                             steps=YEE_STEPS[form], a0=2000.0)
    init = W.standing_wave_initial(300, seed=2)
    _note(f"yee grid, {over}: {w.description}")
    e = R.engine_single(w, init)
    grid = R.YeeGrid(w)
    f = R.field_of(w, grid=grid.g)
    p = R.params_of(w, **over)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w, **over)
    e.set_step(0)
    st, ost = [], []
    for n in range(w.n_steps):
        vals = W.standing_wave_grid_values(w.field, w.t0 + n * w.dt)
        grid.load_numpy(vals)
        e.step(f, p)
        torch.cuda.synchronize()
        st.append(e.stats())
        op.step = n
        ost.append(orc.step(os_, oracle_field(orc, w, grids=vals), op))
    assert e.stats()["n_start"][2] > 100
    assert sum(s["pairs"] for s in ost) > 100
    assert sum(s["dropped"] for s in ost) == 0
    compare_stats(st, ost, label=f"yee {form}")
    compare_all(e, os_, label=f"yee {form}")


def test_forms_that_do_not_combine_are_refused():
    """A factor and the reverse mode on one generator, a deterministic factor that is no
    integer, more than 64 runs, a refill threshold outside 0..64: QED_ERR_ARG before any
    launch, the stores untouched."""
    from paper_1412_6426_amd import qed as Q
    w = W.rotating_e(n=50, periods=0.05, capacity=10_000, lepton_capacity=1000)
    e = R.engine_single(w, W.rotating_e_initial(50, seed=1))
    before = e.read(0, 0)
    for over in (dict(f_photon=2.0, runs_photon=2), dict(f_pair=3.0, runs_pair=3),
                 dict(f_every=1, f_photon=2.5), dict(f_every=1, f_pair=1.5),
                 dict(runs_photon=65), dict(runs_pair=65), dict(refill_min=65),
                 dict(refill_min=-1)):
        _note(f"refused: {over}")
        with pytest.raises(Q.QedError, match="argument"):
            e.step(R.field_of(w), R.params_of(w, **over))
    torch.cuda.synchronize()
    after = e.read(0, 0)
    for c in before:
        assert np.array_equal(before[c], after[c]), c
    assert int(e.step_ctr.item()) == 0


@pytest.mark.parametrize("form", list(FORMS))
def test_mixed_precision_follows_fp64_oracle(orc, form):
    """Both forms in mixed precision (the FP32 lepton, exact and generation kernels of each)
    against the FP64 oracle on the rotating-E cascade from 10^3 seeds: both draw the same
    numbers, so only decisions within FP32 rounding of a threshold differ; the weighted
    photon spectrum within L1 1e-3 and the pairs within 1% (plus three)."""
    import math
    over = FORMS[form]
    kw = dict(n=1000, periods=PERIODS[form], capacity=4_000_000, lepton_capacity=400_000)
    w = W.rotating_e(**kw)
    init = W.rotating_e_initial(1000, seed=21)
    os_ = oracle_stores(orc, init, w.capacity)
    ost = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, **over), w.n_steps)
    assert sum(s["dropped"] for s in ost) == 0

    def spectrum(cols):
        live = cols["id"] != DEAD
        e = np.sqrt(cols["px"][live] ** 2 + cols["py"][live] ** 2 + cols["pz"][live] ** 2)
        lo, hi, bins = W.SPECTRUM_LO, W.SPECTRUM_HI, W.SPECTRUM_BINS
        u = (np.log10(e) - math.log10(lo)) * bins / (math.log10(hi) - math.log10(lo))
        ok = (u >= 0) & (u < bins)
        return np.bincount(u[ok].astype(np.int64), weights=cols["w"][live][ok], minlength=bins)

    h_or = spectrum(os_[2].view())
    p_or = sum(s["pairs"] for s in ost)
    assert p_or > 100
    wm = W.rotating_e(**kw, precision="mixed")
    _note(f"mixed, {over}: {wm.description}")
    e = R.engine_single(wm, init)
    st = R.run(e, R.field_of(wm), R.params_of(wm, **over), wm.n_steps)
    h = spectrum(e.read(0, 2))
    l1 = float(np.abs(h - h_or).sum() / h_or.sum())
    pairs = sum(s["pairs"] for s in st)
    _note(f"mixed {form}: L1 {l1:.3e}, pairs {pairs} vs {p_or}")
    assert l1 <= 1e-3
    assert abs(pairs - p_or) <= 0.01 * p_or + 3
