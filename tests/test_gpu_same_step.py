"""GPU same-step processing (children advanced through the rest of their birth step, Sec.
IV.H) against the oracle: every store to the parity bar of the other cascade tests (ids,
parents, births, event counts and weights bit-exact, momenta within 1e-12 of each particle's
own |p|, positions within 1e-12), and every field of the per-step record, among them the
photons and pairs created, the children advanced in their birth step and the children
deferred to the next one."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import (compare_all, compare_species, compare_stats,
                               lepton_birth_momentum, merge_stats, oracle_field, oracle_params,
                               oracle_stores)

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import runner as R  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402

COUNTERS = ("emitted", "pairs", "children_advanced", "deferred", "dropped")


def _note(msg):
    print(msg, flush=True)


def _check_steps(stats, ostats, label=""):
    assert len(stats) == len(ostats)
    for c in COUNTERS:
        assert [s[c] for s in stats] == [s[c] for s in ostats], c
    assert sum(s["near_threshold"] for s in stats) == 0
    compare_stats(stats, ostats, label=label)


@pytest.mark.parametrize("G", [1, 3])
def test_rotating_cascade_same_step_parity(orc, G):
    """The rotating-E cascade (300 seeds, 300 steps of T/200)."""
    w = W.rotating_e(n=300, periods=1.5, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    _note(f"rotating cascade, G = {G}")
    e = R.engine_single(w, init, same_step=True)
    stats = R.run(e, R.field_of(w), R.params_of(w, same_step_generations=G), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, same_step_generations=G),
                     w.n_steps)
    _check_steps(stats, ostats, label=f"rotating G={G}")
    assert sum(s["children_advanced"] for s in stats) > 10_000
    compare_all(e, os_, label=f"rotating G={G}")


@pytest.mark.parametrize("G", [4, 16])
def test_shower_same_step_parity(orc, G):
    """The Sec. VII shower at a large step (20 seeds, dt = 25000, about 400 lepton
    sub-steps a step, kappa = 0.25, three steps): many generations in every step; with
    G = 4 part of them waits for the next step.  Every decision, id, weight and counter is
    bit-exact.  The momenta carry the problem's own conditioning: a lepton that radiates
    almost all of its energy keeps p (1 - f) with f near 1, so its rounding is relative to
    its momentum at birth (|p| plus the |k| it has emitted, the largest |p| it ever had in
    the pure magnetic field), and leptons born late with a few m c turn through hundreds of
    sub-steps of large rotation angle, which add up rounding; photons inherit it.  The
    oracle run again with B one ulp larger moves its own leptons by about 3e-13 of their
    momentum at birth and its photons by about 1e-12 of their |k|.  So leptons are held to
    their momentum at birth and photons to their own |k|, each within the larger of 1e-12
    and ten times that one-ulp spread; positions within 1e-12 of c t, the distance the run
    lets a particle travel (or ten times the spread)."""
    w = W.shower(n=20, steps=3)
    init = W.shower_initial(w)
    _note(f"shower, G = {G}: {w.description}")
    e = R.engine_single(w, init, same_step=True)
    stats = R.run(e, R.field_of(w), R.params_of(w, same_step_generations=G), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w, same_step_generations=G)
    ostats = orc.run(os_, oracle_field(orc, w), op, w.n_steps)
    assert sum(s["pairs"] for s in stats) > 100
    if G == 4:
        assert sum(s["deferred"] for s in stats) > 0
    birth = lepton_birth_momentum(os_[2].view())
    scales = (birth, birth, None)
    f_ulp = oracle_field(orc, w)
    f_ulp.b0 = (f_ulp.b0[0], f_ulp.b0[1], f_ulp.b0[2] * (1.0 + 2.0 ** -52))
    ou = oracle_stores(orc, init, w.capacity)
    ustats = orc.run(ou, f_ulp, oracle_params(orc, w, same_step_generations=G), w.n_steps)
    spread = 0.0
    for sp in range(3):
        d = compare_species(ou[sp].view(), os_[sp].view(), sp, rtol=1.0, label="ulp",
                            pos_floor=w.dt * w.n_steps, p_scale=scales[sp])
        spread = max(spread, *d.values())
    for a, b in zip(ustats, ostats):
        for f in ("photon_energy", "max_p_emit", "max_p_pair"):
            if b[f] > 0:
                spread = max(spread, abs(a[f] - b[f]) / b[f])
    tol = max(1e-12, 10.0 * spread)
    _note(f"one-ulp spread {spread:.2e}, tolerance {tol:.2e}")
    for c in COUNTERS:
        assert [s[c] for s in stats] == [s[c] for s in ostats], c
    assert sum(s["near_threshold"] for s in stats) == 0
    compare_stats(stats, ostats, label=f"shower G={G}",
                  float_rtol=None if tol <= 1e-12 else tol)
    compare_all(e, os_, rtol=tol, label=f"shower G={G}", pos_floor=w.dt * w.n_steps,
                p_scale=scales)


def test_standing_wave_grid_same_step_parity(orc):
    """Position-dependent fields (a 32^3 Yee grid): children carry their parent's sampled
    fields through the rest of the step."""
    w = W.standing_wave_grid(n=300, cells=32, capacity=200_000, lepton_capacity=20_000,
                             steps=40, a0=2000.0)
    init = W.standing_wave_initial(300, seed=2)
    _note(f"yee grid with same-step children: {w.description}")
    e = R.engine_single(w, init, same_step=True)
    grid = R.YeeGrid(w)
    f = R.field_of(w, grid=grid.g)
    p = R.params_of(w, same_step_generations=2)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w, same_step_generations=2)
    e.set_step(0)
    stats, ostats = [], []
    for n in range(w.n_steps):
        vals = W.standing_wave_grid_values(w.field, w.t0 + n * w.dt)
        grid.load_numpy(vals)
        e.step(f, p)
        torch.cuda.synchronize()
        stats.append(e.stats())
        op.step = n
        ostats.append(orc.step(os_, oracle_field(orc, w, grids=vals), op))
    _check_steps(stats, ostats, label="yee same-step")
    assert sum(s["children_advanced"] for s in stats) > 100
    compare_all(e, os_, label="yee same-step")


def test_generations_zero_is_unchanged(orc):
    """A workspace sized for same-step processing, run without it, gives the plain step."""
    w = W.rotating_e(n=200, periods=1.0, capacity=200_000, lepton_capacity=20_000)
    init = W.rotating_e_initial(200, seed=4)
    e = R.engine_single(w, init, same_step=True)
    stats = R.run(e, R.field_of(w), R.params_of(w), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w), w.n_steps)
    _check_steps(stats, ostats, label="G=0")
    assert sum(s["children_advanced"] for s in stats) == 0
    compare_all(e, os_, label="G=0")


def test_avalanche_same_step_parity(orc):
    """The Sec. VII avalanche at its large step (60 seeds, dt = 173 t_rad, about T / 8, in
    the linearly polarised standing wave): position-dependent fields that children
    inherit, a cascade that grows tenfold per period.  The avalanche is chaotic: the oracle
    run again with the field amplitude one ulp larger (device sincos and libm sin, cos
    differ by about an ulp) moves its own momenta by about 1e-15 after two large steps, 5e-13
    after three and 5e-11 after four, and changes its event counts from the eighth.  So:
    after two steps every store and record to the full bar (1e-12); after six, every
    decision, id, weight and counter still bit-exact, and momenta, positions, the radiated
    energy and the largest probabilities within ten times the spread that the one-ulp change
    makes in the oracle itself."""
    w = W.avalanche(n=60, dt_over_t_rad=173.0, periods=0.75)
    assert w.n_steps == 6
    init = W.avalanche_initial(w)
    _note(f"avalanche: {w.description}")
    e = R.engine_single(w, init, same_step=True)
    p = R.params_of(w, same_step_generations=16)
    op = oracle_params(orc, w, same_step_generations=16)
    os_ = oracle_stores(orc, init, w.capacity)
    first = 2
    stats = R.run(e, R.field_of(w), p, first)
    ostats = orc.run(os_, oracle_field(orc, w), op, first)
    _check_steps(stats, ostats, label="avalanche, two steps")
    assert sum(s["emitted"] for s in stats) > 100
    compare_all(e, os_, label="avalanche, two steps")
    stats += R.run(e, R.field_of(w), p, w.n_steps - first, first_step=first)
    for n in range(first, w.n_steps):
        op.step = n
        ostats.append(orc.step(os_, oracle_field(orc, w), op))
    # the problem's own conditioning: the oracle again with the amplitude one ulp larger
    f_ulp = oracle_field(orc, w)
    f_ulp.amp = f_ulp.amp * (1.0 + 2.0 ** -52)
    ou = oracle_stores(orc, init, w.capacity)
    ustats = orc.run(ou, f_ulp, oracle_params(orc, w, same_step_generations=16), w.n_steps)
    spreads = []
    for sp in range(3):
        spread = compare_species(ou[sp].view(), os_[sp].view(), sp, rtol=1.0, label="ulp")
        spreads.append(max(spread.values()))
    for a, b in zip(ustats, ostats):
        for f in ("photon_energy", "max_p_emit", "max_p_pair"):
            if b[f] > 0:
                spreads.append(abs(a[f] - b[f]) / b[f])
    tol = max(1e-12, 10.0 * max(spreads))
    _note(f"one-ulp spread {max(spreads):.2e}, tolerance {tol:.2e}")
    for c in COUNTERS:
        assert [s[c] for s in ustats] == [s[c] for s in ostats], c
    for c in COUNTERS:
        assert [s[c] for s in stats] == [s[c] for s in ostats], c
    compare_stats(stats, ostats, label="avalanche, six steps", float_rtol=tol)
    assert sum(s["pairs"] for s in stats) > 200
    for sp in range(3):
        compare_species(e.read(0, sp), os_[sp].view(), sp, rtol=tol, label=f"avalanche {sp}")


def test_same_step_with_generator_factors_parity(orc):
    """Children advanced in their birth step (G = 3) together with generator factors f_g = 3
    for photons and 2 for pairs (Sec. VI): the generation kernel samples its own children's
    creation the way the step does, and the parents' weights carry through."""
    w = W.rotating_e(n=300, periods=1.5, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    over = dict(same_step_generations=3, f_photon=3.0, f_pair=2.0)
    _note(f"rotating cascade, {over}")
    e = R.engine_single(w, init, same_step=True)
    stats = R.run(e, R.field_of(w), R.params_of(w, **over), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, **over), w.n_steps)
    _check_steps(stats, ostats, label="same-step with generator factors")
    assert sum(s["children_advanced"] for s in stats) > 1000
    assert sum(s["pairs"] for s in stats) > 5
    compare_all(e, os_, label="same-step with generator factors")


def test_batched_instances_same_step_parity(orc):
    """Four instances of different size, amplitude and seed (one empty) in one launch, with
    children advanced in their birth step (G = 2): the generation passes keep every
    instance's children in its own segment, and each instance equals its own oracle run."""
    w = W.batched_rotating(instances=4, a_lo=600.0, a_hi=2400.0, periods=0.75,
                           n_override=[37, 0, 129, 200], total_capacity=4 * 400_000,
                           precision="f64")
    inits = W.batched_initial(w)
    _note(f"batched same-step: {w.description}")
    e = R.engine_batched(w, inits, same_step=True)
    st = R.run(e, R.field_of(w), R.params_of(w, same_step_generations=2), w.n_steps,
               stop_on_drop=False)
    assert sum(s["dropped"] for s in st) == 0
    assert sum(s["children_advanced"] for s in st) > 100
    per = []
    for i in range(w.instances):
        wi = W.rotating_e(n=w.instance_n[i], a0=w.instance_amp[i], periods=0.75, seed=i,
                          capacity=w.instance_capacity[2],
                          lepton_capacity=w.instance_capacity[1])
        os_ = oracle_stores(orc, inits[i], w.instance_capacity)
        per.append(orc.run(os_, oracle_field(orc, wi),
                           oracle_params(orc, wi, same_step_generations=2), w.n_steps))
        compare_all(e, os_, inst=i, label=f"instance {i}")
    compare_stats(st, merge_stats(per), label="batched same-step")


def test_mixed_precision_same_step_follows_fp64():
    """The mixed form (rate and decision in FP32) with same-step children (G = 2): both forms
    draw the same numbers, so only decisions within FP32 rounding of the threshold can
    differ, and the cascade's totals stay within 1% of the FP64 run's."""
    w = W.rotating_e(n=300, periods=1.5, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    tot = {}
    for prec in ("f64", "mixed"):
        _note(f"same-step G = 2, {prec}")
        e = R.engine_single(w, init, same_step=True)
        st = R.run(e, R.field_of(w),
                   R.params_of(w, same_step_generations=2, precision=R.PRECISION[prec]),
                   w.n_steps)
        tot[prec] = np.array([sum(s[c] for s in st)
                              for c in ("emitted", "pairs", "children_advanced")], float)
    assert tot["f64"][1] > 50
    np.testing.assert_allclose(tot["mixed"], tot["f64"], rtol=1e-2)
