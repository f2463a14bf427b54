"""GPU same-step processing (children advanced through the rest of their birth step, Sec.
IV.H) against the oracle: every store to the parity bar of the other cascade tests (ids,
parents, births, event counts and weights bit-exact, momenta and positions within 1e-12),
and per step the photons and pairs created, the children advanced in their birth step and
the children deferred to the next one."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import (compare_all, compare_species, oracle_field, oracle_params,
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


def _check_steps(stats, ostats):
    assert len(stats) == len(ostats)
    for c in COUNTERS:
        assert [s[c] for s in stats] == [s[c] for s in ostats], c
    assert sum(s["near_threshold"] for s in stats) == 0


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
    _check_steps(stats, ostats)
    assert sum(s["children_advanced"] for s in stats) > 10_000
    compare_all(e, os_, label=f"rotating G={G}")


@pytest.mark.parametrize("G", [4, 16])
def test_shower_same_step_parity(orc, G):
    """The Sec. VII shower at a large step (20 seeds, dt = 25000, about 400 lepton
    sub-steps a step, kappa = 0.25, three steps): many generations in every step; with
    G = 4 part of them waits for the next step.  Momenta and positions are compared within
    1e-12 of the cascade's scales, gamma_0 m c and c t: a lepton that radiates almost all
    of its energy keeps p (1 - f) with f near 1, and there the GPU's fused multiply-adds
    and the oracle's separately rounded products leave remainders that differ by a few
    1e-12 of themselves (2.5e-12 seen) while agreeing to 1e-14 of gamma_0."""
    w = W.shower(n=20, steps=3)
    init = W.shower_initial(w)
    _note(f"shower, G = {G}: {w.description}")
    e = R.engine_single(w, init, same_step=True)
    stats = R.run(e, R.field_of(w), R.params_of(w, same_step_generations=G), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, same_step_generations=G),
                     w.n_steps)
    _check_steps(stats, ostats)
    assert sum(s["pairs"] for s in stats) > 100
    if G == 4:
        assert sum(s["deferred"] for s in stats) > 0
    compare_all(e, os_, label=f"shower G={G}", floor=(W.SHOWER_GAMMA0, w.dt * w.n_steps))


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
    _check_steps(stats, ostats)
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
    _check_steps(stats, ostats)
    assert sum(s["children_advanced"] for s in stats) == 0
    compare_all(e, os_, label="G=0")


def test_avalanche_same_step_parity(orc):
    """The Sec. VII avalanche at its large step (20 seeds, dt = 173 t_rad, about T / 8, in
    the linearly polarised standing wave): position-dependent fields that children
    inherit, a cascade that grows tenfold per period.  The avalanche is chaotic: a change of
    one ulp in the field amplitude changes the oracle's own event counts at the eighth step
    and its momenta by up to about 1e-8 (photons 1e-6) after six (device sincos and libm
    sin, cos differ by about an ulp).  So six steps, with every decision, id and weight
    bit-exact, and momenta and positions within ten times the spread that the one-ulp
    change makes in the oracle itself (at least 1e-12)."""
    w = W.avalanche(n=20, dt_over_t_rad=173.0, periods=0.75)
    assert w.n_steps == 6
    init = W.avalanche_initial(w)
    _note(f"avalanche: {w.description}")
    e = R.engine_single(w, init, same_step=True)
    stats = R.run(e, R.field_of(w), R.params_of(w, same_step_generations=16), w.n_steps)
    op = oracle_params(orc, w, same_step_generations=16)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), op, w.n_steps)
    # the problem's own conditioning: the oracle again with the amplitude one ulp larger
    f_ulp = oracle_field(orc, w)
    f_ulp.amp = f_ulp.amp * (1.0 + 2.0 ** -52)
    ou = oracle_stores(orc, init, w.capacity)
    ustats = orc.run(ou, f_ulp, oracle_params(orc, w, same_step_generations=16), w.n_steps)
    _check_steps(stats, ostats)
    _check_steps(ustats, ostats)
    assert sum(s["pairs"] for s in stats) > 200
    for sp in range(3):
        spread = compare_species(ou[sp].view(), os_[sp].view(), sp, rtol=1.0, label="ulp")
        tol = max(1e-12, 10.0 * max(spread.values()))
        _note(f"species {sp}: one-ulp spread {max(spread.values()):.2e}, tolerance {tol:.2e}")
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
    _check_steps(stats, ostats)
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
    for i in range(w.instances):
        wi = W.rotating_e(n=w.instance_n[i], a0=w.instance_amp[i], periods=0.75, seed=i,
                          capacity=w.instance_capacity[2],
                          lepton_capacity=w.instance_capacity[1])
        os_ = oracle_stores(orc, inits[i], w.instance_capacity)
        orc.run(os_, oracle_field(orc, wi), oracle_params(orc, wi, same_step_generations=2),
                w.n_steps)
        compare_all(e, os_, inst=i, label=f"instance {i}")


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
