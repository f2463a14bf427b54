"""GPU (HIP, through the C ABI) vs the FP64 CPU oracle, element by element.

Integers (ids, parent ids, birth codes, event counts, counts of removed photons) must be
bit-exact; momenta agree within 1e-12 of each particle's own |p|, positions within 1e-12 of
max(|x|, 1); weights exactly.  Every field of the per-step record equals the oracle's (the
counters and both histograms exactly, the radiated energy and the largest probabilities to
1e-12).  The near-threshold counter reports decisions within 1e-12 of their acceptance
probability, the only ones allowed to flip (none did in these cases)."""
import math

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

from paper_1412_6426_amd import qed as Q  # noqa: E402
from paper_1412_6426_amd import runner as R  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402
from paper_1412_6426_amd.engine import Engine  # noqa: E402


def _note(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------------------
def test_tables_match_oracle(orc):
    _note("tables")
    e = Engine([(1, 1, 1)], [0])
    e.build_tables()
    torch.cuda.synchronize()
    raw = e.tables.cpu().numpy()
    ab = raw[0:65536].view(np.float64).reshape(4096, 2)
    bc = raw[65536:131072].view(np.float64).reshape(4096, 2)
    ab32 = raw[131072:163840].view(np.float32).reshape(4096, 2)
    bound = raw[196608:212992].view(np.float64).reshape(128, 16)
    bound32 = raw[212992:221184].view(np.float32).reshape(128, 16)
    series = raw[221184:221248].view(np.float64)
    magic = raw[221248:221252].view(np.uint32)[0]
    gA, gB, gC = orc.table_arrays()
    np.testing.assert_allclose(ab[:, 0], gA, rtol=1e-13, atol=0)
    np.testing.assert_allclose(ab[:, 1], gB, rtol=1e-13, atol=0)
    np.testing.assert_allclose(bc[:, 0], gB, rtol=1e-13, atol=0)
    np.testing.assert_allclose(bc[:, 1], gC, rtol=1e-13, atol=0)
    assert np.array_equal(ab32, ab.astype(np.float32))
    t = orc.tables()
    np.testing.assert_allclose(series[:5], [t.s_b0, t.s_b1, t.s_c0, t.s_c1, t.s_c2], rtol=1e-14)
    assert magic == 0x51454454
    assert np.array_equal(bound32, bound.astype(np.float32))
    # each sub-octave bound really bounds the pair bracket at its interval's top chi
    # (oracle, exact rates), and the bounds grow with chi
    d = np.linspace(1e-4, 0.5, 2000)
    for e in (40, 55, 62, 64, 66, 70, 80):
        for j in (0, 7, 15):
            chi = (0.5 + (j + 1) / 32.0) * 2.0 ** (e - 64)
            brk = [orc.rate_pair(x, chi, 1.0, 1.0, orc.EXACT) * math.sqrt(3) * math.pi
                   for x in d]
            assert max(brk) <= bound[e, j]
    flat = bound.reshape(-1)
    assert np.all(np.diff(flat[flat > 0]) >= 0)


def test_uniform_b_full_size_parity(orc):
    """Uniform static B, 10^4 electrons at gamma = 1000 (chi = 1), dt = T_gyro/100,
    100 steps, emission only, photons recorded: the whole run, both stores."""
    w = W.uniform_b()
    init = W.uniform_b_initial(w)
    _note(f"uniform_b full: {w.description}")
    e = R.engine_single(w, init)
    stats = R.run(e, R.field_of(w), R.params_of(w), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w), w.n_steps)
    assert sum(s["near_threshold"] for s in stats) == 0
    assert all(s["nsub_hist"][8] == 10_000 for s in stats)
    compare_stats(stats, ostats, label="uniform_b")
    # pure magnetic field: a lepton is held to its momentum at birth (|p| plus the |k| it
    # emitted), the scale of the rounding left in p (1 - f) when it radiates nearly all of it
    birth = lepton_birth_momentum(os_[2].view())
    compare_all(e, os_, label="uniform_b", p_scale=(birth, birth, None))
    assert sum(s["saturated"] for s in stats) == 0 and stats[-1]["status"] == 0


# Child appends: through the per-wavefront arenas (default), with an arena so small that
# most children take the direct-reservation path, and with no arena at all.
ARENA_MODES = {"arena": None, "tiny_arena": 5000, "no_arena": 0}


@pytest.mark.parametrize("arena", list(ARENA_MODES))
def test_rotating_cascade_parity(orc, arena):
    """Rotating-E cascade (a0 = 1000, lambda = 0.8 um, dt = T/200) from 300 seeds through
    300 steps: emission, pairs, photon push; every store compared."""
    w = W.rotating_e(n=300, periods=1.5, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    _note(f"rotating cascade ({arena}): {w.description}")
    e = R.engine_single(w, init, arena_records=ARENA_MODES[arena])
    stats = R.run(e, R.field_of(w), R.params_of(w), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w), w.n_steps)
    assert len(stats) == len(ostats) == w.n_steps
    assert sum(s["pairs"] for s in stats) > 20
    assert [s["pairs"] for s in stats] == [s["pairs"] for s in ostats]
    assert [s["emitted"] for s in stats] == [s["emitted"] for s in ostats]
    assert sum(s["near_threshold"] for s in stats) == 0
    compare_stats(stats, ostats, label=f"rotating ({arena})")
    compare_all(e, os_, label="rotating")


@pytest.mark.parametrize("arena", ["arena", "no_arena"])
def test_generator_factor_cascade_parity(orc, arena):
    """The rotating-E cascade with generator factors f_g = 3 for photons and 2 for pairs
    (Sec. VI): every store bit-exact against the oracle (weights too: f_g times the
    parent's), per-step created photons and pairs equal, and fewer photons than events."""
    w = W.rotating_e(n=300, periods=1.5, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    over = dict(f_photon=3.0, f_pair=2.0)
    _note(f"generator factors {over} ({arena})")
    e = R.engine_single(w, init, arena_records=ARENA_MODES[arena])
    stats = R.run(e, R.field_of(w), R.params_of(w, **over), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ostats = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, **over), w.n_steps)
    assert len(stats) == len(ostats) == w.n_steps
    assert sum(s["pairs"] for s in stats) > 5
    assert [s["pairs"] for s in stats] == [s["pairs"] for s in ostats]
    compare_stats(stats, ostats, label="generator factors")
    compare_all(e, os_, label="generator factors")
    lep = [e.read(0, s) for s in (0, 1)]
    events = int(sum(v["n_events"].sum() for v in lep))
    created = len(e.read(0, 2)["id"])
    assert created < events  # some events created no photon
    g = e.read(0, 2)
    seeds = g["parent"] < np.uint64(300)
    assert np.all(g["w"][seeds] == 3.0)  # seeds have weight 1


def test_forced_substeps_and_nonadaptive(orc):
    w = W.rotating_e(n=97, periods=0.25, capacity=50_000, lepton_capacity=5000)
    init = W.rotating_e_initial(97, seed=9)
    for over in (dict(forced_substeps=5), dict(adaptive=0)):
        _note(f"substep variant {over}")
        e = R.engine_single(w, init)
        st = R.run(e, R.field_of(w), R.params_of(w, **over), w.n_steps)
        os_ = oracle_stores(orc, init, w.capacity)
        ost = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w, **over), w.n_steps)
        compare_stats(st, ost, label=str(over))
        compare_all(e, os_, label=str(over))


def test_empty_and_single_particle(orc):
    w = W.rotating_e(n=1, periods=0.1, capacity=1000, lepton_capacity=100)
    _note("empty store")
    e = R.engine_single(w, [W.empty_columns()] * 3)
    st = R.run(e, R.field_of(w), R.params_of(w), 3)
    assert st[-1]["counts"] == [[0, 0, 0]] and st[-1]["substeps"] == 0
    assert int(e.step_ctr.item()) == 3
    _note("single particle")
    init = W.rotating_e_initial(1, seed=1)
    e = R.engine_single(w, init)
    st = R.run(e, R.field_of(w), R.params_of(w), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ost = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w), w.n_steps)
    compare_stats(st, ost, label="single")
    compare_all(e, os_, label="single")


@pytest.mark.parametrize("arena", list(ARENA_MODES))
def test_capacity_overflow_is_counted_and_contained(orc, arena):
    """Tiny photon capacity: drops counted, count clamped, nothing written past the
    instance's segment (a guard instance after it keeps its contents)."""
    w = W.uniform_b(n=500, steps=2)
    init = W.uniform_b_initial(w)
    _note(f"capacity overflow ({arena})")
    e = Engine([(500, 1, 40), (1, 1, 64)], [0, 1], arena_records=ARENA_MODES[arena])
    e.build_tables()
    for s in range(3):
        e.load(0, s, init[s])
    guard = W._seed_columns(*[np.full(64, 7.0)] * 6)
    guard["n_events"] = np.zeros(64, np.uint32)
    e.load(1, 2, guard)
    st = R.run(e, R.field_of(w), R.params_of(w), 1)
    assert st[0]["dropped"] > 0 and st[0]["status"] & Q.QED_STATUS_DROPPED
    inst = e.instances()
    assert inst[0]["count"][2] == 40 and inst[0]["dropped"] == st[0]["dropped"]
    g = e.read(1, 2)
    assert np.all(g["x"] == 7.0) and np.all(g["pz"] == 7.0)
    assert st[0]["emitted"] == 40 + st[0]["dropped"]


def test_failure_counters(orc):
    w = W.uniform_b(n=20, steps=1)
    init = W.uniform_b_initial(w)
    init[0]["px"] = init[0]["px"].copy()
    init[0]["px"][3] = np.nan
    _note("nonfinite")
    e = R.engine_single(w, init)
    st = R.run(e, R.field_of(w), R.params_of(w), 1)
    assert st[0]["nonfinite"] > 0 and st[0]["status"] & Q.QED_STATUS_NONFINITE
    _note("saturation")
    e = R.engine_single(w, W.uniform_b_initial(w))
    p = R.params_of(w, adaptive=0, dt=50 * w.dt)
    st = R.run(e, R.field_of(w), p, 1)
    assert st[0]["saturated"] > 0 and st[0]["status"] & Q.QED_STATUS_SATURATED
    _note("tables not built")
    e = R.engine_single(w, W.uniform_b_initial(w), build_tables=False)
    st = R.run(e, R.field_of(w), R.params_of(w), 1)
    assert st[0]["status"] & Q.QED_STATUS_NO_TABLES and st[0]["substeps"] == 0


def _batched_oracle(orc, w, inits, i, periods):
    wi = W.rotating_e(n=w.instance_n[i], a0=w.instance_amp[i], periods=periods, seed=i,
                      capacity=w.instance_capacity[2], lepton_capacity=w.instance_capacity[1])
    os_ = oracle_stores(orc, inits[i], w.instance_capacity)
    ost = orc.run(os_, oracle_field(orc, wi), oracle_params(orc, wi), w.n_steps)
    return os_, ost


@pytest.mark.parametrize("arena", ["arena", "no_arena"])
def test_batched_instances_match_single_runs(orc, arena):
    """Five instances of different size, amplitude and seed (one empty) in one launch:
    each equals its own oracle run."""
    w = W.batched_rotating(instances=5, a_lo=600.0, a_hi=2400.0, periods=0.75,
                           n_override=[37, 0, 129, 64, 200], total_capacity=5 * 400_000,
                           precision="f64")
    inits = W.batched_initial(w)
    _note(f"batched ({arena}): {w.description}")
    e = R.engine_batched(w, inits, arena_records=ARENA_MODES[arena])
    st = R.run(e, R.field_of(w), R.params_of(w), w.n_steps, stop_on_drop=False)
    assert sum(s["dropped"] for s in st) == 0
    per = []
    for i in range(w.instances):
        os_, ost = _batched_oracle(orc, w, inits, i, 0.75)
        per.append(ost)
        compare_all(e, os_, inst=i, label=f"instance {i}")
    compare_stats(st, merge_stats(per), label="batched")


def test_batched_freeze_on_drop(orc):
    """An instance that runs out of photon slots freezes after that step; the others keep
    going and still equal their oracle runs."""
    w = W.batched_rotating(instances=3, a_lo=700.0, a_hi=2400.0, periods=0.75,
                           n_override=[50, 40, 200], total_capacity=3 * 30_000,
                           precision="f64")
    inits = W.batched_initial(w)
    _note("batched freeze")
    e = R.engine_batched(w, inits)
    st = R.run(e, R.field_of(w), R.params_of(w), w.n_steps, stop_on_drop=False)
    inst = e.instances()
    assert inst[2]["dropped"] > 0 and inst[2]["frozen"] == 1
    assert inst[2]["count"][2] == w.instance_capacity[2]
    first = next(k for k, s in enumerate(st) if s["dropped"] > 0)
    assert first < w.n_steps - 1  # the freeze is exercised for at least one step
    for i in (0, 1):
        assert inst[i]["frozen"] == 0
        os_, _ = _batched_oracle(orc, w, inits, i, 0.75)
        compare_all(e, os_, inst=i, label=f"instance {i}")
    # the frozen instance equals the oracle stopped at the same step, up to which
    # children were dropped: compare its leptons (unaffected by photon drops)
    os_, ost = _batched_oracle(orc, w, inits, 2, 0.75)
    assert len(ost) == first + 1
    compare_species(e.read(2, 0), os_[0].view(), 0, label="frozen e-")
    compare_species(e.read(2, 1), os_[1].view(), 1, label="frozen e+")


def test_runs_are_reproducible(orc):
    w = W.rotating_e(n=500, periods=0.6, capacity=100_000, lepton_capacity=10_000)
    init = W.rotating_e_initial(500, seed=4)
    outs = []
    for rep, tile in enumerate((64, 128, 64)):
        _note(f"determinism run {rep}")
        e = R.engine_single(w, init)
        R.run(e, R.field_of(w), R.params_of(w, tile=tile), w.n_steps)
        outs.append([e.read(0, s) for s in range(3)])
    for s in range(3):
        compare_species(outs[0][s], outs[1][s], s, rtol=0.0, label="rerun")
        # with the child arenas the store order itself is fixed by the work distribution
        for c, v in outs[0][s].items():
            assert np.array_equal(v, outs[2][s][c], equal_nan=True), (s, c)


def test_stats_log_and_graph_replay(orc):
    """Steps captured once in a hipGraph and replayed equal eager steps; qed_append_stats
    appends one record per replay."""
    w = W.rotating_e(n=400, periods=0.5, capacity=100_000, lepton_capacity=10_000)
    init = W.rotating_e_initial(400, seed=5)
    _note("eager reference")
    ref = R.engine_single(w, init)
    R.run(ref, R.field_of(w), R.params_of(w), w.n_steps)
    _note("graph replay")
    e = R.engine_single(w, init)
    log = torch.zeros((w.n_steps + 5) * e.stats_buf.numel(), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    f, p = R.field_of(w), R.params_of(w)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        e.step(f, p, stream=s.cuda_stream)  # warm-up outside the graph
        Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), w.n_steps + 5,
                           cnt.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        e.step(f, p, stream=s.cuda_stream)
        Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), w.n_steps + 5,
                           cnt.data_ptr(), s.cuda_stream)
    for _ in range(w.n_steps - 1):
        g.replay()
        torch.cuda.synchronize()
    assert int(cnt.item()) == w.n_steps
    assert int(e.step_ctr.item()) == w.n_steps
    for sp in range(3):
        compare_species(e.read(0, sp), ref.read(0, sp), sp, rtol=0.0, label="graph")
    recs = log.cpu().numpy()[:w.n_steps * e.stats_buf.numel()].view(np.int64)
    steps = recs.reshape(w.n_steps, -1)[:, 0]
    assert list(steps) == list(range(w.n_steps))


def test_yee_grid_parity(orc):
    """Standing-wave cascade on a small periodic Yee grid (32^3, lambda/32 cells): the
    same FP32 grid values (sampled at every t_n) feed both sides."""
    w = W.standing_wave_grid(n=300, cells=32, capacity=200_000, lepton_capacity=20_000,
                             steps=40, a0=2000.0)
    init = W.standing_wave_initial(300, seed=2)
    _note(f"yee grid: {w.description}")
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
        e.step(f, p)
        torch.cuda.synchronize()
        st.append(e.stats())
        op.step = n
        ost.append(orc.step(os_, oracle_field(orc, w, grids=vals), op))
    assert e.stats()["n_start"][2] > 100
    compare_stats(st, ost, label="yee")
    compare_all(e, os_, label="yee")


def test_yee_grid_random_values_every_wrap(orc):
    """A non-cubic 7x5x4 grid of seeded random values (so every node and every component
    differs) and particles spread over three box lengths per axis, so that positions
    inside, beyond and before the primary box all wrap, and many sit in the last cell of
    a row, where the x-neighbour pair straddles the periodic boundary."""
    import dataclasses
    w = W.standing_wave_grid(n=400, cells=8, capacity=50_000, lepton_capacity=5_000,
                             steps=3, a0=2000.0)
    fs = dataclasses.replace(w.field, grid_n=(7, 5, 4), grid_origin=(-1.3, 0.4, 2.2))
    w = dataclasses.replace(w, field=fs)
    nx, ny, nz = fs.grid_n
    rng = np.random.default_rng(11)
    lo = np.array(fs.grid_origin) - np.array(fs.grid_n) * np.array(fs.grid_dx)
    span = 3.0 * np.array(fs.grid_n) * np.array(fs.grid_dx)
    n = 400
    pos = lo[:, None] + span[:, None] * rng.random((3, n))
    # a quarter of the particles in the last cell along x (the wrapping pair)
    q = n // 4
    pos[0, :q] = fs.grid_origin[0] + (nx - 1 + rng.random(q)) * fs.grid_dx[0]
    init = W.standing_wave_initial(n, seed=3)
    for k, c in enumerate(("x", "y", "z")):
        init[0][c] = pos[k].copy()
    init[0]["px"] = rng.normal(0.0, 300.0, n)
    init[0]["py"] = rng.normal(0.0, 300.0, n)
    init[0]["pz"] = rng.normal(0.0, 300.0, n)
    _note(f"yee random grid {fs.grid_n}: {n} electrons, {w.n_steps} steps")
    e = R.engine_single(w, init)
    grid = R.YeeGrid(w)
    f = R.field_of(w, grid=grid.g)
    p = R.params_of(w)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w)
    e.set_step(0)
    st, ost = [], []
    for step in range(w.n_steps):
        vals = [(1500.0 * rng.standard_normal((nz, ny, nx))).astype(np.float32) for _ in range(6)]
        grid.load_numpy(vals)
        e.step(f, p)
        torch.cuda.synchronize()
        st.append(e.stats())
        op.step = step
        ost.append(orc.step(os_, oracle_field(orc, w, grids=vals), op))
    compare_stats(st, ost, label="yee-random")
    compare_all(e, os_, label="yee-random")


def test_fill_standing_wave_matches_numpy():
    w = W.standing_wave_grid(n=1, cells=16)
    grid = R.YeeGrid(w)
    t = 0.37
    grid.fill(t, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want = W.standing_wave_grid_values(w.field, t)
    for g, v in zip(grid.g, want):
        np.testing.assert_allclose(g.cpu().numpy(), v, rtol=2e-7, atol=1e-3)


# ---------------------------------------------------------------------------------------
# Full size: the rotating-field cascade of the benchmark (10^5 seeds, 10^8 slots per store,
# the benchmark's launch configuration) advanced to step 400 on the GPU; then one more step,
# checked on a random sample of particles that the oracle steps one by one.  Particles are
# independent given the fields, and every draw and child id is keyed by the particle, so
# the sample's next state and its children do not depend on the rest of the store.
def _gather(e, sp, idx):
    t = torch.as_tensor(idx, dtype=torch.int64, device=e.device)
    d = e.cols[sp]
    out = {c: d[c][t].cpu().numpy() for c in ("x", "y", "z", "px", "py", "pz", "w")}
    out["id"] = d["id"][t].cpu().numpy().view(np.uint64)
    out["parent"] = d["parent"][t].cpu().numpy().view(np.uint64)
    out["birth"] = d["birth"][t].cpu().numpy().view(np.uint32)
    out["n_events"] = d["n_events"][t].cpu().numpy().view(np.uint32)
    return out


def test_full_size_sampled_parity(orc):
    w = W.rotating_e(n=100_000, a0=1000.0, periods=3.0, capacity=100_000_000)
    init = W.rotating_e_initial(100_000, seed=0)
    _note("full size: 400 steps of the benchmark cascade")
    e = R.engine_single(w, init)
    field, params = R.field_of(w), R.params_of(w, freeze_on_drop=1)
    n = 400
    st = R.run(e, field, params, n)
    assert sum(s["dropped"] for s in st) == 0
    c0 = e.counts()[0]
    assert c0[0] > 1_000_000 and c0[2] > 10_000_000
    rng = np.random.default_rng(2024)
    sample = {}
    for sp, k in ((0, 3000), (1, 3000), (2, 30000)):
        idx = np.sort(rng.choice(int(c0[sp]), size=k, replace=False))
        cols = _gather(e, sp, idx)
        if sp == 2:
            live = cols["id"] != W.NO_PARENT
            idx = idx[live]
            cols = {c: v[live] for c, v in cols.items()}
        sample[sp] = (idx, cols)
    _note("full size: step 400 and the sample's oracle step")
    e.step(field, params)
    torch.cuda.synchronize()
    c1 = e.counts()[0]
    os_ = [orc.Store(200_000), orc.Store(200_000), orc.Store(400_000, with_events=False)]
    for sp in range(3):
        cols = dict(sample[sp][1])
        if sp == 2:
            cols.pop("n_events")
        os_[sp].load(cols)
    p = oracle_params(orc, w)
    p.step = n
    orc.step(os_, oracle_field(orc, w), p)
    for sp in range(3):
        idx, before = sample[sp]
        m = len(idx)
        got = _gather(e, sp, idx)
        want = os_[sp].view()
        want = {c: (v[:m] if v is not None else None) for c, v in want.items()}
        if sp == 2:
            got.pop("n_events")
            want.pop("n_events", None)
            assert np.array_equal(got["id"], want["id"]), "photons removed by pairs differ"
        compare_species(got, want, sp, label=f"sampled species {sp}")
    # children of the sampled particles, created during step 400
    parents = {0: set(), 2: set()}
    parents[0] = set(sample[0][1]["id"].tolist()) | set(sample[1][1]["id"].tolist())
    parents[2] = set(sample[2][1]["id"].tolist())
    for sp in range(3):
        lo, hi = int(c0[sp]), int(c1[sp])
        region = _gather(e, sp, np.arange(lo, hi))
        keep = np.isin(region["parent"], np.array(sorted(parents[0 if sp == 2 else 2]),
                                                   dtype=np.uint64))
        got = {c: v[keep] for c, v in region.items()}
        m = len(sample[sp][0])
        wv = os_[sp].view()
        want = {c: (v[m:] if v is not None else None) for c, v in wv.items()}
        if sp == 2:
            got.pop("n_events")
            want.pop("n_events", None)
        assert len(got["id"]) == len(want["id"]), f"children of species {sp}"
        compare_species(got, want, sp, label=f"children species {sp}")
    assert len(os_[2].view()["id"]) > len(sample[2][0])  # the sample did emit


def _spectrum(cols, lo=W.SPECTRUM_LO, hi=W.SPECTRUM_HI, bins=W.SPECTRUM_BINS):
    live = cols["id"] != W.NO_PARENT
    e = np.sqrt(cols["px"][live] ** 2 + cols["py"][live] ** 2 + cols["pz"][live] ** 2)
    u = (np.log10(e) - math.log10(lo)) * bins / (math.log10(hi) - math.log10(lo))
    ok = (u >= 0) & (u < bins)
    return np.bincount(u[ok].astype(np.int64), weights=cols["w"][live][ok], minlength=bins)


def test_mixed_precision_spectrum_and_pair_yield(orc):
    """Mixed precision (FP32 tables and sampling, FP64 chi and push) against the FP64
    oracle on the rotating-field cascade from 10^3 seeds over two periods: photon spectrum
    (130 log bins of eps in [1e-8, 1e5]) within L1 1e-3 and pair yield within 1%.  The FP64
    GPU run gives the oracle's spectrum and pair count, and qed_photon_spectrum agrees with
    the histogram of the stores read back."""
    w = W.rotating_e(n=1000, periods=2.0, capacity=4_000_000, lepton_capacity=400_000)
    init = W.rotating_e_initial(1000, seed=21)
    os_ = oracle_stores(orc, init, w.capacity)
    ost = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w), w.n_steps)
    assert sum(s["dropped"] for s in ost) == 0
    h_or = _spectrum(os_[2].view())
    p_or = sum(s["pairs"] for s in ost)
    assert p_or > 1000
    for prec in ("f64", "mixed"):
        _note(f"precision {prec}")
        wp = W.rotating_e(n=1000, periods=2.0, capacity=4_000_000, lepton_capacity=400_000,
                          precision=prec)
        e = R.engine_single(wp, init)
        st = R.run(e, R.field_of(wp), R.params_of(wp), wp.n_steps)
        cols = e.read(0, 2)
        h = _spectrum(cols)
        d = torch.zeros(W.SPECTRUM_BINS, dtype=torch.float64, device="cuda")
        Q.qed_photon_spectrum(e.stores, W.SPECTRUM_LO, W.SPECTRUM_HI, W.SPECTRUM_BINS,
                              d.data_ptr(), e.stream)
        torch.cuda.synchronize()
        assert np.allclose(d.cpu().numpy(), h, rtol=1e-12, atol=0)
        l1 = float(np.abs(h - h_or).sum() / h_or.sum())
        pairs = sum(s["pairs"] for s in st)
        _note(f"{prec}: L1 {l1:.3e}, pairs {pairs} vs {p_or}")
        if prec == "f64":
            assert l1 <= 1e-9 and pairs == p_or
        else:
            assert l1 <= 1e-3
            assert abs(pairs - p_or) <= 0.01 * p_or


def test_yee_grid_mixed_precision_follows_fp64_oracle(orc):
    """The mixed form on the 32^3 Yee-grid cascade (its own photon and lepton kernels, with
    the same FP32 grid gathers) against the FP64 oracle: both draw the same numbers, so only
    decisions within FP32 rounding of a threshold differ; emissions and live photons within
    1%, the photon spectrum within L1 1e-2."""
    w = W.standing_wave_grid(n=300, cells=32, capacity=200_000, lepton_capacity=20_000,
                             steps=40, a0=2000.0, precision="mixed")
    init = W.standing_wave_initial(300, seed=2)
    _note(f"yee grid, mixed: {w.description}")
    e = R.engine_single(w, init)
    grid = R.YeeGrid(w)
    f = R.field_of(w, grid=grid.g)
    p = R.params_of(w)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w)
    emitted_gpu = emitted_or = 0
    e.set_step(0)
    for n in range(w.n_steps):
        vals = W.standing_wave_grid_values(w.field, w.t0 + n * w.dt)
        grid.load_numpy(vals)
        e.step(f, p)
        torch.cuda.synchronize()
        emitted_gpu += e.stats()["emitted"]
        op.step = n
        emitted_or += orc.step(os_, oracle_field(orc, w, grids=vals), op)["emitted"]
    assert emitted_or > 1000
    assert abs(emitted_gpu - emitted_or) <= 0.01 * emitted_or
    h_or = _spectrum(os_[2].view())
    h = _spectrum(e.read(0, 2))
    assert abs(h.sum() - h_or.sum()) <= 0.01 * h_or.sum()
    l1 = float(np.abs(h - h_or).sum() / h_or.sum())
    _note(f"mixed yee: emitted {emitted_gpu} vs {emitted_or}, L1 {l1:.3e}")
    assert l1 <= 1e-2


def test_checkpoint_resume_is_bit_exact(orc):
    """A cascade stopped after 60 steps, its stores read back to the host (the checkpoint)
    and loaded into a fresh engine that continues from step 60, ends bit-identical to the
    uninterrupted run, store order included: every draw is keyed by (id, step, sub-step),
    and the state is the stores plus the step index."""
    w = W.rotating_e(n=400, periods=0.6, capacity=100_000, lepton_capacity=10_000)
    init = W.rotating_e_initial(400, seed=6)
    K = 60
    M = w.n_steps - K
    _note(f"resume: {K} + {M} steps")
    full = R.engine_single(w, init)
    R.run(full, R.field_of(w), R.params_of(w), w.n_steps)
    first = R.engine_single(w, init)
    R.run(first, R.field_of(w), R.params_of(w), K)
    ckpt = [first.read(0, s) for s in range(3)]
    del first
    resumed = R.engine_single(w, ckpt)
    st = R.run(resumed, R.field_of(w), R.params_of(w), M, first_step=K)
    assert sum(s["emitted"] for s in st) > 0
    for s in range(3):
        a, b = full.read(0, s), resumed.read(0, s)
        for c, v in a.items():
            assert np.array_equal(v, b[c], equal_nan=True), (s, c)


# ---------------------------------------------------------------------------------------
# The batched ensemble in its own precision: several rotating-field cascades of different
# amplitude and size in one mixed-precision launch, each against its own FP64 oracle run.
def _batched_mixed_workload():
    return W.batched_rotating(instances=3, a_lo=1000.0, a_hi=2000.0, periods=1.25,
                              n_override=[1500, 600, 150], total_capacity=3 * 4_000_000,
                              precision="mixed")


def test_batched_mixed_precision_against_oracle(orc):
    """Three cascades (a0 = 1000, 1414, 2000 from 1500, 600, 150 seeds, 1.25 periods) in one
    mixed-precision step (FP32 rates and decisions, FP64 chi, push and n_sub): per instance,
    against that instance's FP64 oracle run, the photon spectrum (130 weighted log bins of
    eps in [1e-8, 1e5]) within L1 1e-3 and the pair yield within 1%.  Both sides draw the
    same numbers, so only decisions within FP32 rounding of a threshold can differ."""
    w = _batched_mixed_workload()
    inits = W.batched_initial(w)
    _note(f"batched mixed: {w.description}")
    e = R.engine_batched(w, inits)
    st = R.run(e, R.field_of(w), R.params_of(w), w.n_steps, stop_on_drop=False)
    assert sum(s["dropped"] for s in st) == 0 and sum(s["saturated"] for s in st) == 0
    for i in range(w.instances):
        os_, ost = _batched_oracle(orc, w, inits, i, 1.25)
        h_or = _spectrum(os_[2].view())
        h = _spectrum(e.read(i, 2))
        l1 = float(np.abs(h - h_or).sum() / h_or.sum())
        pairs_or = sum(s["pairs"] for s in ost)
        pairs = len(e.read(i, 1)["id"])  # every positron comes from a pair
        _note(f"instance {i}: L1 {l1:.3e}, pairs {pairs} vs {pairs_or}")
        assert pairs_or > 1000
        assert l1 <= 1e-3
        assert abs(pairs - pairs_or) <= 0.01 * pairs_or


def test_batched_mixed_graph_replay_equals_eager(orc):
    """One mixed-precision batched step captured in a hipGraph and replayed step after step
    (with eager work and synchronisations between the replays) gives the same stores, store
    order included, and the same per-step records as the same steps run eagerly (the sum of
    the radiated energy to 1e-12: workgroups add their partial sums in any order)."""
    w = _batched_mixed_workload()
    inits = W.batched_initial(w)
    K = 120
    _note("batched mixed, eager")
    ref = R.engine_batched(w, inits)
    est = R.run(ref, R.field_of(w), R.params_of(w), K, stop_on_drop=False)
    _note("batched mixed, graph replay")
    e = R.engine_batched(w, inits)
    log = torch.zeros(K * e.stats_buf.numel(), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    f, p = R.field_of(w), R.params_of(w)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        e.step(f, p, stream=s.cuda_stream)
        Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), K, cnt.data_ptr(),
                           s.cuda_stream)
    # capture enqueued nothing: the store is still at its seeds
    assert int(e.step_ctr.item()) == 0 and int(cnt.item()) == 0
    for n in range(K):
        g.replay()
        torch.cuda.synchronize()
        assert e.counts().tolist() == est[n]["counts"]
    assert int(cnt.item()) == K
    recs = log.cpu().numpy().tobytes()
    size = e.stats_buf.numel()
    for n in range(K):
        r = Q.qed_stats.from_buffer_copy(recs[n * size:(n + 1) * size]).as_dict()
        for k, v in r.items():
            if isinstance(v, float):  # workgroup partial sums add up in any order
                assert abs(v - est[n][k]) <= 1e-12 * abs(est[n][k]), (n, k)
            else:
                assert v == est[n][k], (n, k)
    for i in range(w.instances):
        for sp in range(3):
            a, b = e.read(i, sp), ref.read(i, sp)
            for c, v in a.items():
                assert np.array_equal(v, b[c], equal_nan=True), (i, sp, c)


@pytest.mark.parametrize("refill", [1, 17, 64])
def test_refill_threshold_leaves_results_unchanged(orc, refill):
    """The lepton kernel's work-queue threshold (qed_params.refill_min) changes when idle
    lanes take new particles, not what happens to any particle: the rotating cascade and the
    32^3 Yee-grid cascade equal the oracle at thresholds 1, 17 and 64."""
    w = W.rotating_e(n=300, periods=1.0, capacity=400_000, lepton_capacity=40_000)
    init = W.rotating_e_initial(300, seed=3)
    _note(f"rotating cascade, refill_min {refill}")
    e = R.engine_single(w, init)
    st = R.run(e, R.field_of(w), R.params_of(w, refill_min=refill), w.n_steps)
    os_ = oracle_stores(orc, init, w.capacity)
    ost = orc.run(os_, oracle_field(orc, w), oracle_params(orc, w), w.n_steps)
    compare_stats(st, ost, label=f"rotating refill {refill}")
    compare_all(e, os_, label=f"rotating refill {refill}")
    w = W.standing_wave_grid(n=300, cells=32, capacity=200_000, lepton_capacity=20_000,
                             steps=30, a0=2000.0)
    init = W.standing_wave_initial(300, seed=2)
    _note(f"yee grid, refill_min {refill}")
    e = R.engine_single(w, init)
    grid = R.YeeGrid(w)
    f = R.field_of(w, grid=grid.g)
    p = R.params_of(w, refill_min=refill)
    os_ = oracle_stores(orc, init, w.capacity)
    op = oracle_params(orc, w)
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
    compare_stats(st, ost, label=f"yee refill {refill}")
    compare_all(e, os_, label=f"yee refill {refill}")
