#!/usr/bin/env python3
"""Benchmark of the GPU QED step on the rotating-electric-field cascade.

Workload (default): E = a0 (cos t, sin t, 0), B = 0, a0 = 1000, lambda = 0.8 um;
10^5 seed electrons at rest, uniform in a 1 um^3 box; emission + Breit-Wheeler pairs;
dt = T/200; 3 laser periods (600 steps); capacity 10^8 per species store.  One "step" is
one global time step of the whole hot path (fields, chi, adaptive sub-steps, Boris push,
emission and pair decisions, append) over every live particle.  The cascade grows until a
store is full; from then on the instance is frozen (its steps do nothing) and the run's
particle-step count stops growing.

Each GPU job runs three times from the same seeds: an untimed tuning run that picks the
launch shape (work-chunk size, persistent grid) per size class of the live count, the
timed run (one captured step graph per chosen shape, replayed for every step of the job),
and an eager run with HIP events around the lepton and photon kernels of every step.

`--steps K` times K steps of the 600-step job, the middle step of each of K equal parts,
with HIP events around each of them inside the timed run (the other steps replay untimed
between them); `value` is their particle-steps over their summed time, and the config lists
the steps.  Without --steps every step is timed.  The whole job's time and rate are in the
config too.  The roofline is taken over every launch of the dominant kernel in the eager
run.

Prints one JSON line: the headline and its roofline, and a short summary per further leg:
the same job in mixed precision with its photon-spectrum L1 distance and pair yield against
the FP64 job, the batched ensemble (64 rotating-field cascades, a0 log-spaced over
500-3000, 10^3-10^5 seeds each, 2 periods, 2*10^8 slots split evenly) as full jobs in mixed
precision and in FP64 with the same comparison, the standing-wave cascade on a 256^3 Yee
grid (field fill timed apart) and past its capacity with thinning per cell, the
rotating-field cascade carried past its capacity by thinning (also with the generator
factor in its random and deterministic forms, the reverse mode and the cap per parent),
the Sec. VII shower and avalanche, 10^4 electrons in a uniform B, Schwinger pairs, the
three emission generators, and the FP64 CPU oracle's rate on a bounded sample of the
rotating-field workload on this host.  Each leg's full record goes to stderr as a
`bench-detail <leg> <json>` line.

HBM traffic of the dominant kernel comes from the rocprofv3 counter summary committed
under profiles/ (FETCH_SIZE and WRITE_SIZE scaled by the same counters' reading for a copy
kernel of known size); it is reported only while the kernel source still has the hash
recorded there, else null.  Next to the published 8 TB/s the roofline also gives the rate
of a plain device copy measured by the calibration program on this GPU (`copy_gbs`) and
the kernel's fraction of it.
"""
import argparse
import ctypes as C
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QED particle-steps/s + HBM roofline %, mixed vs FP64 at fixed spectrum error"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
KERNEL_SRC = os.path.join(ROOT, "paper_1412_6426_amd", "csrc", "qed_step.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "photon_kernel_rotating_cascade_hbm_counters.md")
# algorithmic bytes (per unit of work) of the two persistent kernels
LEPTON_STEP_BYTES = 112   # read x,p (48) id (8) n_events (4); write x,p (48) n_events (4)
PHOTON_STEP_BYTES = 80    # read x,k (48) id (8); write x (24)
DEAD_SLOT_BYTES = 8       # id of a removed photon, read and skipped
EMISSION_BYTES = 84       # photon child written (x,k,w,id,parent,birth = 76) + parent w read (8)


class HipEvents:
    """Raw hipEvent_t handles (timing), for kernels launched inside libqed on our stream."""

    def __init__(self):
        self.lib = C.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.lib.hipEventDestroy.argtypes = [C.c_void_p]
        self.lib.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]

    def create(self, n):
        out = []
        for _ in range(n):
            h = C.c_void_p()
            if self.lib.hipEventCreate(C.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            out.append(h.value)
        return out

    def elapsed_ms(self, a, b):
        f = C.c_float()
        if self.lib.hipEventElapsedTime(C.byref(f), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(f.value)

    def destroy(self, evs):
        for e in evs:
            self.lib.hipEventDestroy(e)


def _stats_records(raw, K):
    from paper_1412_6426_amd import qed as Q
    n = C.sizeof(Q.qed_stats)
    return [Q.qed_stats.from_buffer_copy(raw[i * n:(i + 1) * n]) for i in range(K)]


def make_job(kind, args, precision):
    """The workload, its engine (inputs loaded) and a function that reloads the seeds."""
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd import workloads as W
    if kind == "rotating":
        w = W.rotating_e(n=args.seeds, a0=args.a0, periods=3.0, capacity=args.capacity,
                         precision=precision)
        inits = [W.rotating_e_initial(args.seeds, seed=0)]
        e = R.engine_single(w, inits[0])
    else:
        w = W.batched_rotating(precision=precision)
        inits = W.batched_initial(w)
        e = R.engine_batched(w, inits)

    def reload():
        e.reset_instances()
        for i, init in enumerate(inits):
            for s in range(3):
                e.load(i, s, init[s])
        e.set_step(0)
    return w, e, reload


def sampled_steps(n_steps, k):
    """The steps timed for the headline: the middle step of each of k equal parts of the
    job (all of them when k is None or at least the job's length)."""
    if k is None or k >= n_steps:
        return list(range(n_steps))
    k = max(int(k), 1)
    return sorted({int((i + 0.5) * n_steps / k) for i in range(k)})


def gpu_run(args, precision, kind="rotating", thin=None, fg=None, sample=None, over=None,
            per_parent=None):
    """One job (every step of it) three times from the same seeds: a tuning run that picks
    the launch shape per size class (untimed); the timed run, one captured graph per chosen
    shape replayed step by step, with HIP events around the whole job and around each step
    of `sample` (the steps sampled_steps() picks; None: every step); and an eager run with
    HIP events around the lepton and photon kernels of every step (per-kernel durations for
    the roofline).  The three runs compute the same thing.  thin = (trigger, target):
    qed_thin on the photon store after every step (timed with the step).  fg = (f_photon,
    f_pair): the generator factors of Sec. VI; `over`: other step parameters (the
    deterministic factor, the reverse mode); per_parent: qed_thin_children on the photon
    store after every step with that cap (timed with the step, as thinning)."""
    import numpy as np
    import torch
    from paper_1412_6426_amd import autotune as AT
    from paper_1412_6426_amd import qed as Q
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd import workloads as W

    w, e, reload = make_job(kind, args, precision)
    field = R.field_of(w)
    params = R.params_of(w, freeze_on_drop=1, tile=args.tile, grid_blocks=args.grid_blocks)
    if fg is not None:
        params.f_photon, params.f_pair = fg
    for k, v in (over or {}).items():
        setattr(params, k, v)
    thinning = thin is not None or per_parent is not None
    K = w.n_steps
    timed = sampled_steps(K, sample)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    log = torch.zeros(K * e.stats_buf.numel(), dtype=torch.uint8, device=e.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=e.device)

    def restart():
        torch.cuda.synchronize()
        reload()
        cnt.zero_()
        torch.cuda.synchronize()

    def thin_now():
        if per_parent is not None:
            e.thin_children(Q.QED_PHOTON, per_parent, stream=sp)
        if thin is not None:
            e.thin(Q.QED_PHOTON, thin[0], thin[1], stream=sp)

    # warm-up steps on the same stores, then back to the seed state
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            e.step(field, params, stream=sp)
            thin_now()
    # ---- tuning run: launch shape per size class ----
    if args.no_tune:
        sched = AT.Schedule(steps=[0], shapes=[(args.tile, args.grid_blocks, 0, 0)])
    else:
        restart()
        props = torch.cuda.get_device_properties(0)
        cache = AT.TuneCache(args.tune_cache) if args.tune_cache else None
        key = AT.TuneCache.key(getattr(props, "gcnArchName", "gpu"), precision, w.description)
        with torch.cuda.stream(stream):
            sched = AT.tune_run(e, field, params, K,
                                AT.default_candidates(props.multi_processor_count),
                                after_step=thin_now,
                                known=cache.get(key) if cache else None)
        if cache is not None:
            cache.put(key, sched.choices)
    shape_of = [sched.shape_at(n) for n in range(K)]

    # ---- timed: one captured step (and its stats record) per shape, replayed K times ----
    graphs = {}
    for shape in sched.distinct():
        AT.apply_shape(e, params, shape)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            e.step(field, params, stream=sp)
            thin_now()
            Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), K, cnt.data_ptr(), sp)
        graphs[shape] = g
    plan = [graphs[s] for s in shape_of]
    hip = HipEvents()
    jev = hip.create(2)
    sev = hip.create(2 * len(timed))
    slot_of = {n: i for i, n in enumerate(timed)}
    restart()
    wall0 = time.perf_counter()
    with torch.cuda.stream(stream):  # replay() launches on the current stream
        hip.lib.hipEventRecord(C.c_void_p(jev[0]), C.c_void_p(sp))
        for n, g in enumerate(plan):
            i = slot_of.get(n)
            if i is not None:
                hip.lib.hipEventRecord(C.c_void_p(sev[2 * i]), C.c_void_p(sp))
            g.replay()
            if i is not None:
                hip.lib.hipEventRecord(C.c_void_p(sev[2 * i + 1]), C.c_void_p(sp))
        hip.lib.hipEventRecord(C.c_void_p(jev[1]), C.c_void_p(sp))
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    job_ms = hip.elapsed_ms(jev[0], jev[1])
    step_ms = [hip.elapsed_ms(sev[2 * i], sev[2 * i + 1]) for i in range(len(timed))]
    hip.destroy(jev)
    hip.destroy(sev)
    recs = _stats_records(log.cpu().numpy().tobytes(), K)
    counts = e.counts().tolist()
    hist = None
    if args.spectrum:
        hist = torch.zeros(W.SPECTRUM_BINS, dtype=torch.float64, device=e.device)
        Q.qed_photon_spectrum(e.stores, W.SPECTRUM_LO, W.SPECTRUM_HI, W.SPECTRUM_BINS,
                              hist.data_ptr(), sp)
        torch.cuda.synchronize()
        hist = hist.cpu().numpy()
    del plan, graphs

    # ---- per-kernel durations: the same K steps eagerly, HIP events on our stream ----
    restart()
    evs = hip.create(4 * K)
    tev = hip.create(2 * K) if thinning else []
    with torch.cuda.stream(stream):
        for n in range(K):
            AT.apply_shape(e, params, shape_of[n])
            for j in range(4):
                params.events[j] = evs[4 * n + j]
            e.step(field, params, stream=sp)
            if thinning:
                hip.lib.hipEventRecord(C.c_void_p(tev[2 * n]), C.c_void_p(sp))
                thin_now()
                hip.lib.hipEventRecord(C.c_void_p(tev[2 * n + 1]), C.c_void_p(sp))
            Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), K, cnt.data_ptr(), sp)
    torch.cuda.synchronize()
    for j in range(4):
        params.events[j] = None
    lep_t = [hip.elapsed_ms(evs[4 * n], evs[4 * n + 1]) for n in range(K)]
    pho_t = [hip.elapsed_ms(evs[4 * n + 2], evs[4 * n + 3]) for n in range(K)]
    thin_t = [hip.elapsed_ms(tev[2 * n], tev[2 * n + 1]) for n in range(K)] if thinning else []
    hip.destroy(evs)
    hip.destroy(tev)
    recs2 = _stats_records(log.cpu().numpy().tobytes(), K)
    same = all(a.emitted == b.emitted and a.pairs == b.pairs and
               list(a.advanced) == list(b.advanced) for a, b in zip(recs, recs2))

    step_ps = [int(sum(r.advanced)) for r in recs]
    adv = [sum(r.advanced[s] for r in recs) for s in range(3)]
    dead_slots = sum(r.n_start[2] - r.advanced[2] for r in recs)
    emitted = sum(r.emitted for r in recs)
    pairs = sum(r.pairs for r in recs)
    lep_bytes = LEPTON_STEP_BYTES * (adv[0] + adv[1]) + EMISSION_BYTES * emitted
    pho_bytes = PHOTON_STEP_BYTES * adv[2] + DEAD_SLOT_BYTES * dead_slots
    active = sum(1 for r in recs if sum(r.advanced) > 0)
    first_drop = next((r.step for r in recs if r.dropped > 0), None)
    sampled_ps = sum(step_ps[n] for n in timed)
    out = dict(
        workload=w.description, steps=K, active_steps=active, first_drop_step=first_drop,
        job_ms=job_ms, wall_s=wall, particle_steps=int(sum(adv)),
        value_job=sum(adv) / (job_ms / 1e3) if job_ms > 0 else 0.0,
        timed_steps=timed, timed_ms=sum(step_ms), timed_particle_steps=int(sampled_ps),
        value=sampled_ps / (sum(step_ms) / 1e3) if sum(step_ms) > 0 else 0.0,
        advanced=[int(a) for a in adv], emitted=int(emitted),
        pairs=int(pairs), lep_ms=sum(lep_t), pho_ms=sum(pho_t), thin_ms=sum(thin_t),
        launches=K, lep_bytes=lep_bytes,
        pho_bytes=pho_bytes, final_counts=[int(sum(c[s] for c in counts)) for s in range(3)],
        eager_matches_graph=bool(same),
        schedule=[dict(from_step=k, tile=t, grid_blocks=g, arena_div=a, refill_min=r)
                  for k, (t, g, a, r) in zip(sched.steps, sched.shapes)],
        substeps=int(sum(r.substeps for r in recs)),
        nsub_refined=int(sum(r.nsub_refined for r in recs)),
        low_occupancy_iters=int(sum(r.low_occupancy_iters for r in recs)),
        wave_iters=int(sum(r.wave_iters for r in recs)),
        near_threshold=int(sum(r.near_threshold for r in recs)),
        saturated=int(sum(r.saturated for r in recs)),
        max_p_emit=float(max((r.max_p_emit for r in recs), default=0.0)),
        max_p_pair=float(max((r.max_p_pair for r in recs), default=0.0)),
        early_out=int(sum(r.early_out for r in recs)),
        dropped=int(sum(r.dropped for r in recs)),
        # per step, for the precision comparison
        step_pairs=[int(r.pairs) for r in recs], step_emitted=[int(r.emitted) for r in recs],
        step_hist=np.array([list(r.photon_hist) for r in recs], dtype=np.float64),
        step_dropped=[int(r.dropped) for r in recs], spectrum=hist,
    )
    del e
    torch.cuda.empty_cache()
    return out


def _rounded(v, digits=6):
    """Floats to `digits` significant digits (the leg summaries of the one-line record; the
    full values are in the bench-detail lines)."""
    if isinstance(v, float):
        return float(f"{v:.{digits}g}")
    if isinstance(v, dict):
        return {k: _rounded(x, digits) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_rounded(x, digits) for x in v]
    return v


def thin_cells_arg(args):
    frac, cap = args.thin_cells.split(":")
    return float(frac), int(cap)


def gpu_run_yee(args, precision, sort_every=None, sort_species=None, thin=None):
    """Standing-wave cascade on a 256^3 Yee grid (two counter-propagating CP waves, a0 =
    2000 each, cells of lambda/32, 10^6 seeds Gaussian sigma = 0.1 lambda about the node,
    dt = T/100, 2*10^8 photon slots).  The grid is refilled with the analytic wave before
    every step (a stand-in for the field solver, timed separately); steps run eagerly with
    HIP events around the fill, the whole step, and the lepton and photon kernels.  Every
    `sort_every` steps (0: never) the stores `sort_species` are sorted by cell
    (qed_sort_cells) before the step; that time counts as part of the step and is also
    reported apart.  thin = (fraction, cap): after each step, every store holding more slots
    than that fraction of its capacity is thinned per cell block to at most `cap` particles
    (qed_thin_cells; the counts are read on the host each step), so the job runs all its
    steps without dropping children; the thinning is timed and counts in `value`."""
    import torch
    from paper_1412_6426_amd import qed as Q
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd import workloads as W

    w = W.standing_wave_grid(precision=precision)
    init = W.standing_wave_initial(w.n_seed, seed=0)
    e = R.engine_single(w, init)
    grid = R.YeeGrid(w)
    field = R.field_of(w, grid=grid.g)
    params = R.params_of(w, freeze_on_drop=0 if thin else 1, tile=args.tile,
                         grid_blocks=args.grid_blocks)
    K = w.n_steps
    S = args.sort_every if sort_every is None else sort_every
    if sort_species is None:
        sort_species = [int(v) for v in args.sort_species.split(",") if v.strip()]
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    log = torch.zeros(K * e.stats_buf.numel(), dtype=torch.uint8, device=e.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=e.device)
    hip = HipEvents()
    evs = hip.create(8 * K)
    tev = hip.create(2 * K) if thin else []
    thin_calls = 0
    if S:
        e.sort_cells(0, field, stream=sp)  # allocates the sort workspace outside the timing
    if thin:
        for s_ in range(3):  # the thinning workspace and records, outside the timing
            e.thin_cells(s_, field, 1 << 62, stream=sp)
    torch.cuda.synchronize()
    e.set_step(0)
    with torch.cuda.stream(stream):
        for n in range(K):
            ev = evs[8 * n:8 * n + 8]
            hip.lib.hipEventRecord(C.c_void_p(ev[0]), C.c_void_p(sp))
            grid.fill(w.t0 + n * w.dt, sp)
            hip.lib.hipEventRecord(C.c_void_p(ev[1]), C.c_void_p(sp))
            if S and n % S == 0:
                for s_ in sort_species:
                    e.sort_cells(s_, field, stream=sp)
            hip.lib.hipEventRecord(C.c_void_p(ev[7]), C.c_void_p(sp))
            for j in range(4):
                params.events[j] = ev[2 + j]
            e.step(field, params, stream=sp)
            hip.lib.hipEventRecord(C.c_void_p(ev[6]), C.c_void_p(sp))
            Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), K, cnt.data_ptr(), sp)
            if thin:
                hip.lib.hipEventRecord(C.c_void_p(tev[2 * n]), C.c_void_p(sp))
                stream.synchronize()
                counts = e.counts()[0]
                for s_ in range(3):
                    if counts[s_] > thin[0] * w.capacity[s_]:
                        e.thin_cells(s_, field, thin[1], stream=sp)
                        thin_calls += 1
                hip.lib.hipEventRecord(C.c_void_p(tev[2 * n + 1]), C.c_void_p(sp))
    torch.cuda.synchronize()
    for j in range(4):
        params.events[j] = None
    thin_ms = sum(hip.elapsed_ms(tev[2 * n], tev[2 * n + 1]) for n in range(K)) if thin else 0.0
    hip.destroy(tev)
    fill_ms = sum(hip.elapsed_ms(evs[8 * n], evs[8 * n + 1]) for n in range(K))
    step_ms = sum(hip.elapsed_ms(evs[8 * n + 1], evs[8 * n + 6]) for n in range(K))
    sort_ms = sum(hip.elapsed_ms(evs[8 * n + 1], evs[8 * n + 7]) for n in range(K))
    lep_ms = sum(hip.elapsed_ms(evs[8 * n + 2], evs[8 * n + 3]) for n in range(K))
    pho_ms = sum(hip.elapsed_ms(evs[8 * n + 4], evs[8 * n + 5]) for n in range(K))
    hip.destroy(evs)
    recs = _stats_records(log.cpu().numpy().tobytes(), K)
    adv = [sum(r.advanced[s] for r in recs) for s in range(3)]
    emitted = sum(r.emitted for r in recs)
    dead_slots = sum(r.n_start[2] - r.advanced[2] for r in recs)
    out = dict(
        workload=w.description, precision=precision, steps=K,
        first_drop_step=next((r.step for r in recs if r.dropped > 0), None),
        particle_steps=int(sum(adv)), advanced=[int(a) for a in adv], emitted=int(emitted),
        pairs=int(sum(r.pairs for r in recs)), step_ms=step_ms, fill_ms=fill_ms,
        sort_every=S, sort_species=list(sort_species) if S else [], sort_ms=sort_ms, lep_ms=lep_ms, pho_ms=pho_ms,
        value=sum(adv) / ((step_ms + thin_ms) / 1e3),
        thin=list(thin) if thin else None, thin_ms=thin_ms, thin_calls=thin_calls,
        dropped=int(sum(r.dropped for r in recs)), final_counts=e.counts()[0].tolist(),
        substeps=int(sum(r.substeps for r in recs)),
        nsub_max=max((k for r in recs for k in range(len(r.nsub_hist)) if r.nsub_hist[k]),
                     default=0),
        saturated=int(sum(r.saturated for r in recs)),
        near_threshold=int(sum(r.near_threshold for r in recs)),
        lepton_roofline_gbs=(LEPTON_STEP_BYTES * (adv[0] + adv[1]) + EMISSION_BYTES * emitted)
        / (lep_ms / 1e3) / 1e9 if lep_ms > 0 else 0.0,
        photon_roofline_gbs=(PHOTON_STEP_BYTES * adv[2] + DEAD_SLOT_BYTES * dead_slots)
        / (pho_ms / 1e3) / 1e9 if pho_ms > 0 else 0.0,
    )
    del e, grid
    torch.cuda.empty_cache()
    return out


def gpu_uniform_b(args):
    """The uniform-B workload: 10^4 electrons at gamma = 1000 across a uniform B with
    chi = 1, eight sub-steps each (dt = T_gyro/100), 100 steps, emission only, photons
    recorded and not pushed.  Steps run eagerly on one stream with HIP events around each step and around its
    lepton kernel, then again from the seeds as one captured step replayed 100 times.  10^4
    electrons fill 157 wavefronts: these runs show the step's fixed cost per launch, not a
    bandwidth."""
    import torch
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd import workloads as W

    w = W.uniform_b()
    init = W.uniform_b_initial(w)
    e = R.engine_single(w, init)
    field = R.field_of(w)
    params = R.params_of(w)
    K = w.n_steps
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    hip = HipEvents()
    evs = hip.create(4 * K)
    torch.cuda.synchronize()
    e.set_step(0)
    with torch.cuda.stream(stream):
        for n in range(K):
            ev = evs[4 * n:4 * n + 4]
            hip.lib.hipEventRecord(C.c_void_p(ev[0]), C.c_void_p(sp))
            params.events[0] = ev[1]
            params.events[1] = ev[2]
            e.step(field, params, stream=sp)
            hip.lib.hipEventRecord(C.c_void_p(ev[3]), C.c_void_p(sp))
    torch.cuda.synchronize()
    step_ms = sum(hip.elapsed_ms(evs[4 * n], evs[4 * n + 3]) for n in range(K))
    lep_ms = sum(hip.elapsed_ms(evs[4 * n + 1], evs[4 * n + 2]) for n in range(K))
    hip.destroy(evs)
    photons = int(e.counts()[0, 2])
    # The same K steps again from the seeds, as one captured step replayed K times (the
    # step index lives on the device, so each replay is the next step): the launch
    # overheads of the eight kernels no longer add up step by step.
    params.events[0] = params.events[1] = None
    e.reset_instances()
    for s in range(3):
        e.load(0, s, init[s])
    e.set_step(0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        e.step(field, params, stream=sp)
    e.reset_instances()
    for s in range(3):
        e.load(0, s, init[s])
    e.set_step(0)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0.record(stream)
        for _ in range(K):
            g.replay()
        t1.record(stream)
    torch.cuda.synchronize()
    graph_ms = t0.elapsed_time(t1)
    photons_graph = int(e.counts()[0, 2])
    del g
    lepton_steps = w.n_seed * K
    del e
    torch.cuda.empty_cache()
    return dict(workload=w.description, steps=K, lepton_steps=lepton_steps,
                substeps=8 * lepton_steps, photons_emitted=photons,
                photons_emitted_graph=photons_graph,
                us_per_step=1e3 * step_ms / K, lepton_kernel_us_per_step=1e3 * lep_ms / K,
                us_per_step_graph=1e3 * graph_ms / K,
                lepton_steps_per_s_graph=lepton_steps / (graph_ms / 1e3),
                lepton_steps_per_s=lepton_steps / (step_ms / 1e3),
                lepton_kernel_gbs=(LEPTON_STEP_BYTES * lepton_steps + EMISSION_BYTES * photons)
                / (lep_ms / 1e3) / 1e9)


def gpu_schwinger_grid(args):
    """Schwinger pairs (Sec. V.B) on the 256^3 Yee grid of the standing-wave workload (cells of
    lambda/32, lambda = 0.8 um, dt = T/100), the wave's amplitude raised so that its antinodes
    reach 0.075 E_S, where vacuum pairs set in for cells this size: qed_schwinger over 20
    steps (the grid refilled with the wave at every t_n, untimed), each launch timed with HIP
    events on its stream.
    Algorithmic bytes: the three FP32 E components of each cell, 12 B."""
    import torch
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd import workloads as W
    from paper_1412_6426_amd.engine import Engine

    e_max = 0.075
    w = W.standing_wave_grid(n=1)
    a_wave = e_max / (2.0 * w.eps_r)  # |E| = 2 a |cos kx| for the CP standing wave
    w.field.grid_wave_amp = a_wave
    grid = R.YeeGrid(w)
    field = R.field_of(w, grid=grid.g)
    e = Engine([(1_000_000, 1_000_000, 16)], seeds=[0])
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    hip = HipEvents()
    K = 20
    evs = hip.create(2 * K)
    pairs = expected = 0.0
    cells = 0
    torch.cuda.synchronize()
    # Everything is queued on one stream without host waits, so the host runs ahead and each
    # launch starts as soon as the grid refill before it ends; each step's record is copied
    # aside on the stream.
    rec = e.schwinger_record_buffer()
    recs = torch.empty((K, rec.numel()), dtype=torch.uint8, device=rec.device)
    with torch.cuda.stream(stream):
        for n in range(K):
            e.set_step(n)
            grid.fill(w.t0 + n * w.dt, sp)
            hip.lib.hipEventRecord(C.c_void_p(evs[2 * n]), C.c_void_p(sp))
            e.schwinger(field, w.dt, w.eps_r, 1.0, stream=sp)
            hip.lib.hipEventRecord(C.c_void_p(evs[2 * n + 1]), C.c_void_p(sp))
            recs[n].copy_(rec)
    torch.cuda.synchronize()
    for raw in recs.cpu().numpy():
        r = Engine.decode_schwinger_record(raw.tobytes())
        pairs += r["pairs"]
        expected += r["expected"]
        cells += r["cells"]
    ms = [hip.elapsed_ms(evs[2 * n], evs[2 * n + 1]) for n in range(K)]
    hip.destroy(evs)
    tot_ms = sum(ms)
    achieved = 12.0 * cells / (tot_ms / 1e3) / 1e9
    out = dict(
        workload=f"256^3 Yee grid, CP standing wave with |E| up to {e_max} E_S "
                 f"(a = {a_wave:.4g}), lambda = 0.8 um, cells of lambda/32, dt = T/100, "
                 f"{K} steps",
        cells_per_s=cells / (tot_ms / 1e3), avg_launch_us=1e3 * tot_ms / K,
        pairs=int(pairs), expected_pairs=expected, counts=e.counts().tolist()[0][:2],
        roofline={"bound": "hbm", "kernel": "schwinger_kernel", "achieved": achieved,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                  "algorithmic_bytes_per_cell": 12})
    del e, grid
    torch.cuda.empty_cache()
    return out


def gpu_generator_comparison(args):
    """The three emission generators of Sec. IV.G as independent trials in the setting of
    the paper's comparison of their spectra: gamma = 100, chi = 1, 10^7 trials per
    generator, an interval with dtfac = 31.25 (the modified generator's P_m stays below
    about 0.5) and the standard generator's cutoff delta_min = 10^-3.  Each generator's
    launch (for the standard one: its W table and the trials) is timed with HIP events over
    5 repetitions; the emitted deltas are then counted per decade (untimed)."""
    import torch
    from paper_1412_6426_amd import qed as Q

    gamma, chi, dtfac, dmin, n, reps = 100.0, 1.0, 0.5 * 100.0 / 1.6, 1e-3, 10_000_000, 5
    tab = torch.zeros(Q.qed_table_bytes() + 256, dtype=torch.uint8, device="cuda")
    tp = tab.data_ptr() + ((-tab.data_ptr()) % 256)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    Q.qed_build_tables(tp, Q.qed_table_bytes(), sp)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    hip = HipEvents()
    res = {}
    edges = [10.0 ** k for k in range(-9, 1)]  # decades 1e-9 .. 1
    for name, gen in (("modified", Q.QED_GEN_MODIFIED), ("alternative", Q.QED_GEN_ALTERNATIVE),
                      ("standard", Q.QED_GEN_STANDARD)):
        wb = Q.qed_generator_work_bytes(gen, chi, dmin)
        work = torch.empty(wb + 256, dtype=torch.uint8, device="cuda") if wb else None
        wp = work.data_ptr() + ((-work.data_ptr()) % 256) if wb else None
        evs = hip.create(2 * reps)
        torch.cuda.synchronize()
        Q.qed_generator_trials(tp, gen, chi, gamma, dtfac, dmin, 0xE4, 0, n, out.data_ptr(),
                               wp, wb, sp)  # warm-up
        for r in range(reps):
            hip.lib.hipEventRecord(C.c_void_p(evs[2 * r]), C.c_void_p(sp))
            Q.qed_generator_trials(tp, gen, chi, gamma, dtfac, dmin, 0xE4, 0, n,
                                   out.data_ptr(), wp, wb, sp)
            hip.lib.hipEventRecord(C.c_void_p(evs[2 * r + 1]), C.c_void_p(sp))
        torch.cuda.synchronize()
        ms = sum(hip.elapsed_ms(evs[2 * r], evs[2 * r + 1]) for r in range(reps)) / reps
        hip.destroy(evs)
        d = out[out > 0]
        counts = torch.histc(torch.log10(d), bins=9, min=-9.0, max=0.0).long().tolist()
        res[name] = dict(ms_per_launch=ms, trials_per_s=n / (ms / 1e3),
                         emitted=int(d.numel()), emitted_per_decade=dict(
                             zip([f"{edges[k]:.0e}-{edges[k + 1]:.0e}" for k in range(9)],
                                 counts)))
        del work
    del out, tab
    torch.cuda.empty_cache()
    return dict(workload=f"gamma = {gamma:g}, chi = {chi:g}, dtfac = {dtfac:g}, "
                         f"delta_min = {dmin:g} (standard), {n} trials per generator",
                generators=res)


def roofline_of(r):
    dom = "photon" if r["pho_ms"] >= r["lep_ms"] else "lepton"
    kbytes = r["pho_bytes"] if dom == "photon" else r["lep_bytes"]
    kms = r["pho_ms"] if dom == "photon" else r["lep_ms"]
    achieved = kbytes / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    return dom, kbytes, kms, achieved


def precision_compare(r64, rmx):
    """Mixed vs FP64 over the steps before either run first drops a child: L1 distance of
    the emitted-photon spectra (130 log bins of eps in [1e-8, 1e5]) and the pair yield."""
    import numpy as np
    K = len(r64["step_pairs"])
    d = [k for k in range(K) if r64["step_dropped"][k] or rmx["step_dropped"][k]]
    upto = d[0] if d else K
    h64 = r64["step_hist"][:upto].sum(axis=0)
    hmx = rmx["step_hist"][:upto].sum(axis=0)
    p64 = sum(r64["step_pairs"][:upto])
    pmx = sum(rmx["step_pairs"][:upto])
    return {
        "steps_compared": upto,
        "spectrum_l1_vs_f64": float(np.abs(hmx - h64).sum() / max(h64.sum(), 1.0)),
        "photons_f64": int(h64.sum()), "photons_mixed": int(hmx.sum()),
        "pairs_f64": int(p64), "pairs_mixed": int(pmx),
        "pair_yield_rel_diff": (pmx - p64) / max(p64, 1),
    }


def traffic_summary_path(dom):
    """The counter summary of the dominant kernel on the rotating-field cascade."""
    return os.path.join(ROOT, "profiles", f"{dom}_kernel_rotating_cascade_hbm_counters.md")


def copy_peak_gbs():
    """The HBM rate a plain device copy reaches on this GPU (the best of the five launches of
    the calibration program lib/hbm_copy, 800 MB each way, run as a child process), the
    practical ceiling next to the published 8 TB/s; None if it cannot run."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1412_6426_amd", "lib", "hbm_copy")
    if not os.path.exists(exe):
        return None
    try:
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    rates = [float(w.split("=")[1]) for w in out.split() if w.startswith("GB/s=")]
    return max(rates) if rates else None


def measured_traffic(dom, kernel):
    """HBM bytes per launch of `kernel` (its full template name) from the committed counter
    summary, if the kernel source is unchanged since the counters were taken."""
    try:
        text = open(traffic_summary_path(dom)).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    from paper_1412_6426_amd.calib.profile_summary import source_digest
    if vals.get("kernel") != kernel or vals.get("kernel_source_sha256") != source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_name(dom, precision):
    """Full template name of the rotating-field step kernel, as the profiler prints it."""
    mixed = "true" if precision == "mixed" else "false"
    return f"photon_kernel<{mixed}, 1>" if dom == "photon" else f"lepton_kernel<{mixed}, 1, false>"


def detail(name, record):
    """A leg's full record, on stderr (the JSON line on stdout keeps a summary)."""
    def conv(v):
        if hasattr(v, "tolist"):
            return v.tolist()
        return v
    rec = {k: conv(v) for k, v in record.items()} if isinstance(record, dict) else record
    print(f"bench-detail {name} " + json.dumps(rec, default=conv), file=sys.stderr, flush=True)


def cpu_baseline(args):
    """The FP64 oracle on a bounded sample of the same workload: the rotating-field
    cascade from `cpu_seeds` seeds, stepped until ~cpu_seconds of CPU time has passed."""
    from oracle import oracle as orc
    from paper_1412_6426_amd import workloads as W
    from tests.parity_util import oracle_field, oracle_params, oracle_stores

    # same per-seed capacity as the GPU run (10^8 slots per store for 10^5 seeds)
    cap = max(1000, args.capacity * args.cpu_seeds // args.seeds)
    w = W.rotating_e(n=args.cpu_seeds, a0=args.a0, periods=3.0, capacity=cap,
                     lepton_capacity=cap)
    init = W.rotating_e_initial(args.cpu_seeds, seed=0)
    st = oracle_stores(orc, init, w.capacity)
    fld, par = oracle_field(orc, w), oracle_params(orc, w)
    orc.tables()
    done, steps = 0, 0
    t0 = time.perf_counter()
    for n in range(w.n_steps):
        alive = st[0].count + st[1].count + int((st[2].id[:st[2].count] != orc.ID_DEAD).sum())
        par.step = n
        s = orc.step(st, fld, par)
        done += alive
        steps += 1
        if s["dropped"] or time.perf_counter() - t0 > args.cpu_seconds:
            break
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=done / dt, unit="particle-steps/s", cores=threads, kind="oracle",
                sample=f"rotating-E cascade a0={args.a0:g} from {args.cpu_seeds} seeds, "
                       f"first {steps} of {w.n_steps} steps ({done} particle-steps, "
                       f"{dt:.1f} s), FP64 C oracle, OpenMP over particles")


def _time_step_runs(runs_spec, n_inst, samples, count, label):
    """Run each (name, workload, generations, steps_per_sample, arena_records) of runs_spec
    on n_inst instances (instance i seeded with i, the same initial particles) for
    `samples` intervals, timing the steps of each interval with HIP events on the engine's
    stream.  count(engine) gives per-instance quantities [n_inst, q] after each interval.
    The first run is the reference: the others get z-scores of their interval means over
    the instances against it."""
    import numpy as np
    import torch
    from paper_1412_6426_amd import qed as Q
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd.engine import Engine

    runs = {}
    for name, w, init, G, sps, arena in runs_spec:
        print(f"bench: {label}, {name}", file=sys.stderr, flush=True)
        caps = tuple(w.capacity)
        e = Engine([caps] * n_inst, seeds=list(range(n_inst)), same_step=G > 0,
                   arena_records=arena)
        e.build_tables()
        for i in range(n_inst):
            for s in range(3):
                e.load(i, s, init[s])
        field = R.field_of(w)
        params = R.params_of(w, same_step_generations=G)
        K = sps * samples
        log = torch.zeros(K * e.stats_buf.numel(), dtype=torch.uint8, device=e.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=e.device)
        stream = torch.cuda.Stream()
        sp = stream.cuda_stream
        hip = HipEvents()
        evs = hip.create(2 * samples)
        counts = []
        e.set_step(0)
        torch.cuda.synchronize()
        for m in range(samples):
            with torch.cuda.stream(stream):
                hip.lib.hipEventRecord(C.c_void_p(evs[2 * m]), C.c_void_p(sp))
                for _ in range(sps):
                    e.step(field, params, stream=sp)
                    Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), K, cnt.data_ptr(),
                                       sp)
                hip.lib.hipEventRecord(C.c_void_p(evs[2 * m + 1]), C.c_void_p(sp))
            torch.cuda.synchronize()
            counts.append(count(e))
        step_ms = sum(hip.elapsed_ms(evs[2 * m], evs[2 * m + 1]) for m in range(samples))
        hip.destroy(evs)
        recs = _stats_records(log.cpu().numpy().tobytes(), K)
        runs[name] = dict(
            dt=w.dt, kappa=w.kappa, generations=G, steps=K, step_ms=step_ms,
            substeps=int(sum(r.substeps for r in recs)),
            particle_steps=int(sum(sum(r.advanced) for r in recs)),
            children_advanced=int(sum(r.children_advanced for r in recs)),
            deferred=int(sum(r.deferred for r in recs)),
            dropped=int(sum(r.dropped for r in recs)),
            saturated=int(sum(r.saturated for r in recs)),
            final_counts=[int(x) for x in e.counts().sum(0)],
            counts=np.array(counts))  # [sample, instance, quantity]
        del e, log
        torch.cuda.empty_cache()
    names = list(runs)
    ref = runs[names[0]]["counts"]
    out = {}
    for name in names:
        r = runs[name]
        c = r.pop("counts")
        r["mean_counts"] = c.mean(1).round(2).tolist()  # [sample][quantity], per instance
        if name != names[0]:
            se = np.sqrt(c.var(1, ddof=1) / n_inst + ref.var(1, ddof=1) / n_inst)
            z = (c.mean(1) - ref.mean(1)) / np.where(se > 0, se, np.inf)
            r["z_vs_" + names[0]] = z.round(2).tolist()
            r["max_abs_z"] = float(np.abs(z).max())
            r["ratio_vs_" + names[0]] = (c.mean(1) / np.where(ref.mean(1) > 0, ref.mean(1),
                                                               np.nan)).round(3).tolist()
            r["speedup_vs_" + names[0]] = runs[names[0]]["step_ms"] / r["step_ms"]
        out[name] = r
    return out


def gpu_shower(args):
    """Sec. VII cascade development (the shower) at the paper's scale: 10^3 runs, as 8
    instances of 125 seed electrons (gamma_0 = 2e5 across B = 0.2 E_S), counted every 25000
    hbar / m c^2 up to `shower_samples` times that (1.39 t_rad for 5): the particles of each
    species above 1e-3 gamma_0 m c^2, weighted, per instance.  Runs:
      small_dt            dt = 62.5, one sub-step per particle (the reference);
      large_dt_same_step  dt = 25000, about 400 lepton sub-steps a step at kappa = 0.25,
                          children advanced in their birth step (16 generations);
      ..._kappa_0.1       the same with sub-steps 2.5 times shorter;
      large_dt_next_step  the same large step with children left for the next step."""
    import numpy as np
    from paper_1412_6426_amd import qed as Q
    from paper_1412_6426_amd import workloads as W

    n_inst = 8
    per = max(args.shower_seeds // n_inst, 1)
    interval = 25_000.0
    thr = 1e-3 * W.SHOWER_GAMMA0
    caps = (args.shower_lepton_cap // n_inst, args.shower_lepton_cap // n_inst,
            args.shower_photon_cap // n_inst)
    dead = -1  # the removed-photon id 2^64 - 1, as the int64 the id column holds

    def count(e):
        live = e.counts()
        out = np.zeros((n_inst, 3))
        for i in range(n_inst):
            for s in range(3):
                b, n = int(e.base[i, s]), int(live[i, s])
                if n == 0:
                    continue
                col = e.cols[s]
                p2 = (col["px"][b:b + n] ** 2 + col["py"][b:b + n] ** 2 +
                      col["pz"][b:b + n] ** 2)
                if s == Q.QED_PHOTON:
                    above = (p2 > thr * thr) & (col["id"][b:b + n] != dead)
                else:
                    above = (1.0 + p2) > thr * thr
                out[i, s] = float((col["w"][b:b + n] * above).sum().item())
        return out

    spec = []
    for name, dt, kappa, G in (("small_dt", 62.5, 1.0, 0),
                               ("large_dt_same_step", interval, 0.25, 16),
                               ("large_dt_same_step_kappa_0.1", interval, 0.1, 16),
                               ("large_dt_next_step", interval, 0.25, 0)):
        sps = int(round(interval / dt))
        w = W.shower(n=per, dt=dt, steps=sps * args.shower_samples, kappa=kappa, capacity=caps)
        # a large step's children (all generations) pass through the arenas: size them
        # for the step's photons
        arena = min(args.shower_photon_cap // 2, 1 << 27) if G > 0 else None
        spec.append((name, w, W.shower_initial(w), G, sps, arena))
    out = dict(workload=f"{n_inst} x {per} e-, gamma0 = {W.SHOWER_GAMMA0:g} across "
                        f"B = {W.SHOWER_B} E_S; counts (e-, e+, photons) above {thr:g} m c^2 "
                        f"every {interval:g} hbar/mc^2 (t_rad = {W.shower_t_rad():.4g})",
               t=[interval * (m + 1) for m in range(args.shower_samples)])
    out.update(_time_step_runs(spec, n_inst, args.shower_samples, count, "shower"))
    return out


def gpu_avalanche(args):
    """Sec. VII avalanche-type cascade: electrons at x = lambda/8 with p_y = 1000 m c in the
    plane standing wave E_y(0) = 1e-2 E_S sin(kx), lambda = 1 um, as 8 instances of
    `avalanche_seeds` / 8 independent runs; the pairs created so far (positrons, weighted)
    and the photons, per instance, every two large steps (about T / 4) for
    `avalanche_samples` intervals.  Runs:
      small_dt            dt = 173/1018 t_rad (about 0.17 t_rad: no sub-division);
      large_dt_same_step  dt = 173 t_rad (about T / 8; the field is sampled 8 times a
                          period), kappa = 0.25, children in their birth step;
      large_dt_next_step  the same large step with children left for the next step."""
    import numpy as np
    from paper_1412_6426_amd import workloads as W

    n_inst = 8
    per = max(args.avalanche_seeds // n_inst, 1)
    periods = args.avalanche_samples * 2 * 173.0 * W.avalanche_t_rad() / (2 * np.pi)
    caps = (args.avalanche_lepton_cap // n_inst, args.avalanche_lepton_cap // n_inst,
            args.avalanche_photon_cap // n_inst)

    def count(e):
        live = e.counts()
        out = np.zeros((n_inst, 2))
        for i in range(n_inst):
            b, n = int(e.base[i, 1]), int(live[i, 1])
            if n:
                out[i, 0] = float(e.cols[1]["w"][b:b + n].sum().item())
            out[i, 1] = float(live[i, 2])
        return out

    spec = []
    for name, ratio, kappa, G, sps in (("small_dt", 173.0 / 1018.0, 1.0, 0, 2 * 1018),
                                       ("large_dt_same_step", 173.0, 0.25, 16, 2),
                                       ("large_dt_next_step", 173.0, 0.25, 0, 2)):
        w = W.avalanche(n=per, dt_over_t_rad=ratio, periods=periods, kappa=kappa,
                        capacity=caps)
        arena = min(args.avalanche_photon_cap // 2, 1 << 27) if G > 0 else None
        spec.append((name, w, W.avalanche_initial(w), G, sps, arena))
    T_large = 173.0 * W.avalanche_t_rad()
    out = dict(workload=f"{n_inst} x {per} e- at lambda/8, p_y = {W.AVALANCHE_P0:g} m c, "
                        f"standing wave E_y(0) = {W.AVALANCHE_E0:g} E_S sin(kx), lambda = 1 um; "
                        "per instance: pairs created, photon slots",
               t_over_period=[round((m + 1) * 2 * T_large / (2 * np.pi), 4)
                              for m in range(args.avalanche_samples)])
    out.update(_time_step_runs(spec, n_inst, args.avalanche_samples, count, "avalanche"))
    # growth of the pair count (e-folds per period) over the second half of the interval
    t = out["t_over_period"]
    k = len(t) // 2
    for name, _, _, _, _, _ in spec:
        c = [row[0] for row in out[name]["mean_counts"]]
        if c[k] > 0 and c[-1] > 0 and t[-1] > t[k]:
            out[name]["pair_growth_per_period"] = round(np.log(c[-1] / c[k]) / (t[-1] - t[k]), 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="steps of the 600-step job timed for the headline, spread evenly "
                         "over it (default: every step)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=("f64", "mixed"), default="f64")
    ap.add_argument("--seeds", type=int, default=100_000)
    ap.add_argument("--a0", type=float, default=1000.0)
    ap.add_argument("--capacity", type=int, default=100_000_000)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--cpu-seeds", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run and its accuracy comparison")
    ap.add_argument("--spectrum", action="store_true",
                    help="also histogram the final photon stores")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-ensemble runs (64 cascades, mixed and FP64)")
    ap.add_argument("--no-thin", action="store_true",
                    help="skip the cascade run past the capacity with thinning")
    ap.add_argument("--no-yee", action="store_true",
                    help="skip the standing-wave cascade on the 256^3 Yee grid")
    ap.add_argument("--no-shower", action="store_true",
                    help="skip the Sec. VII shower at small and large time steps")
    ap.add_argument("--shower-only", action="store_true",
                    help="run only the shower comparison and print its record (profiling)")
    ap.add_argument("--shower-seeds", type=int, default=1000)
    ap.add_argument("--shower-samples", type=int, default=5)
    ap.add_argument("--shower-photon-cap", type=int, default=300_000_000)
    ap.add_argument("--shower-lepton-cap", type=int, default=20_000_000)
    ap.add_argument("--no-avalanche", action="store_true",
                    help="skip the Sec. VII avalanche at small and large time steps")
    ap.add_argument("--avalanche-only", action="store_true",
                    help="run only the avalanche comparison and print its record (profiling)")
    ap.add_argument("--avalanche-seeds", type=int, default=200)
    ap.add_argument("--avalanche-samples", type=int, default=6)
    ap.add_argument("--avalanche-photon-cap", type=int, default=200_000_000)
    ap.add_argument("--avalanche-lepton-cap", type=int, default=40_000_000)
    ap.add_argument("--no-schwinger", action="store_true",
                    help="skip Schwinger pair production on the 256^3 grid")
    ap.add_argument("--schwinger-only", action="store_true",
                    help="run only the Schwinger leg and print its record (profiling)")
    ap.add_argument("--no-uniform-b", action="store_true",
                    help="skip the 10^4 electrons in a uniform B")
    ap.add_argument("--thin-cells", default="0.5:1024",
                    help="grid cascade past its capacity: FRACTION:CAP, thin a store per cell "
                         "block to CAP particles once it holds FRACTION of its slots")
    ap.add_argument("--only", choices=("uniform-b", "yee", "yee-thinned", "batched"),
                    default=None,
                    help="run only this leg and print its record (profiling)")
    ap.add_argument("--no-generators", action="store_true",
                    help="skip the comparison of the three emission generators")
    ap.add_argument("--generators-only", action="store_true",
                    help="run only the generator comparison and print its record (profiling)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned shapes per (arch, precision, workload): read "
                         "before tuning (known size classes are not tried again), written after")
    ap.add_argument("--sort-every", type=int, default=3,
                    help="grid cascade: sort stores by cell every this many steps (0: never)")
    ap.add_argument("--sort-species", default="0,1",
                    help="grid cascade: the stores --sort-every sorts (0 e-, 1 e+, 2 photons; "
                         "photons are born in their parents' order)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use --tile / --grid-blocks for every step instead of tuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.shower_only:
        print(json.dumps({"shower_time_step_invariance": gpu_shower(args)}), flush=True)
        return
    if args.avalanche_only:
        print(json.dumps({"avalanche_time_step_invariance": gpu_avalanche(args)}), flush=True)
        return
    if args.schwinger_only:
        print(json.dumps({"schwinger_grid": gpu_schwinger_grid(args)}), flush=True)
        return
    if args.only == "uniform-b":
        print(json.dumps({"uniform_b": gpu_uniform_b(args)}), flush=True)
        return
    if args.only == "yee":
        print(json.dumps({"standing_wave_grid": gpu_run_yee(args, args.precision)}), flush=True)
        return
    if args.only == "yee-thinned":
        print(json.dumps({"standing_wave_grid_thinned": gpu_run_yee(
            args, args.precision, thin=thin_cells_arg(args))}), flush=True)
        return
    if args.only == "batched":
        out = {}
        for prec in ("mixed", "f64"):
            rb = gpu_run(args, prec, kind="batched")
            out[prec] = dict(value=rb["value_job"], ms=rb["job_ms"],
                             lep_ms=rb["lep_ms"], pho_ms=rb["pho_ms"])
        print(json.dumps({"batched": out}), flush=True)
        return
    if args.generators_only:
        print(json.dumps({"generator_comparison": gpu_generator_comparison(args)}), flush=True)
        return
    print(f"bench: rotating-E cascade, {args.seeds} seeds, precision {args.precision}",
          file=sys.stderr, flush=True)
    r = gpu_run(args, args.precision, sample=args.steps)
    nt = len(r["timed_steps"])
    print(f"bench: {r['timed_particle_steps']} particle-steps in {r['timed_ms']:.1f} ms over "
          f"{nt} timed steps; whole job {r['particle_steps']} in {r['job_ms']:.1f} ms",
          file=sys.stderr, flush=True)
    dom, kbytes, kms, achieved = roofline_of(r)
    launches = r["launches"]
    traffic = measured_traffic(dom, kernel_name(dom, args.precision))
    copy_gbs = copy_peak_gbs()
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": nt,
        "warmup": args.warmup,
        "ms_per_step": r["timed_ms"] / nt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f64+f32",
        "data": "synthetic (seeded)",
        "config": {
            "workload": "rotating_e_cascade",
            "a0": args.a0, "lambda_um": 0.8, "seeds": args.seeds, "dt": "T/200",
            "capacity_per_species": args.capacity, "precision": args.precision,
            "job_steps": r["steps"], "active_steps": r["active_steps"],
            "first_drop_step": r["first_drop_step"],
            "timed_steps": r["timed_steps"] if nt < r["steps"] else "all",
            "timed_particle_steps": r["timed_particle_steps"],
            "job_particle_steps": r["particle_steps"], "job_ms": round(r["job_ms"], 3),
            "job_value": r["value_job"], "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel_name(dom, args.precision),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "copy_gbs": copy_gbs,
            "frac_copy": achieved / copy_gbs if copy_gbs else None,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch",
            "algorithmic_bytes_per_launch": kbytes / launches,
            "avg_launch_us": kms * 1e3 / launches,
            "launches": launches,
        },
    }
    detail("rotating_e_cascade", {k: v for k, v in r.items() if not k.startswith("step_")})
    line["detail"] = {k: r[k] for k in ("saturated", "max_p_emit", "max_p_pair",
                                        "near_threshold", "nsub_refined", "dropped",
                                        "eager_matches_graph")}
    legs = {}
    if not args.no_mixed:
        other = "mixed" if args.precision == "f64" else "f64"
        print(f"bench: the same job in {other}", file=sys.stderr, flush=True)
        m = gpu_run(args, other)
        r64, rmx = (r, m) if args.precision == "f64" else (m, r)
        cmp_ = precision_compare(r64, rmx)
        detail("mixed_vs_f64", dict(lep_ms_mixed=rmx["lep_ms"], pho_ms_mixed=rmx["pho_ms"],
                                    lep_ms_f64=r64["lep_ms"], pho_ms_f64=r64["pho_ms"], **cmp_))
        legs["mixed_vs_f64"] = dict(
            value_f64=r64["value_job"], value_mixed=rmx["value_job"],
            speedup=rmx["value_job"] / r64["value_job"],
            spectrum_l1=cmp_["spectrum_l1_vs_f64"], pair_yield_rel=cmp_["pair_yield_rel_diff"])
    if not args.no_batched:
        # batched ensemble: 64 independent cascades in one step, mixed and FP64, full jobs
        b = {}
        for prec in ("mixed", "f64"):
            print(f"bench: batched ensemble, {prec}", file=sys.stderr, flush=True)
            b[prec] = gpu_run(args, prec, kind="batched")
        cmp_ = precision_compare(b["f64"], b["mixed"])
        bdom, bbytes, bms, bach = roofline_of(b["mixed"])
        for prec in ("mixed", "f64"):
            detail(f"batched_{prec}", {k: v for k, v in b[prec].items()
                                       if not k.startswith("step_")})
        legs["batched"] = dict(
            value_mixed=b["mixed"]["value_job"], value_f64=b["f64"]["value_job"],
            speedup=b["mixed"]["value_job"] / b["f64"]["value_job"],
            spectrum_l1=cmp_["spectrum_l1_vs_f64"], pair_yield_rel=cmp_["pair_yield_rel_diff"],
            frac_mixed=bach / HBM_PEAK_GBS)
    if not args.no_thin:
        # the same cascade past the capacity: the photon store is thinned to 40% of its
        # slots whenever it holds more than 80% (global even redistribution)
        cap = args.capacity
        print("bench: rotating-E cascade with thinning", file=sys.stderr, flush=True)
        rt = gpu_run(args, args.precision, thin=(int(0.8 * cap), int(0.4 * cap)))
        detail("thinned_cascade", {k: v for k, v in rt.items() if not k.startswith("step_")})
        legs["thinned_cascade"] = dict(value=rt["value_job"], thin_ms=rt["thin_ms"],
                                       dropped=rt["dropped"])
        # both cost controls of Sec. VI: photons created with probability 1/4 at four times
        # the weight, and the same thinning
        print("bench: rotating-E cascade with f_g = 4 for photons and thinning",
              file=sys.stderr, flush=True)
        rf = gpu_run(args, args.precision, thin=(int(0.8 * cap), int(0.4 * cap)),
                     fg=(4.0, 1.0))
        detail("generator_factor_cascade",
               {k: v for k, v in rf.items() if not k.startswith("step_")})
        legs["generator_factor_cascade"] = dict(value=rf["value_job"], dropped=rf["dropped"])
        # the other forms of Sec. VI and VII on the same job: the factor taken once every
        # f_g events, the reverse mode (two emission runs per sub-step at half the weight),
        # and at most one photon per lepton and step kept (the cap per parent), each with
        # the same global thinning past the capacity
        forms = {}
        for name, kw in (("every", dict(fg=(4.0, 1.0), over=dict(f_every=1))),
                         ("reverse", dict(over=dict(runs_photon=2))),
                         ("capped", dict(per_parent=1))):
            print(f"bench: rotating-E cascade, {name}", file=sys.stderr, flush=True)
            rr = gpu_run(args, args.precision, thin=(int(0.8 * cap), int(0.4 * cap)), **kw)
            detail(f"generator_forms_{name}",
                   {k: v for k, v in rr.items() if not k.startswith("step_")})
            forms[name] = rr["value_job"]
            forms[name + "_drop"] = rr["dropped"]
        legs["generator_forms"] = forms
    if not args.no_shower:
        sh = gpu_shower(args)
        detail("shower_time_step_invariance", sh)
        big = sh["large_dt_same_step"]
        legs["shower"] = dict(speedup=big["speedup_vs_small_dt"], max_abs_z=big["max_abs_z"],
                              saturated=big["saturated"])
    if not args.no_avalanche:
        av = gpu_avalanche(args)
        detail("avalanche_time_step_invariance", av)
        legs["avalanche"] = dict(
            speedup=av["large_dt_same_step"]["speedup_vs_small_dt"],
            growth_large=av["large_dt_same_step"].get("pair_growth_per_period"),
            growth_small=av["small_dt"].get("pair_growth_per_period"),
            saturated=av["large_dt_same_step"]["saturated"])
    if not args.no_yee:
        print("bench: standing-wave cascade on the Yee grid", file=sys.stderr, flush=True)
        y = gpu_run_yee(args, args.precision)
        detail("standing_wave_grid", y)
        legs["standing_wave_grid"] = dict(
            value=y["value"], step_ms=y["step_ms"], sort_every=y["sort_every"],
            sort_ms=round(y["sort_ms"], 2),
            lepton_frac=y["lepton_roofline_gbs"] / HBM_PEAK_GBS,
            photon_frac=y["photon_roofline_gbs"] / HBM_PEAK_GBS, saturated=y["saturated"])
        print("bench: the same cascade thinned per cell past its capacity", file=sys.stderr,
              flush=True)
        yt = gpu_run_yee(args, args.precision, thin=thin_cells_arg(args))
        detail("standing_wave_grid_thinned", yt)
        legs["grid_thinned"] = dict(value=yt["value"], thin_ms=round(yt["thin_ms"], 1),
                                    dropped=yt["dropped"])
    if not args.no_uniform_b:
        print("bench: uniform B, 10^4 electrons", file=sys.stderr, flush=True)
        u = gpu_uniform_b(args)
        detail("uniform_b", u)
        legs["uniform_b"] = dict(us_per_step_graph=u["us_per_step_graph"],
                                 lepton_steps_per_s_graph=u["lepton_steps_per_s_graph"])
    if not args.no_schwinger:
        print("bench: Schwinger pairs on the Yee grid", file=sys.stderr, flush=True)
        sc = gpu_schwinger_grid(args)
        detail("schwinger_grid", sc)
        legs["schwinger_grid"] = dict(avg_launch_us=sc["avg_launch_us"],
                                      frac=sc["roofline"]["frac"])
    if not args.no_generators:
        print("bench: the three emission generators", file=sys.stderr, flush=True)
        gc = gpu_generator_comparison(args)
        detail("generator_comparison", gc)
        legs["generator_comparison"] = {k: round(v["ms_per_launch"], 4)
                                        for k, v in gc["generators"].items()}
    line["legs"] = _rounded(legs)
    if not args.no_cpu_baseline:
        print("bench: oracle sample on the host", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
