#!/usr/bin/env python3
"""Benchmark of the GPU QED step on the rotating-electric-field cascade.

Workload (default): E = a0 (cos t, sin t, 0), B = 0, a0 = 1000, lambda = 0.8 um;
10^5 seed electrons at rest, uniform in a 1 um^3 box; emission + Breit-Wheeler pairs;
dt = T/200; 3 laser periods (600 steps); capacity 10^8 per species store.  One "step" is
one global time step of the whole hot path (fields, chi, adaptive sub-steps, Boris push,
emission and pair decisions, append) over every live particle.  The cascade grows until a
store is full; from then on the instance is frozen (its steps do nothing) and the run's
particle-step count stops growing.

Prints one JSON line: particle-steps/s over the timed steps, the roofline of the dominant
kernel (algorithmic bytes / its event-timed duration vs 8 TB/s), and the FP64 CPU
oracle's rate on a bounded sample of the same workload on this host.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# algorithmic bytes (per unit of work) of the two persistent kernels
LEPTON_STEP_BYTES = 112   # read x,p (48) id (8) n_events (4); write x,p (48) n_events (4)
PHOTON_STEP_BYTES = 80    # read x,k (48) id (8); write x (24)
DEAD_SLOT_BYTES = 8       # id of a removed photon, read and skipped
EMISSION_BYTES = 84       # photon child written (x,k,w,id,parent,birth = 76) + parent w read (8)
PAIR_BYTES = 176          # two lepton children (2 x 80) + photon w read (8) + tombstone id (8)


class HipEvents:
    """Raw hipEvent_t handles (timing), for kernels launched inside libqed on our stream."""

    def __init__(self):
        self.lib = C.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.lib.hipEventDestroy.argtypes = [C.c_void_p]

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


def gpu_run(args, precision):
    import numpy as np
    import torch
    from paper_1412_6426_amd import qed as Q
    from paper_1412_6426_amd import runner as R
    from paper_1412_6426_amd import workloads as W

    w = W.rotating_e(n=args.seeds, a0=args.a0, periods=3.0, capacity=args.capacity,
                     precision=precision)
    init = W.rotating_e_initial(args.seeds, seed=0)
    e = R.engine_single(w, init)
    field = R.field_of(w)
    params = R.params_of(w, freeze_on_drop=1, tile=args.tile, grid_blocks=args.grid_blocks)
    torch.cuda.synchronize()

    # warm-up steps on the same stores, then back to the seed state
    for _ in range(args.warmup):
        e.step(field, params)
    torch.cuda.synchronize()
    e.reset_instances()
    for s in range(3):
        e.load(0, s, init[s])
    e.set_step(0)
    torch.cuda.synchronize()

    K = args.steps if args.steps is not None else w.n_steps
    hip = HipEvents()
    evs = hip.create(4 * K)
    log = torch.zeros(K * e.stats_buf.numel(), dtype=torch.uint8, device=e.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=e.device)
    stream = e.stream
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for n in range(K):
        for j in range(4):
            params.events[j] = evs[4 * n + j]
        e.step(field, params)
        Q.qed_append_stats(e.stats_buf.data_ptr(), log.data_ptr(), K, cnt.data_ptr(), stream)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t_start.elapsed_time(t_end)

    raw = log.cpu().numpy().tobytes()
    recs = [Q.qed_stats.from_buffer_copy(raw[i * C.sizeof(Q.qed_stats):(i + 1) * C.sizeof(Q.qed_stats)])
            for i in range(K)]
    lep_ms = sum(hip.elapsed_ms(evs[4 * n], evs[4 * n + 1]) for n in range(K))
    pho_ms = sum(hip.elapsed_ms(evs[4 * n + 2], evs[4 * n + 3]) for n in range(K))
    hip.destroy(evs)
    adv = [sum(r.advanced[s] for r in recs) for s in range(3)]
    dead_slots = sum(r.n_start[2] - r.advanced[2] for r in recs)
    emitted = sum(r.emitted for r in recs)
    pairs = sum(r.pairs for r in recs)
    lep_bytes = LEPTON_STEP_BYTES * (adv[0] + adv[1]) + EMISSION_BYTES * emitted
    pho_bytes = PHOTON_STEP_BYTES * adv[2] + DEAD_SLOT_BYTES * dead_slots + PAIR_BYTES * pairs
    active = sum(1 for r in recs if sum(r.advanced) > 0)
    first_drop = next((r.step for r in recs if r.dropped > 0), None)
    out = dict(
        ms=ms, wall_s=wall, steps=K, active_steps=active, first_drop_step=first_drop,
        particle_steps=int(sum(adv)), advanced=[int(a) for a in adv], emitted=int(emitted),
        pairs=int(pairs), lep_ms=lep_ms, pho_ms=pho_ms, lep_bytes=lep_bytes,
        pho_bytes=pho_bytes, final_counts=e.counts()[0].tolist(),
        substeps=int(sum(r.substeps for r in recs)),
        low_occupancy_iters=int(sum(r.low_occupancy_iters for r in recs)),
        wave_iters=int(sum(r.wave_iters for r in recs)),
        near_threshold=int(sum(r.near_threshold for r in recs)),
        saturated=int(sum(r.saturated for r in recs)),
        early_out=int(sum(r.early_out for r in recs)),
    )
    if args.spectrum:
        hist = torch.zeros(W.SPECTRUM_BINS, dtype=torch.float64, device=e.device)
        Q.qed_photon_spectrum(e.stores, W.SPECTRUM_LO, W.SPECTRUM_HI, W.SPECTRUM_BINS,
                              hist.data_ptr(), stream)
        torch.cuda.synchronize()
        out["spectrum"] = hist.cpu().numpy()
    del e
    torch.cuda.empty_cache()
    return out


def cpu_baseline(args):
    """The FP64 oracle on a bounded sample of the same workload: the rotating-field
    cascade from `cpu_seeds` seeds, stepped until ~cpu_seconds of CPU time has passed."""
    from oracle import oracle as orc
    from paper_1412_6426_amd import workloads as W
    from tests.parity_util import oracle_field, oracle_params, oracle_stores

    w = W.rotating_e(n=args.cpu_seeds, a0=args.a0, periods=3.0, capacity=4_000_000,
                     lepton_capacity=400_000)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: 600)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=("f64", "mixed"), default="f64")
    ap.add_argument("--seeds", type=int, default=100_000)
    ap.add_argument("--a0", type=float, default=1000.0)
    ap.add_argument("--capacity", type=int, default=100_000_000)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--cpu-seeds", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-mixed", action="store_true",
                    help="also run the mixed-precision form and report its rate and accuracy")
    ap.add_argument("--spectrum", action="store_true")
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
    if args.compare_mixed:
        args.spectrum = True
    print(f"bench: rotating-E cascade, {args.seeds} seeds, precision {args.precision}",
          file=sys.stderr, flush=True)
    r = gpu_run(args, args.precision)
    secs = r["ms"] / 1e3
    value = r["particle_steps"] / secs
    dom = "photon" if r["pho_ms"] >= r["lep_ms"] else "lepton"
    kbytes = r["pho_bytes"] if dom == "photon" else r["lep_bytes"]
    kms = r["pho_ms"] if dom == "photon" else r["lep_ms"]
    achieved = kbytes / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    line = {
        "metric": "QED particle-steps/s (rotating-E cascade)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / r["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f64+f32 (mixed)",
        "data": "synthetic (seeded)",
        "config": {
            "workload": "rotating_e_cascade",
            "a0": args.a0, "lambda_um": 0.8, "seeds": args.seeds, "dt": "T/200",
            "job_steps": 600, "capacity_per_species": args.capacity,
            "precision": args.precision, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom}_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
        },
        "detail": {k: r[k] for k in ("active_steps", "first_drop_step", "particle_steps",
                                     "advanced", "emitted", "pairs", "final_counts",
                                     "lep_ms", "pho_ms", "substeps", "wave_iters",
                                     "low_occupancy_iters", "near_threshold", "saturated",
                                     "early_out")},
    }
    if args.compare_mixed:
        import numpy as np
        m = gpu_run(args, "mixed")
        h64, hm = r["spectrum"], m["spectrum"]
        l1 = float(np.abs(hm - h64).sum() / max(h64.sum(), 1e-300))
        line["mixed"] = {
            "value": m["particle_steps"] / (m["ms"] / 1e3),
            "speedup_vs_f64": (m["particle_steps"] / m["ms"]) / (r["particle_steps"] / r["ms"]),
            "spectrum_l1_vs_f64": l1,
            "pairs_f64": r["pairs"], "pairs_mixed": m["pairs"],
            "pair_yield_rel_diff": (m["pairs"] - r["pairs"]) / max(r["pairs"], 1),
            "lep_ms": m["lep_ms"], "pho_ms": m["pho_ms"],
        }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
