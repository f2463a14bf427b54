"""Launch tuner for qed_step: work-chunk size (`tile`), persistent grid, child-arena size and
the lepton work queue's refill threshold.

What a step decides does not depend on these (every draw and child id is keyed by the
particle), only how fast it runs does, and that depends mostly on how many particles are
alive.  The tuner therefore works inside a run of the real job:

* the live count is split into size classes (a factor `class_factor` apart);
* when the run enters a new class, the next steps try the candidates, each step timed
  around the whole qed_step on the engine's stream.  First the launch shapes (the
  per-wavefront work queue's chunk size and the persistent grid) with the engine's own
  arena; then, with the best of those, the child-arena sizes (records = photon slots /
  divisor: the per-wavefront shares and pool the lepton and pair producers write their
  children into before the ordered copy), only those with room for the children of the
  class's last steps (a full arena sends children to slower direct reservations, which the
  first steps of a class may not show, and a class chosen by live count can come back with
  another mix of species, after a thinning: a choice whose arena some step of its class
  outgrew falls back to the engine's whole arena); then, with the best of those, the refill
  thresholds of the lepton kernel's work queue (idle lanes taken in batches of at least
  that many).  The lowest time per particle-step wins;
* the result is a schedule: (first step, shape) pairs, shape = (tile, grid, arena divisor,
  refill threshold).

A cascade is deterministic, so a second run of the same job from the same seeds reaches the
same counts at the same steps and can replay the schedule without synchronising, for
instance with one captured graph per shape.  Choices can be kept in a JSON file keyed by
(GPU architecture, precision, workload) and reused by later runs, which then skip the
trials for the size classes they know.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import qed as Q

# (tile, grid_blocks, arena divisor, refill threshold); 0 = the library's or the engine's
# default
Shape = Tuple[int, int, int, int]
DEFAULT_SHAPE: Shape = (0, 0, 0, 0)


def default_candidates(cu_count: int) -> List[Shape]:
    """Chunks of 64..512 particles on the library's resident grid, and 128-particle chunks
    on smaller and larger grids."""
    return [(64, 0, 0, 0), (128, 0, 0, 0), (256, 0, 0, 0), (512, 0, 0, 0),
            (128, 2 * cu_count, 0, 0), (128, 8 * cu_count, 0, 0)]


# Child-arena sizes tried with the best launch shape: photon slots / divisor records.
DEFAULT_ARENA_DIVISORS = (32, 8, 2)
# Refill thresholds tried last (1: every idle lane at once; 0, the library's default, is
# the shape they are compared with).
DEFAULT_REFILLS = (1, 16, 40)
# An arena is tried only if it holds ARENA_ROOM times the children of the class's busiest
# trial step, scaled by the class factor (the class ends with that many times the
# particles): half of an arena is the wavefronts' equal shares, which the busiest
# wavefronts outgrow first.
ARENA_ROOM = 2.0


def step_children(st) -> int:
    """Arena records a step's children take: a photon record per emission, and pair
    records, whose arena is a quarter of the photon arena's size, counted four times."""
    return int(st.get("emitted", 0)) + 4 * int(st.get("pairs", 0))


class HipTimer:
    """HIP events around one step on a stream."""

    def __init__(self):
        self.lib = C.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.lib.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        self.lib.hipEventSynchronize.argtypes = [C.c_void_p]
        self.lib.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.lib.hipEventDestroy.argtypes = [C.c_void_p]
        self.a, self.b = C.c_void_p(), C.c_void_p()
        if self.lib.hipEventCreate(C.byref(self.a)) or self.lib.hipEventCreate(C.byref(self.b)):
            raise RuntimeError("hipEventCreate failed")

    def start(self, stream: int):
        self.lib.hipEventRecord(self.a, C.c_void_p(stream))

    def stop_ms(self, stream: int) -> float:
        self.lib.hipEventRecord(self.b, C.c_void_p(stream))
        self.lib.hipEventSynchronize(self.b)
        f = C.c_float()
        self.lib.hipEventElapsedTime(C.byref(f), self.a, self.b)
        return float(f.value)

    def close(self):
        self.lib.hipEventDestroy(self.a)
        self.lib.hipEventDestroy(self.b)


@dataclass
class Schedule:
    """Shape per step: shapes[i] applies from steps[i] on."""
    steps: List[int] = field(default_factory=list)
    shapes: List[Shape] = field(default_factory=list)
    trials: List[Dict] = field(default_factory=list)
    choices: Dict[int, Shape] = field(default_factory=dict)  # size class -> shape

    def shape_at(self, n: int) -> Shape:
        s = self.shapes[0] if self.shapes else DEFAULT_SHAPE
        for k, sh in zip(self.steps, self.shapes):
            if n >= k:
                s = sh
        return s

    def distinct(self) -> List[Shape]:
        out: List[Shape] = []
        for s in self.shapes:
            if s not in out:
                out.append(s)
        return out or [DEFAULT_SHAPE]


class TuneCache:
    """Size-class choices kept in a JSON file, keyed by (arch, precision, workload)."""

    def __init__(self, path: str):
        self.path = path
        self.data: Dict[str, Dict[str, List[int]]] = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    @staticmethod
    def key(arch: str, precision: str, workload: str) -> str:
        return f"{arch}|{precision}|{workload}"

    def get(self, key: str) -> Dict[int, Shape]:
        # entries written before the refill threshold was tuned have three fields
        return {int(c): tuple(list(s) + [0] * (4 - len(s)))
                for c, s in self.data.get(key, {}).items()}

    def put(self, key: str, choices: Dict[int, Shape]):
        self.data[key] = {str(c): list(s) for c, s in sorted(choices.items())}
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def apply_shape(e, params: Q.qed_params, shape: Shape):
    """Set the launch shape and refill threshold in the step parameters and the arena size
    on the engine."""
    params.tile, params.grid_blocks = int(shape[0]), int(shape[1])
    params.refill_min = int(shape[3])
    e.set_arena(int(shape[2]))


def tune_run(e, field, params: Q.qed_params, n_steps: int, candidates: Sequence[Shape],
             arena_divisors: Sequence[int] = DEFAULT_ARENA_DIVISORS,
             refills: Sequence[int] = DEFAULT_REFILLS, rounds: int = 2,
             class_factor: float = 4.0, min_live: int = 1 << 16, stop_on_drop: bool = False,
             after_step: Optional[Callable[[], None]] = None, timer=None,
             known: Optional[Dict[int, Shape]] = None,
             sync: Optional[Callable[[], None]] = None) -> Schedule:
    """Run n_steps steps of the job on engine `e`, tuning the shape per size class.

    Below `min_live` live particles the default shape is used untimed (those steps are
    launch-bound).  `known` holds choices for size classes from an earlier run (a
    TuneCache); those classes are not tried again.  The returned schedule gives every step
    the best shape of its size class (trial steps included), and its `choices` every class
    chosen.  `after_step()`, if given, runs after every step (on the engine's stream) as
    part of the job, for instance thinning.  `timer` times one step on a stream (HipTimer by
    default); `sync` waits for the device at the end (torch.cuda.synchronize by default).
    `e` ends in the state after the run."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    ev = timer if timer is not None else HipTimer()
    trials: List[Dict] = []
    best: Dict[int, Shape] = dict(known or {})
    pending: List[Shape] = []
    timings: Dict[Shape, List[float]] = {}
    phase = 0  # 0: launch shapes, 1: arena sizes, 2: refill thresholds
    peak_children = 0  # the busiest trial step of the class being tuned
    records_for = getattr(e, "arena_records_for", None)
    class_children: Dict[int, int] = {}  # the busiest step of each class over the run
    cls_of_step: List[int] = []
    tuning: Optional[int] = None  # class whose trials are running

    def fastest():
        live = {s: v for s, v in timings.items() if v}
        return min(live, key=lambda s: min(live[s])) if live else None

    def start_phase(ph, base: Optional[Shape]):
        nonlocal phase, pending, timings
        phase = ph
        if ph == 0:
            cands = list(candidates)
        elif ph == 1:
            need = ARENA_ROOM * class_factor * peak_children
            cands = [(base[0], base[1], d, base[3]) for d in arena_divisors
                     if records_for is None or records_for(d) >= need]
        else:
            cands = [(base[0], base[1], base[2], r) for r in refills]
        if ph > 0 and base not in cands:
            cands.append(base)
        pending = [s for _ in range(rounds) for s in cands]
        timings = {s: [] for s in cands}

    def settle(c):
        """End the trials of class c: keep the best of what was timed."""
        if c is None or c in best:
            return
        b = fastest()
        if b is not None:
            best[c] = b

    live = int(e.counts().sum())
    stream = e.stream
    for n in range(n_steps):
        cls = -1 if live < min_live else int(math.log(live / min_live, class_factor))
        cls_of_step.append(cls)
        if cls >= 0 and cls not in best and cls != tuning:
            settle(tuning)  # a class left before its trials ended keeps its best so far
            tuning = cls
            peak_children = 0
            start_phase(0, None)
        if cls < 0:
            shape = DEFAULT_SHAPE
        elif cls in best:
            shape = best[cls]
        else:
            shape = pending.pop(0)
        apply_shape(e, params, shape)
        ev.start(stream)
        e.step(field, params)
        ms = ev.stop_ms(stream)
        if after_step is not None:
            after_step()
        st = e.stats()
        done = sum(st["advanced"])
        live = int(e.counts().sum())
        if cls >= 0:
            class_children[cls] = max(class_children.get(cls, 0), step_children(st))
        if cls >= 0 and cls not in best:
            peak_children = max(peak_children, step_children(st))
            if done > 0:
                timings[shape].append(ms / done)
            trials.append(dict(step=n, cls=cls, tile=shape[0], grid=shape[1],
                               arena_div=shape[2], refill=shape[3], ms=ms,
                               particle_steps=done))
            if not pending:
                b = fastest()
                nxt = phase + 1
                if nxt == 1 and not arena_divisors:
                    nxt = 2
                if b is None or nxt > 2 or (nxt == 2 and not refills):
                    settle(cls)
                else:
                    start_phase(nxt, b)
        if stop_on_drop and st["dropped"] > 0:
            break
    settle(tuning)
    if records_for is not None:
        for c, s in list(best.items()):
            if s[2] > 0 and records_for(s[2]) < ARENA_ROOM * class_children.get(c, 0):
                best[c] = (s[0], s[1], 0, s[3])
    sync()
    if timer is None:
        ev.close()
    sched = Schedule(trials=trials, choices=dict(best))
    for n, cls in enumerate(cls_of_step):
        shape = best.get(cls, DEFAULT_SHAPE) if cls >= 0 else DEFAULT_SHAPE
        if not sched.shapes or sched.shapes[-1] != shape:
            sched.steps.append(n)
            sched.shapes.append(shape)
    return sched
