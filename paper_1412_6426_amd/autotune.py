"""Launch-shape tuner for qed_step: work-chunk size (`tile`) and persistent grid.

What a step decides does not depend on the launch shape (every draw and child id is keyed
by the particle), only how fast it runs does, and that depends mostly on how many
particles are alive.  The tuner therefore works inside a run of the real job:

* the live count is split into size classes (a factor `class_factor` apart);
* when the run enters a new class, the next steps cycle through the candidate shapes,
  each step timed with HIP events around the whole qed_step on the engine's stream, and
  the shape with the lowest time per particle-step becomes the class's choice;
* the result is a schedule: (first step, shape) pairs.

A cascade is deterministic, so a second run of the same job from the same seeds reaches
the same counts at the same steps and can replay the schedule without synchronising,
for instance with one captured graph per shape.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

from . import qed as Q

Shape = Tuple[int, int]  # (tile, grid_blocks); 0 = library default


def default_candidates(cu_count: int) -> List[Shape]:
    """Chunks of 64..512 particles on the library's resident grid, and 128-particle chunks
    on smaller and larger grids."""
    return [(64, 0), (128, 0), (256, 0), (512, 0), (128, 2 * cu_count), (128, 8 * cu_count)]


class _Events:
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
    """Launch shape per step: shapes[i] applies from steps[i] on."""
    steps: List[int] = field(default_factory=list)
    shapes: List[Shape] = field(default_factory=list)
    trials: List[Dict] = field(default_factory=list)

    def shape_at(self, n: int) -> Shape:
        s = self.shapes[0] if self.shapes else (0, 0)
        for k, sh in zip(self.steps, self.shapes):
            if n >= k:
                s = sh
        return s

    def distinct(self) -> List[Shape]:
        out: List[Shape] = []
        for s in self.shapes:
            if s not in out:
                out.append(s)
        return out or [(0, 0)]


def tune_run(e, field, params: Q.qed_params, n_steps: int, candidates: Sequence[Shape],
             rounds: int = 2, class_factor: float = 4.0, min_live: int = 1 << 16,
             stop_on_drop: bool = False, after_step=None) -> Schedule:
    """Run n_steps steps of the job on engine `e`, tuning the shape per size class.

    Below `min_live` live particles the library default shape is used untimed (those steps
    are launch-bound).  The returned schedule gives every step the best shape of its size
    class (trial steps included).  `after_step()`, if given, runs after every step (on the
    engine's stream) as part of the job, for instance thinning.  `e` ends in the state
    after the run."""
    import torch

    ev = _Events()
    trials: List[Dict] = []
    best: Dict[int, Shape] = {}
    pending: List[Shape] = []
    timings: Dict[Shape, List[float]] = {}
    cls_of_step: List[int] = []
    tuning: Optional[int] = None  # class whose trials are running

    def settle(c):
        if c is not None and c not in best and any(timings.values()):
            best[c] = min(timings, key=lambda s: min(timings[s]) if timings[s] else math.inf)

    live = int(e.counts().sum())
    stream = e.stream
    for n in range(n_steps):
        cls = -1 if live < min_live else int(math.log(live / min_live, class_factor))
        cls_of_step.append(cls)
        if cls >= 0 and cls not in best and cls != tuning:
            settle(tuning)  # a class left before its trials ended keeps its best so far
            tuning = cls
            pending = [c for _ in range(rounds) for c in candidates]
            timings = {c: [] for c in candidates}
        if cls < 0:
            shape = (0, 0)
        elif cls in best:
            shape = best[cls]
        else:
            shape = pending.pop(0)
        params.tile, params.grid_blocks = shape
        ev.start(stream)
        e.step(field, params)
        ms = ev.stop_ms(stream)
        if after_step is not None:
            after_step()
        st = e.stats()
        done = sum(st["advanced"])
        live = int(e.counts().sum())
        if cls >= 0 and cls not in best:
            if done > 0:
                timings[shape].append(ms / done)
            trials.append(dict(step=n, cls=cls, tile=shape[0], grid=shape[1], ms=ms,
                               particle_steps=done))
            if not pending:
                settle(cls)
        if stop_on_drop and st["dropped"] > 0:
            break
    settle(tuning)
    torch.cuda.synchronize()
    ev.close()
    sched = Schedule(trials=trials)
    for n, cls in enumerate(cls_of_step):
        shape = best.get(cls, (0, 0)) if cls >= 0 else (0, 0)
        if not sched.shapes or sched.shapes[-1] != shape:
            sched.steps.append(n)
            sched.shapes.append(shape)
    return sched
