"""Set up and drive the GPU step for a seeded workload (see workloads.py)."""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from . import qed as Q
from . import workloads as W
from .engine import Engine

PRECISION = {"f64": Q.QED_FP64, "mixed": Q.QED_MIXED}


def field_of(w: W.Workload, grid=None) -> Q.qed_field:
    f = w.field
    if f.kind == W.FIELD_YEE:
        return Engine.make_field(Q.QED_FIELD_YEE, grid=grid, n=f.grid_n, dx=f.grid_dx,
                                 origin=f.grid_origin, amp=f.grid_wave_amp, omega=f.omega)
    return Engine.make_field(f.kind, e0=f.e0, b0=f.b0, amp=f.amp, omega=f.omega, phase=f.phase)


def params_of(w: W.Workload, **over) -> Q.qed_params:
    kw = dict(dt=w.dt, eps_r=w.eps_r, kappa=w.kappa, t0=w.t0, adaptive=w.adaptive,
              emission=w.emission, pairs=w.pairs, push_photons=w.push_photons,
              precision=PRECISION[w.precision], freeze_on_drop=1 if w.instances > 1 else 0)
    kw.update(over)
    return Engine.make_params(**kw)


def engine_single(w: W.Workload, init: Sequence[Dict[str, np.ndarray]],
                  capacity: Optional[Sequence[int]] = None, seed: Optional[int] = None,
                  build_tables: bool = True, arena_records: Optional[int] = None,
                  same_step: bool = False) -> Engine:
    cap = tuple(capacity) if capacity is not None else tuple(w.capacity)
    e = Engine([cap], [w.seed if seed is None else seed], arena_records=arena_records,
               same_step=same_step)
    if build_tables:
        e.build_tables()
    for s in range(3):
        e.load(0, s, init[s])
    return e


def engine_batched(w: W.Workload, inits: Sequence[Sequence[Dict[str, np.ndarray]]],
                   build_tables: bool = True, arena_records: Optional[int] = None,
                   same_step: bool = False) -> Engine:
    caps = [tuple(w.instance_capacity)] * w.instances
    e = Engine(caps, list(range(w.instances)), amps=w.instance_amp,
               arena_records=arena_records, same_step=same_step)
    if build_tables:
        e.build_tables()
    for i, init in enumerate(inits):
        for s in range(3):
            e.load(i, s, init[s])
    return e


class YeeGrid:
    """Six FP32 device arrays of a periodic Yee grid, refilled with the standing wave at
    every step (the workload's stand-in for a field solver)."""

    def __init__(self, w: W.Workload, device="cuda:0"):
        import torch
        nx, ny, nz = w.field.grid_n
        self.w = w
        self.g = [torch.zeros((nz, ny, nx), dtype=torch.float32, device=device) for _ in range(6)]

    def fill(self, t: float, stream: int):
        f = self.w.field
        Q.qed_fill_standing_wave([g.data_ptr() for g in self.g], f.grid_n, f.grid_dx,
                                 f.grid_origin, f.grid_wave_amp, f.omega, f.phase, t, stream)

    def load_numpy(self, arrays: List[np.ndarray]):
        import torch
        for g, a in zip(self.g, arrays):
            g.copy_(torch.from_numpy(a))


def run(e: Engine, field: Q.qed_field, params: Q.qed_params, n_steps: int,
        stop_on_drop: bool = True, grid: Optional[YeeGrid] = None, dt: float = 0.0,
        t0: float = 0.0, first_step: int = 0) -> List[Dict]:
    """Advance n_steps steps, reading the stats record after each (synchronising)."""
    import torch
    out = []
    e.set_step(first_step)
    for n in range(first_step, first_step + n_steps):
        if grid is not None:
            grid.fill(t0 + n * dt, e.stream)
        e.step(field, params)
        torch.cuda.synchronize()
        s = e.stats()
        s["counts"] = e.counts().tolist()
        out.append(s)
        if stop_on_drop and s["dropped"] > 0:
            break
    return out
