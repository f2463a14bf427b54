"""Device-memory owner around the C ABI: stores, instance table, tables, workspace, stats.

PyTorch tensors provide the device memory and the stream; every call into the QED step
goes through ``qed.py`` to libqed's kernels.  The helpers here only copy seeded inputs in
and results out.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import qed as Q

FLOAT_COLS = ("x", "y", "z", "px", "py", "pz", "w")


def _torch():
    import torch
    return torch


class Engine:
    """SoA stores for n instances, each owning a segment of every species store."""

    def __init__(self, capacities: Sequence[Tuple[int, int, int]], seeds: Sequence[int],
                 amps: Optional[Sequence[float]] = None, device: str = "cuda:0",
                 arena_records: Optional[int] = None, same_step: bool = False):
        torch = _torch()
        if not torch.cuda.is_available():
            raise Q.QedError("no HIP device visible: the QED step runs only on the GPU")
        self.device = torch.device(device)
        self.n_inst = len(capacities)
        if amps is None:
            amps = [1.0] * self.n_inst
        caps = np.asarray(capacities, dtype=np.int64).reshape(self.n_inst, 3)
        self.caps = caps
        self.base = np.zeros_like(caps)
        self.base[1:] = np.cumsum(caps, axis=0)[:-1]
        self.total = caps.sum(axis=0)
        self.cols: List[Dict[str, "torch.Tensor"]] = []
        for s in range(3):
            n = max(int(self.total[s]), 1)
            d = {c: torch.zeros(n, dtype=torch.float64, device=self.device) for c in FLOAT_COLS}
            d["id"] = torch.zeros(n, dtype=torch.int64, device=self.device)
            d["parent"] = torch.zeros(n, dtype=torch.int64, device=self.device)
            d["birth"] = torch.zeros(n, dtype=torch.int32, device=self.device)
            d["n_events"] = torch.zeros(n, dtype=torch.int32, device=self.device)
            self.cols.append(d)
        inst = (Q.qed_instance * self.n_inst)()
        for i in range(self.n_inst):
            for s in range(3):
                inst[i].base[s] = int(self.base[i, s])
                inst[i].capacity[s] = int(caps[i, s])
                inst[i].count[s] = 0
            inst[i].dropped = 0
            inst[i].seed = int(seeds[i])
            inst[i].amp = float(amps[i])
            inst[i].frozen = 0
        self._inst_init = np.frombuffer(bytes(inst), dtype=np.uint8).copy()
        self.inst = torch.from_numpy(self._inst_init.copy()).to(self.device)
        self.tables = torch.zeros(Q.qed_table_bytes(), dtype=torch.uint8, device=self.device)
        pslots = int(self.cols[2]["x"].numel())
        if arena_records is None:
            # same-step processing advances only the children that reach an arena (a full
            # wavefront share defers them), so it gets roomier arenas
            floor = 1 << 20 if same_step else 1 << 18
            arena_records = min(max(pslots // 8, floor), 1 << 26)
        self.arena_records = int(arena_records)
        # same_step: room for advancing children in their birth step
        # (qed_params.same_step_generations > 0)
        self.work_bytes = Q.qed_work_bytes(self.n_inst, pslots, self.arena_records, same_step)
        self.work = torch.zeros(self.work_bytes, dtype=torch.uint8, device=self.device)
        self._pslots, self._same_step = pslots, same_step
        self.step_work_bytes = self.work_bytes  # what qed_step is told (set_arena)
        self.stats_buf = torch.zeros(C.sizeof(Q.qed_stats), dtype=torch.uint8, device=self.device)
        self.step_ctr = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.stores = Q.qed_stores()
        for s in range(3):
            soa = self.stores.species[s]
            d = self.cols[s]
            for c in FLOAT_COLS:
                setattr(soa, c, C.cast(C.c_void_p(d[c].data_ptr()), Q._dp))
            soa.id = C.cast(C.c_void_p(d["id"].data_ptr()), Q._u64p)
            soa.parent = C.cast(C.c_void_p(d["parent"].data_ptr()), Q._u64p)
            soa.birth = C.cast(C.c_void_p(d["birth"].data_ptr()), Q._u32p)
            soa.n_events = C.cast(C.c_void_p(d["n_events"].data_ptr()), Q._u32p)
        for s in range(3):
            self.stores.slots[s] = int(self.cols[s]["x"].numel())
        self.stores.d_instances = self.inst.data_ptr()
        self.stores.n_instances = self.n_inst

    # ------------------------------------------------------------------ helpers
    @property
    def stream(self) -> int:
        return _torch().cuda.current_stream(self.device).cuda_stream

    def reset_instances(self):
        """Back to the constructed descriptors: counts 0, nothing dropped or frozen."""
        self.inst.copy_(_torch().from_numpy(self._inst_init.copy()))

    def build_tables(self):
        Q.qed_build_tables(self.tables.data_ptr(), self.tables.numel(), self.stream)

    def set_step(self, n: int):
        self.step_ctr.fill_(int(n))

    def load(self, inst: int, species: int, cols: Dict[str, np.ndarray]):
        """Copy seeded columns into the instance's segment and set its count."""
        torch = _torch()
        n = len(cols["x"])
        if n > self.caps[inst, species]:
            raise ValueError("more particles than the segment's capacity")
        b = int(self.base[inst, species])
        d = self.cols[species]
        for c in FLOAT_COLS:
            d[c][b:b + n] = torch.from_numpy(np.ascontiguousarray(cols[c], dtype=np.float64))
        d["id"][b:b + n] = torch.from_numpy(np.asarray(cols["id"], dtype=np.uint64).view(np.int64))
        par = cols.get("parent", np.full(n, Q.QED_NO_PARENT, dtype=np.uint64))
        d["parent"][b:b + n] = torch.from_numpy(np.asarray(par, dtype=np.uint64).view(np.int64))
        bir = cols.get("birth", np.zeros(n, dtype=np.uint32))
        d["birth"][b:b + n] = torch.from_numpy(np.asarray(bir, dtype=np.uint32).view(np.int32))
        ne = cols.get("n_events", np.zeros(n, dtype=np.uint32))
        d["n_events"][b:b + n] = torch.from_numpy(np.asarray(ne, dtype=np.uint32).view(np.int32))
        self._set_count(inst, species, n)

    def _instances_host(self):
        raw = self.inst.cpu().numpy().tobytes()
        return (Q.qed_instance * self.n_inst).from_buffer_copy(raw)

    def _set_count(self, inst: int, species: int, n: int):
        off = inst * C.sizeof(Q.qed_instance) + Q.qed_instance.count.offset + 8 * species
        self.inst[off:off + 8] = _torch().from_numpy(
            np.frombuffer(np.int64(n).tobytes(), dtype=np.uint8).copy()).to(self.device)

    def set_frozen(self, inst: int, frozen: bool = True):
        """Freeze (skip) or release one instance."""
        off = inst * C.sizeof(Q.qed_instance) + Q.qed_instance.frozen.offset
        self.inst[off:off + 4] = _torch().from_numpy(
            np.frombuffer(np.int32(1 if frozen else 0).tobytes(), dtype=np.uint8).copy()).to(
                self.device)

    def instances(self) -> List[Dict]:
        out = []
        for r in self._instances_host():
            out.append({"count": list(r.count), "dropped": r.dropped, "frozen": r.frozen,
                        "capacity": list(r.capacity), "base": list(r.base), "seed": r.seed,
                        "amp": r.amp})
        return out

    def counts(self) -> np.ndarray:
        return np.array([r["count"] for r in self.instances()], dtype=np.int64)

    def read(self, inst: int, species: int) -> Dict[str, np.ndarray]:
        """Live slots of one instance's segment, as numpy arrays (ids as uint64)."""
        n = int(self.counts()[inst, species])
        b = int(self.base[inst, species])
        d = self.cols[species]
        out = {c: d[c][b:b + n].cpu().numpy() for c in FLOAT_COLS}
        out["id"] = d["id"][b:b + n].cpu().numpy().view(np.uint64)
        out["parent"] = d["parent"][b:b + n].cpu().numpy().view(np.uint64)
        out["birth"] = d["birth"][b:b + n].cpu().numpy().view(np.uint32)
        out["n_events"] = d["n_events"][b:b + n].cpu().numpy().view(np.uint32)
        return out

    def stats(self) -> Dict:
        raw = self.stats_buf.cpu().numpy().tobytes()
        return Q.qed_stats.from_buffer_copy(raw).as_dict()

    # ------------------------------------------------------------------ thinning
    def thin(self, species: int, trigger: int, target: int, stream: Optional[int] = None):
        """qed_thin on one species of every instance; records stay on the device until
        thin_records() reads them."""
        torch = _torch()
        need = max(Q.qed_thin_work_bytes(self.n_inst, int(self.cols[s]["x"].numel()))
                   for s in range(3))
        if getattr(self, "_thin_work", None) is None or self._thin_work.numel() < need:
            torch.cuda.synchronize()  # no call may still use a buffer being replaced
            self._thin_work = torch.zeros(need, dtype=torch.uint8, device=self.device)
            self._thin_rec = torch.zeros(self.n_inst * C.sizeof(Q.qed_thin_record),
                                         dtype=torch.uint8, device=self.device)
        Q.qed_thin(self.stores, species, int(trigger), int(target), self.step_ctr.data_ptr(),
                   self._thin_rec.data_ptr(), self._thin_work.data_ptr(),
                   self._thin_work.numel(), self.stream if stream is None else stream)

    def thin_records(self) -> List[Dict]:
        raw = self._thin_rec.cpu().numpy().tobytes()
        n = C.sizeof(Q.qed_thin_record)
        return [Q.qed_thin_record.from_buffer_copy(raw[i * n:(i + 1) * n]).as_dict()
                for i in range(self.n_inst)]

    def thin_cells(self, species: int, field: Q.qed_field, max_per_cell: int,
                   stream: Optional[int] = None):
        """qed_thin_cells on one species of every instance (workspace allocated on first
        use); records stay on the device until thin_cells_records() reads them."""
        torch = _torch()
        # sized once for the largest store: a buffer replaced while a call on another
        # stream still used it would be reused by the allocator under that call
        need = max(Q.qed_thin_cells_work_bytes(self.n_inst, int(self.cols[s]["x"].numel()))
                   for s in range(3))
        if getattr(self, "_tc_work", None) is None or self._tc_work.numel() < need:
            torch.cuda.synchronize()
            self._tc_work = torch.zeros(need, dtype=torch.uint8, device=self.device)
            self._tc_rec = torch.zeros(self.n_inst * C.sizeof(Q.qed_thin_cells_record),
                                       dtype=torch.uint8, device=self.device)
        Q.qed_thin_cells(self.stores, species, field, int(max_per_cell),
                         self.step_ctr.data_ptr(), self._tc_rec.data_ptr(),
                         self._tc_work.data_ptr(), self._tc_work.numel(),
                         self.stream if stream is None else stream)

    def thin_cells_records(self) -> List[Dict]:
        raw = self._tc_rec.cpu().numpy().tobytes()
        n = C.sizeof(Q.qed_thin_cells_record)
        return [Q.qed_thin_cells_record.from_buffer_copy(raw[i * n:(i + 1) * n]).as_dict()
                for i in range(self.n_inst)]

    def thin_children(self, species: int, max_per_parent: int, stream: Optional[int] = None):
        """qed_thin_children on one species of every instance, after the step the step
        counter has just passed (workspace allocated on first use, for the largest store);
        records stay on the device until thin_children_records() reads them."""
        torch = _torch()
        need = max(Q.qed_thin_children_work_bytes(self.n_inst, int(self.cols[s]["x"].numel()))
                   for s in range(3))
        if getattr(self, "_tp_work", None) is None or self._tp_work.numel() < need:
            torch.cuda.synchronize()  # no call may still use a buffer being replaced
            self._tp_work = torch.zeros(need, dtype=torch.uint8, device=self.device)
            self._tp_rec = torch.zeros(self.n_inst * C.sizeof(Q.qed_thin_children_record),
                                       dtype=torch.uint8, device=self.device)
        Q.qed_thin_children(self.stores, species, int(max_per_parent), self.step_ctr.data_ptr(),
                            self._tp_rec.data_ptr(), self._tp_work.data_ptr(),
                            self._tp_work.numel(), self.stream if stream is None else stream)

    def thin_children_records(self) -> List[Dict]:
        raw = self._tp_rec.cpu().numpy().tobytes()
        n = C.sizeof(Q.qed_thin_children_record)
        return [Q.qed_thin_children_record.from_buffer_copy(raw[i * n:(i + 1) * n]).as_dict()
                for i in range(self.n_inst)]

    # ------------------------------------------------------------------ cell sort
    def sort_cells(self, species: int, field: Q.qed_field, stream: Optional[int] = None):
        """qed_sort_cells on one species of every instance (workspace allocated on first
        use, large enough for any species)."""
        torch = _torch()
        need = max(Q.qed_sort_work_bytes(self.n_inst, int(self.cols[s]["x"].numel()))
                   for s in range(3))
        if getattr(self, "_sort_work", None) is None or self._sort_work.numel() < need:
            torch.cuda.synchronize()  # no call may still use a buffer being replaced
            self._sort_work = torch.zeros(need, dtype=torch.uint8, device=self.device)
        Q.qed_sort_cells(self.stores, species, field, self._sort_work.data_ptr(),
                         self._sort_work.numel(), self.stream if stream is None else stream)

    # ------------------------------------------------------------------ Schwinger pairs
    def schwinger(self, field: Q.qed_field, dt: float, eps_r: float, weight: float = 1.0,
                  stream: Optional[int] = None):
        """qed_schwinger for step n = the step counter, on every instance; the record stays
        on the device until schwinger_record() reads it."""
        Q.qed_schwinger(self.stores, field, float(dt), float(eps_r), float(weight),
                        self.step_ctr.data_ptr(), self.schwinger_record_buffer().data_ptr(),
                        self.stream if stream is None else stream)

    def schwinger_record_buffer(self):
        """The device bytes of the last qed_schwinger record (allocated on first use)."""
        if not hasattr(self, "_sch_rec"):
            torch = _torch()
            self._sch_rec = torch.zeros(C.sizeof(Q.qed_schwinger_record), dtype=torch.uint8,
                                        device=self.device)
        return self._sch_rec

    @staticmethod
    def decode_schwinger_record(raw: bytes) -> Dict:
        return Q.qed_schwinger_record.from_buffer_copy(raw).as_dict()

    def schwinger_record(self) -> Dict:
        return self.decode_schwinger_record(self.schwinger_record_buffer().cpu().numpy().tobytes())

    # ------------------------------------------------------------------ the step
    @staticmethod
    def make_field(kind: int, e0=(0, 0, 0), b0=(0, 0, 0), amp=0.0, omega=1.0, phase=0.0,
                   grid=None, n=(0, 0, 0), dx=(1, 1, 1), origin=(0, 0, 0)) -> Q.qed_field:
        f = Q.qed_field()
        f.kind = kind
        f.e0 = (C.c_double * 3)(*[float(v) for v in e0])
        f.b0 = (C.c_double * 3)(*[float(v) for v in b0])
        f.amp, f.omega, f.phase = float(amp), float(omega), float(phase)
        if grid is not None:
            for i, g in enumerate(grid):
                f.grid[i] = C.cast(C.c_void_p(g.data_ptr()), Q._fp)
        f.n = (C.c_int * 3)(*[int(v) for v in n])
        f.dx = (C.c_double * 3)(*[float(v) for v in dx])
        f.origin = (C.c_double * 3)(*[float(v) for v in origin])
        return f

    @staticmethod
    def make_params(dt, eps_r, kappa=1.0, t0=0.0, adaptive=1, forced_substeps=0, emission=1,
                    pairs=1, push_photons=1, precision=Q.QED_FP64, freeze_on_drop=0, tile=0,
                    block=0, grid_blocks=0, f_photon=1.0, f_pair=1.0,
                    same_step_generations=0, f_every=0, runs_photon=1,
                    runs_pair=1, refill_min=0) -> Q.qed_params:
        p = Q.qed_params()
        p.f_photon, p.f_pair = float(f_photon), float(f_pair)
        p.same_step_generations = int(same_step_generations)
        p.f_every, p.runs_photon, p.runs_pair = int(f_every), int(runs_photon), int(runs_pair)
        p.refill_min = int(refill_min)
        p.dt, p.eps_r, p.kappa, p.t0 = float(dt), float(eps_r), float(kappa), float(t0)
        p.adaptive, p.forced_substeps = int(adaptive), int(forced_substeps)
        p.emission, p.pairs, p.push_photons = int(emission), int(pairs), int(push_photons)
        p.precision, p.freeze_on_drop = int(precision), int(freeze_on_drop)
        p.tile, p.block, p.grid_blocks = int(tile), int(block), int(grid_blocks)
        return p

    def arena_records_for(self, divisor: int = 0) -> int:
        """Records of the photon arena that set_arena(divisor) gives (bounded by the
        workspace allocated at construction)."""
        if divisor <= 0:
            return self.arena_records
        return min(max(self._pslots // int(divisor), 1024), self.arena_records)

    def set_arena(self, divisor: int = 0):
        """Child arenas of photon slots / divisor records for the following steps (within
        the workspace allocated at construction; qed_step uses the largest arena that fits
        in the bytes it is given); 0: the whole workspace."""
        if divisor <= 0:
            self.step_work_bytes = self.work_bytes
            return
        records = max(self._pslots // int(divisor), 1024)
        need = Q.qed_work_bytes(self.n_inst, self._pslots, records, self._same_step)
        self.step_work_bytes = min(need, self.work_bytes)

    def step(self, field: Q.qed_field, params: Q.qed_params, stream: Optional[int] = None):
        Q.qed_step(self.tables.data_ptr(), self.stores, field, params, self.step_ctr.data_ptr(),
                   self.stats_buf.data_ptr(), self.work.data_ptr(), self.step_work_bytes,
                   self.stream if stream is None else stream)
