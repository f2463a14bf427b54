"""Python binding of libqed (include/qed.h): argument marshalling only.

The ctypes structures mirror the C ABI field by field and the functions keep the C names
(``qed_build_tables``, ``qed_step``, ``qed_append_stats``, ...).  Device memory and
streams come from PyTorch; every step of the QED computation runs in the HIP kernels of
``lib/libqed.so``.  There is no fallback: if the library is missing, or no GPU is
present when a device call is made, the call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libqed.so")

QED_OK, QED_ERR_ARG, QED_ERR_HIP, QED_ERR_UNSUPPORTED, QED_ERR_SCRATCH = 0, 1, 2, 3, 4
QED_STEP_SCRATCH_BYTES = 64 << 20
QED_FP64, QED_MIXED = 0, 1
QED_ELECTRON, QED_POSITRON, QED_PHOTON = 0, 1, 2
QED_FIELD_UNIFORM, QED_FIELD_ROTATING_E, QED_FIELD_CP_STANDING, QED_FIELD_YEE = 0, 1, 2, 3
QED_FIELD_LP_STANDING = 4
QED_TABLE_N = 4096
QED_ID_DEAD = 0xFFFFFFFFFFFFFFFF
QED_NO_PARENT = 0xFFFFFFFFFFFFFFFF
QED_NSUB_MAX = 16383
QED_NSUB_HIST = 32
QED_SPECTRUM_BINS = 130
QED_STATUS_DROPPED, QED_STATUS_NONFINITE, QED_STATUS_SATURATED = 1, 2, 4
QED_STATUS_NSUB_CLAMPED, QED_STATUS_NO_TABLES = 8, 16

_dp = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)
_fp = C.POINTER(C.c_float)


class qed_soa(C.Structure):
    _fields_ = [("x", _dp), ("y", _dp), ("z", _dp), ("px", _dp), ("py", _dp), ("pz", _dp),
                ("w", _dp), ("id", _u64p), ("parent", _u64p), ("birth", _u32p),
                ("n_events", _u32p)]


class qed_instance(C.Structure):
    _fields_ = [("base", C.c_int64 * 3), ("capacity", C.c_int64 * 3), ("count", C.c_int64 * 3),
                ("dropped", C.c_int64), ("seed", C.c_uint64), ("amp", C.c_double),
                ("frozen", C.c_int32), ("reserved", C.c_int32)]


class qed_stores(C.Structure):
    _fields_ = [("species", qed_soa * 3), ("slots", C.c_int64 * 3), ("d_instances", C.c_void_p),
                ("n_instances", C.c_int)]


class qed_field(C.Structure):
    _fields_ = [("kind", C.c_int), ("e0", C.c_double * 3), ("b0", C.c_double * 3),
                ("amp", C.c_double), ("omega", C.c_double), ("phase", C.c_double),
                ("grid", _fp * 6), ("n", C.c_int * 3), ("dx", C.c_double * 3),
                ("origin", C.c_double * 3)]


class qed_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("eps_r", C.c_double), ("kappa", C.c_double),
                ("t0", C.c_double), ("adaptive", C.c_int), ("forced_substeps", C.c_int),
                ("emission", C.c_int), ("pairs", C.c_int), ("push_photons", C.c_int),
                ("precision", C.c_int), ("freeze_on_drop", C.c_int), ("tile", C.c_int),
                ("block", C.c_int), ("grid_blocks", C.c_int), ("events", C.c_void_p * 4),
                ("f_photon", C.c_double), ("f_pair", C.c_double),
                ("same_step_generations", C.c_int), ("f_every", C.c_int),
                ("runs_photon", C.c_int), ("runs_pair", C.c_int), ("refill_min", C.c_int)]


class qed_stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_start", C.c_int64 * 3), ("advanced", C.c_int64 * 3),
                ("emitted", C.c_int64),
                ("pairs", C.c_int64), ("dropped", C.c_int64), ("saturated", C.c_int64),
                ("near_threshold", C.c_int64), ("nsub_near_int", C.c_int64),
                ("nsub_clamped", C.c_int64), ("nonfinite", C.c_int64), ("substeps", C.c_int64),
                ("wave_iters", C.c_int64), ("low_occupancy_iters", C.c_int64),
                ("early_out", C.c_int64), ("children_advanced", C.c_int64),
                ("deferred", C.c_int64), ("nsub_refined", C.c_int64),
                ("photon_energy", C.c_double),
                ("max_p_emit", C.c_double), ("max_p_pair", C.c_double),
                ("nsub_hist", C.c_int64 * QED_NSUB_HIST),
                ("photon_hist", C.c_int64 * QED_SPECTRUM_BINS),
                ("status", C.c_uint32), ("reserved", C.c_uint32)]

    def as_dict(self) -> Dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class qed_thin_record(C.Structure):
    _fields_ = [("live_before", C.c_int64), ("kept", C.c_int64), ("weight_before", C.c_double),
                ("factor", C.c_double), ("thinned", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class qed_thin_cells_record(C.Structure):
    _fields_ = [("live_before", C.c_int64), ("kept", C.c_int64), ("groups", C.c_int64),
                ("groups_thinned", C.c_int64), ("weight_before", C.c_double),
                ("weight_after", C.c_double)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class qed_thin_children_record(C.Structure):
    _fields_ = [("children", C.c_int64), ("groups", C.c_int64), ("groups_thinned", C.c_int64),
                ("kept", C.c_int64), ("weight_before", C.c_double), ("weight_after", C.c_double)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class qed_schwinger_record(C.Structure):
    _fields_ = [("cells", C.c_int64), ("pairs", C.c_int64), ("dropped", C.c_int64),
                ("saturated", C.c_int64), ("expected", C.c_double), ("reserved", C.c_int64)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


#: every symbol include/qed.h declares
EXPORTS = ("qed_table_bytes", "qed_build_tables", "qed_work_bytes", "qed_step",
           "qed_step_noalloc",
           "qed_thin_work_bytes", "qed_thin", "qed_sort_work_bytes", "qed_sort_cells",
           "qed_thin_cells_work_bytes", "qed_thin_cells",
           "qed_thin_children_work_bytes", "qed_thin_children",
           "qed_schwinger", "qed_generator_work_bytes",
           "qed_generator_trials", "qed_standard_w_table",
           "qed_append_stats", "qed_photon_spectrum", "qed_fill_standing_wave",
           "qed_status_string", "qed_version")

_lib = None


class QedError(RuntimeError):
    pass


def lib():
    """Load libqed.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise QedError(f"{LIB_PATH} is missing: run `python -m paper_1412_6426_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.qed_table_bytes.restype = C.c_size_t
        L.qed_table_bytes.argtypes = []
        L.qed_build_tables.restype = C.c_int
        L.qed_build_tables.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p]
        L.qed_work_bytes.restype = C.c_size_t
        L.qed_work_bytes.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int]
        L.qed_step.restype = C.c_int
        L.qed_step.argtypes = [C.c_void_p, C.POINTER(qed_stores), C.POINTER(qed_field),
                               C.POINTER(qed_params), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_size_t, C.c_void_p]
        L.qed_step_noalloc.restype = C.c_int
        L.qed_step_noalloc.argtypes = [C.c_void_p, C.POINTER(qed_stores), C.POINTER(qed_field),
                                       C.POINTER(qed_params), C.c_void_p, C.c_void_p,
                                       C.c_void_p]
        L.qed_append_stats.restype = C.c_int
        L.qed_thin_work_bytes.restype = C.c_size_t
        L.qed_thin_work_bytes.argtypes = [C.c_int, C.c_int64]
        L.qed_thin.restype = C.c_int
        L.qed_thin.argtypes = [C.POINTER(qed_stores), C.c_int, C.c_int64, C.c_int64, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.qed_append_stats.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_void_p]
        L.qed_sort_work_bytes.restype = C.c_size_t
        L.qed_sort_work_bytes.argtypes = [C.c_int, C.c_int64]
        L.qed_sort_cells.restype = C.c_int
        L.qed_sort_cells.argtypes = [C.POINTER(qed_stores), C.c_int, C.POINTER(qed_field),
                                     C.c_void_p, C.c_size_t, C.c_void_p]
        L.qed_thin_cells_work_bytes.restype = C.c_size_t
        L.qed_thin_cells_work_bytes.argtypes = [C.c_int, C.c_int64]
        L.qed_thin_cells.restype = C.c_int
        L.qed_thin_cells.argtypes = [C.POINTER(qed_stores), C.c_int, C.POINTER(qed_field),
                                     C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_size_t, C.c_void_p]
        L.qed_thin_children_work_bytes.restype = C.c_size_t
        L.qed_thin_children_work_bytes.argtypes = [C.c_int, C.c_int64]
        L.qed_thin_children.restype = C.c_int
        L.qed_thin_children.argtypes = [C.POINTER(qed_stores), C.c_int, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.qed_schwinger.restype = C.c_int
        L.qed_schwinger.argtypes = [C.POINTER(qed_stores), C.POINTER(qed_field), C.c_double,
                                    C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        L.qed_generator_work_bytes.restype = C.c_size_t
        L.qed_generator_work_bytes.argtypes = [C.c_int, C.c_double, C.c_double]
        L.qed_generator_trials.restype = C.c_int
        L.qed_generator_trials.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double,
                                           C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                           C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t,
                                           C.c_void_p]
        L.qed_standard_w_table.restype = C.c_int
        L.qed_standard_w_table.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int,
                                           C.c_double, C.c_void_p, C.c_void_p]
        L.qed_photon_spectrum.restype = C.c_int
        L.qed_photon_spectrum.argtypes = [C.POINTER(qed_stores), C.c_double, C.c_double,
                                          C.c_int, C.c_void_p, C.c_void_p]
        L.qed_fill_standing_wave.restype = C.c_int
        L.qed_fill_standing_wave.argtypes = [_fp * 6, C.c_int * 3, C.c_double * 3,
                                             C.c_double * 3, C.c_double, C.c_double,
                                             C.c_double, C.c_double, C.c_void_p]
        L.qed_status_string.restype = C.c_char_p
        L.qed_status_string.argtypes = [C.c_int]
        L.qed_version.restype = C.c_int
        L.qed_version.argtypes = []
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != QED_OK:
        raise QedError(f"{what}: {lib().qed_status_string(rc).decode()} ({rc})")


# ---- the C entry points, same names -------------------------------------------------
def qed_table_bytes() -> int:
    return int(lib().qed_table_bytes())


def qed_build_tables(d_tables: int, nbytes: int, stream: int) -> None:
    _check(lib().qed_build_tables(d_tables, nbytes, stream), "qed_build_tables")


def qed_work_bytes(n_instances: int, photon_slots: int, arena_records: int = 0,
                   same_step: bool = False) -> int:
    return int(lib().qed_work_bytes(n_instances, photon_slots, arena_records,
                                    1 if same_step else 0))


def qed_step(d_tables: int, stores: qed_stores, field: qed_field, params: qed_params,
             d_step: int, d_stats: int, d_work: int, work_bytes: int, stream: int) -> None:
    _check(lib().qed_step(d_tables, C.byref(stores), C.byref(field), C.byref(params), d_step,
                          d_stats, d_work, work_bytes, stream), "qed_step")


def qed_step_noalloc(d_tables: int, stores: qed_stores, field: qed_field, params: qed_params,
                     d_step: int, d_stats: int, stream: int) -> None:
    _check(lib().qed_step_noalloc(d_tables, C.byref(stores), C.byref(field), C.byref(params),
                                  d_step, d_stats, stream), "qed_step_noalloc")


def qed_thin_work_bytes(n_instances: int, species_slots: int) -> int:
    return int(lib().qed_thin_work_bytes(n_instances, species_slots))


def qed_thin(stores: qed_stores, species: int, trigger: int, target: int, d_step: int,
             d_records: int, d_work: int, work_bytes: int, stream: int) -> None:
    _check(lib().qed_thin(C.byref(stores), species, trigger, target, d_step, d_records, d_work,
                          work_bytes, stream), "qed_thin")


def qed_sort_work_bytes(n_instances: int, species_slots: int) -> int:
    return int(lib().qed_sort_work_bytes(n_instances, species_slots))


def qed_sort_cells(stores: qed_stores, species: int, field: qed_field, d_work: int,
                   work_bytes: int, stream: int) -> None:
    _check(lib().qed_sort_cells(C.byref(stores), species, C.byref(field), d_work, work_bytes,
                                stream), "qed_sort_cells")


def qed_thin_cells_work_bytes(n_instances: int, species_slots: int) -> int:
    return int(lib().qed_thin_cells_work_bytes(n_instances, species_slots))


def qed_thin_cells(stores: qed_stores, species: int, field: qed_field, max_per_cell: int,
                   d_step: int, d_records: int, d_work: int, work_bytes: int,
                   stream: int) -> None:
    _check(lib().qed_thin_cells(C.byref(stores), species, C.byref(field), int(max_per_cell),
                                d_step, d_records, d_work, work_bytes, stream),
           "qed_thin_cells")


def qed_thin_children_work_bytes(n_instances: int, species_slots: int) -> int:
    return int(lib().qed_thin_children_work_bytes(n_instances, species_slots))


def qed_thin_children(stores: qed_stores, species: int, max_per_parent: int, d_step: int,
                      d_records: int, d_work: int, work_bytes: int, stream: int) -> None:
    _check(lib().qed_thin_children(C.byref(stores), species, int(max_per_parent), d_step,
                                   d_records, d_work, work_bytes, stream),
           "qed_thin_children")


def qed_schwinger(stores: qed_stores, field: qed_field, dt: float, eps_r: float,
                  weight: float, d_step: int, d_record: int, stream: int) -> None:
    _check(lib().qed_schwinger(C.byref(stores), C.byref(field), dt, eps_r, weight, d_step,
                               d_record, stream), "qed_schwinger")


QED_GEN_MODIFIED, QED_GEN_ALTERNATIVE, QED_GEN_STANDARD = 0, 1, 2


def qed_generator_work_bytes(generator: int, chi: float, delta_min: float) -> int:
    return int(lib().qed_generator_work_bytes(generator, chi, delta_min))


def qed_generator_trials(d_tables: int, generator: int, chi: float, gamma: float, dtfac: float,
                         delta_min: float, key: int, first: int, n: int, d_delta: int,
                         d_work: int, work_bytes: int, stream: int) -> None:
    _check(lib().qed_generator_trials(d_tables, generator, chi, gamma, dtfac, delta_min, key,
                                      first, n, d_delta, d_work, work_bytes, stream),
           "qed_generator_trials")


def qed_standard_w_table(d_tables: int, chi_min: float, chi_max: float, n: int,
                         delta_min: float, d_w: int, stream: int) -> None:
    _check(lib().qed_standard_w_table(d_tables, chi_min, chi_max, n, delta_min, d_w, stream),
           "qed_standard_w_table")


def qed_append_stats(d_stats: int, d_log: int, log_capacity: int, d_log_count: int,
                     stream: int) -> None:
    _check(lib().qed_append_stats(d_stats, d_log, log_capacity, d_log_count, stream),
           "qed_append_stats")


def qed_photon_spectrum(stores: qed_stores, lo: float, hi: float, bins: int, d_hist: int,
                        stream: int) -> None:
    _check(lib().qed_photon_spectrum(C.byref(stores), lo, hi, bins, d_hist, stream),
           "qed_photon_spectrum")


def qed_fill_standing_wave(grid_ptrs: Sequence[int], n: Sequence[int], dx: Sequence[float],
                           origin: Sequence[float], amp: float, omega: float, phase: float,
                           t: float, stream: int) -> None:
    g = (_fp * 6)(*[C.cast(C.c_void_p(p), _fp) for p in grid_ptrs])
    _check(lib().qed_fill_standing_wave(g, (C.c_int * 3)(*n), (C.c_double * 3)(*dx),
                                        (C.c_double * 3)(*origin), amp, omega, phase, t,
                                        stream), "qed_fill_standing_wave")


def qed_version() -> int:
    return int(lib().qed_version())
