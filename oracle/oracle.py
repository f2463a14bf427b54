"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module.  It loads ``oracle/liboracle.so`` (built by
``oracle/build.py``) and never touches the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QED_ORACLE_LIB: another build of qed_oracle.c to load instead (the mutation tests load
# copies with a mistake planted, to show that the pins catch it)
LIB_PATH = os.environ.get("QED_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

EXACT, TABLE = 0, 1
FIELD_UNIFORM, FIELD_ROTATING_E, FIELD_CP_STANDING, FIELD_YEE = 0, 1, 2, 3
FIELD_LP_STANDING = 4
ID_DEAD = 0xFFFFFFFFFFFFFFFF
NO_PARENT = 0xFFFFFFFFFFFFFFFF
TABLE_N = 4096
U_LO, U_HI = -20.0, 7.0
NSUB_HIST = 32
SPECTRUM_BINS = 130
ELECTRON, POSITRON, PHOTON = 0, 1, 2

_dp = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)
_fp = C.POINTER(C.c_float)


class OrTables(C.Structure):
    _fields_ = [("n", C.c_int), ("u_lo", C.c_double), ("u_hi", C.c_double), ("du", C.c_double),
                ("gA", _dp), ("gB", _dp), ("gC", _dp),
                ("s_b0", C.c_double), ("s_b1", C.c_double), ("s_c0", C.c_double),
                ("s_c1", C.c_double), ("s_c2", C.c_double)]


class OrStore(C.Structure):
    _fields_ = [("x", _dp), ("y", _dp), ("z", _dp), ("px", _dp), ("py", _dp), ("pz", _dp),
                ("w", _dp), ("id", _u64p), ("parent", _u64p), ("birth", _u32p),
                ("n_events", _u32p), ("count", C.c_int64), ("capacity", C.c_int64)]


class OrThinRecord(C.Structure):
    _fields_ = [("live_before", C.c_int64), ("kept", C.c_int64), ("weight_before", C.c_double),
                ("weight_after", C.c_double), ("factor", C.c_double)]


class OrThinCellsRecord(C.Structure):
    _fields_ = [("live_before", C.c_int64), ("kept", C.c_int64), ("groups", C.c_int64),
                ("groups_thinned", C.c_int64), ("weight_before", C.c_double),
                ("weight_after", C.c_double)]


class OrField(C.Structure):
    _fields_ = [("kind", C.c_int), ("e0", C.c_double * 3), ("b0", C.c_double * 3),
                ("amp", C.c_double), ("omega", C.c_double), ("phase", C.c_double),
                ("grid", _fp * 6), ("n", C.c_int * 3), ("dx", C.c_double * 3),
                ("origin", C.c_double * 3)]


class OrParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("eps_r", C.c_double), ("kappa", C.c_double),
                ("t0", C.c_double), ("adaptive", C.c_int), ("forced_substeps", C.c_int),
                ("emission", C.c_int), ("pairs", C.c_int), ("push_photons", C.c_int),
                ("backend", C.c_int), ("seed", C.c_uint64), ("step", C.c_int64),
                ("f_photon", C.c_double), ("f_pair", C.c_double),
                ("same_step_generations", C.c_int), ("f_every", C.c_int),
                ("runs_photon", C.c_int), ("runs_pair", C.c_int)]


class OrThinChildrenRecord(C.Structure):
    _fields_ = [("children", C.c_int64), ("groups", C.c_int64), ("groups_thinned", C.c_int64),
                ("kept", C.c_int64), ("weight_before", C.c_double),
                ("weight_after", C.c_double)]


class OrSchwingerRecord(C.Structure):
    _fields_ = [("cells", C.c_int64), ("pairs", C.c_int64), ("dropped", C.c_int64),
                ("saturated", C.c_int64), ("expected", C.c_double)]


class OrStats(C.Structure):
    _fields_ = [("n_start", C.c_int64 * 3), ("advanced", C.c_int64 * 3),
                ("emitted", C.c_int64), ("pairs", C.c_int64), ("dropped", C.c_int64),
                ("saturated", C.c_int64), ("near_threshold", C.c_int64),
                ("nsub_near_int", C.c_int64), ("nsub_clamped", C.c_int64),
                ("nonfinite", C.c_int64), ("substeps", C.c_int64), ("nsub_refined", C.c_int64),
                ("children_advanced", C.c_int64), ("deferred", C.c_int64),
                ("photon_energy", C.c_double), ("max_p_emit", C.c_double),
                ("max_p_pair", C.c_double), ("nsub_hist", C.c_int64 * NSUB_HIST),
                ("photon_hist", C.c_int64 * SPECTRUM_BINS)]
    _arrays = ("n_start", "advanced", "nsub_hist", "photon_hist")

    def as_dict(self) -> Dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name not in self._arrays}
        for name in self._arrays:
            d[name] = list(getattr(self, name))
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (local build script)
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint32)]
        L.or_uniform.argtypes = [C.c_uint32, C.c_uint32]
        L.or_uniform.restype = C.c_double
        L.or_kint_scaled.argtypes = [C.c_double, C.c_int, C.c_double]
        L.or_kint_scaled.restype = C.c_double
        for fn in ("or_A", "or_B", "or_C", "or_F1", "or_F2"):
            getattr(L, fn).argtypes = [C.c_double]
            getattr(L, fn).restype = C.c_double
        L.or_tables_build.argtypes = [C.POINTER(OrTables)]
        L.or_tables_build.restype = C.c_int
        L.or_tables_free.argtypes = [C.POINTER(OrTables)]
        L.or_eval_abc.argtypes = [C.POINTER(OrTables), C.c_int, C.c_double, _dp, _dp, _dp]
        for fn in ("or_rate_emission", "or_rate_modified", "or_rate_pair"):
            getattr(L, fn).argtypes = [C.POINTER(OrTables), C.c_int, C.c_double, C.c_double,
                                       C.c_double, C.c_double]
            getattr(L, fn).restype = C.c_double
        for fn in ("or_chi_lepton", "or_chi_photon"):
            getattr(L, fn).argtypes = [_dp, _dp, _dp, C.c_double]
            getattr(L, fn).restype = C.c_double
        L.or_boris.argtypes = [_dp, C.c_double, C.c_double, _dp, _dp]
        L.or_field_at.argtypes = [C.POINTER(OrField), _dp, C.c_double, _dp, _dp]
        L.or_substeps.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int),
                                  C.POINTER(C.c_int)]
        L.or_substeps.restype = C.c_int
        L.or_dtq_lepton.argtypes = [C.c_double] * 4
        L.or_dtq_lepton.restype = C.c_double
        L.or_dtq_photon.argtypes = [C.c_double] * 4
        L.or_dtq_photon.restype = C.c_double
        L.or_child_id.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int, C.c_int]
        L.or_child_id.restype = C.c_uint64
        L.or_step.argtypes = [C.POINTER(OrTables), C.POINTER(OrStore), C.POINTER(OrField),
                              C.POINTER(OrParams), C.POINTER(OrStats)]
        L.or_step.restype = C.c_int
        L.or_thin.argtypes = [C.POINTER(OrStore), C.c_int64, C.c_int64, C.c_uint64, C.c_int64,
                              C.POINTER(OrThinRecord)]
        L.or_thin.restype = C.c_int
        L.or_thin_cells.argtypes = [C.POINTER(OrStore), C.c_int, C.c_int * 3, C.c_double * 3,
                                    C.c_double * 3, C.c_int64, C.c_uint64, C.c_int64,
                                    C.POINTER(OrThinCellsRecord)]
        L.or_thin_cells.restype = C.c_int
        L.or_thin_children.argtypes = [C.POINTER(OrStore), C.c_int, C.c_int64, C.c_uint64,
                                       C.c_int64, C.POINTER(OrThinChildrenRecord)]
        L.or_thin_children.restype = C.c_int
        L.or_schwinger.argtypes = [C.POINTER(OrStore), C.POINTER(OrField), C.c_double,
                                   C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                   C.POINTER(OrSchwingerRecord)]
        L.or_schwinger.restype = C.c_int
        L.or_generator_trials.argtypes = [C.POINTER(OrTables), C.c_int, C.c_int, C.c_double,
                                          C.c_double, C.c_double, C.c_double, C.c_uint64,
                                          C.c_int64, C.c_int64, _dp]
        L.or_generator_trials.restype = C.c_int64
        L.or_standard_w.argtypes = [C.POINTER(OrTables), C.c_int] + [C.c_double] * 5
        L.or_standard_w.restype = C.c_double
        for fn in ("or_emission_trials", "or_pair_trials"):
            getattr(L, fn).argtypes = [C.POINTER(OrTables), C.c_int, C.c_double, C.c_double,
                                       C.c_double, C.c_uint64, C.c_int64, _dp]
            getattr(L, fn).restype = C.c_int64
        _lib = L
    return _lib


def _d3(v) -> "C.Array":
    return (C.c_double * 3)(*[float(a) for a in v])


# ---------------------------------------------------------------------------------------
# scalar helpers
# ---------------------------------------------------------------------------------------
def philox(ctr: Sequence[int], key: Sequence[int]):
    c = (C.c_uint32 * 4)(*[int(a) & 0xFFFFFFFF for a in ctr])
    k = (C.c_uint32 * 2)(*[int(a) & 0xFFFFFFFF for a in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return tuple(int(a) for a in o)


def uniform(lo: int, hi: int) -> float:
    return lib().or_uniform(lo & 0xFFFFFFFF, hi & 0xFFFFFFFF)


def kint_scaled(nu: float, over_cosh: int, z: float) -> float:
    return lib().or_kint_scaled(nu, over_cosh, z)


def A(z):
    return lib().or_A(float(z))


def B(z):
    return lib().or_B(float(z))


def Cint(z):
    return lib().or_C(float(z))


def F1(x):
    return lib().or_F1(float(x))


def F2(x):
    return lib().or_F2(float(x))


_tables: Optional[OrTables] = None


def tables() -> OrTables:
    """The oracle's own rate tables (built once per process)."""
    global _tables
    if _tables is None:
        t = OrTables()
        if lib().or_tables_build(C.byref(t)) != 0:
            raise MemoryError("oracle table build failed")
        _tables = t
    return _tables


def table_arrays():
    t = tables()
    n = t.n
    return (np.ctypeslib.as_array(t.gA, shape=(n,)).copy(),
            np.ctypeslib.as_array(t.gB, shape=(n,)).copy(),
            np.ctypeslib.as_array(t.gC, shape=(n,)).copy())


def eval_abc(z: float, backend: int = TABLE):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().or_eval_abc(C.byref(tables()), backend, float(z), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def rate_emission(delta, chi, gamma, dtfac, backend=TABLE):
    return lib().or_rate_emission(C.byref(tables()), backend, delta, chi, gamma, dtfac)


def rate_modified(r1, chi, gamma, dtfac, backend=TABLE):
    return lib().or_rate_modified(C.byref(tables()), backend, r1, chi, gamma, dtfac)


def rate_pair(delta_e, chi_g, kabs, dtfac, backend=TABLE):
    return lib().or_rate_pair(C.byref(tables()), backend, delta_e, chi_g, kabs, dtfac)


def chi_lepton(p, E, B_, eps_r):
    return lib().or_chi_lepton(_d3(p), _d3(E), _d3(B_), eps_r)


def chi_photon(k, E, B_, eps_r):
    return lib().or_chi_photon(_d3(k), _d3(E), _d3(B_), eps_r)


def boris(p, q, h, E, B_):
    pp = _d3(p)
    lib().or_boris(pp, q, h, _d3(E), _d3(B_))
    return np.array(pp[:])


def substeps(dt, dtq):
    ni, cl = C.c_int(), C.c_int()
    n = lib().or_substeps(dt, dtq, C.byref(ni), C.byref(cl))
    return n, ni.value, cl.value


def dtq_lepton(chi, gamma, eps_r, kappa=1.0):
    return lib().or_dtq_lepton(chi, gamma, eps_r, kappa)


def dtq_photon(chi_g, kabs, eps_r, kappa=1.0):
    return lib().or_dtq_photon(chi_g, kabs, eps_r, kappa)


def child_id(parent, seed, step, substep, purpose):
    return int(lib().or_child_id(parent, seed, step, substep, purpose))


def emission_trials(chi, gamma, dtfac, key, n, backend=TABLE):
    out = np.empty(int(n), dtype=np.float64)
    m = lib().or_emission_trials(C.byref(tables()), backend, chi, gamma, dtfac, key, int(n),
                                 out.ctypes.data_as(_dp))
    return out[:m]


GEN_MODIFIED, GEN_ALTERNATIVE, GEN_STANDARD = 0, 1, 2


def generator_trials(generator, chi, gamma, dtfac, key, n, first=0, delta_min=1e-3,
                     backend=TABLE):
    """Per-trial delta of one emission generator of Sec. IV.G (0: no emission)."""
    out = np.empty(int(n), dtype=np.float64)
    m = lib().or_generator_trials(C.byref(tables()), backend, int(generator), chi, gamma,
                                  dtfac, float(delta_min), key, int(first), int(n),
                                  out.ctypes.data_as(_dp))
    if m < 0:
        raise ValueError("unknown generator or delta_min outside (0, 1)")
    return out


def standard_w(x, chi, gamma, dtfac, delta_min, backend=TABLE):
    """W(x) of the standard generator, Eq. (23)."""
    return lib().or_standard_w(C.byref(tables()), backend, chi, gamma, dtfac, delta_min, x)


def pair_trials(chi_g, kabs, dtfac, key, n, backend=TABLE):
    out = np.empty(int(n), dtype=np.float64)
    m = lib().or_pair_trials(C.byref(tables()), backend, chi_g, kabs, dtfac, key, int(n),
                             out.ctypes.data_as(_dp))
    return out[:m]


# ---------------------------------------------------------------------------------------
# particle stores and the step
# ---------------------------------------------------------------------------------------
COLUMNS_F = ("x", "y", "z", "px", "py", "pz", "w")


class Store:
    """SoA particle store held in numpy arrays (one species)."""

    def __init__(self, capacity: int, with_events: bool = True):
        self.capacity = int(capacity)
        for c in COLUMNS_F:
            setattr(self, c, np.zeros(self.capacity, dtype=np.float64))
        self.id = np.zeros(self.capacity, dtype=np.uint64)
        self.parent = np.zeros(self.capacity, dtype=np.uint64)
        self.birth = np.zeros(self.capacity, dtype=np.uint32)
        self.n_events = np.zeros(self.capacity, dtype=np.uint32) if with_events else None
        self.count = 0

    def load(self, cols: Dict[str, np.ndarray]) -> "Store":
        n = len(cols["x"])
        if n > self.capacity:
            raise ValueError("more particles than capacity")
        for c in COLUMNS_F:
            getattr(self, c)[:n] = cols[c]
        self.id[:n] = cols["id"]
        self.parent[:n] = cols.get("parent", np.full(n, NO_PARENT, dtype=np.uint64))
        self.birth[:n] = cols.get("birth", np.zeros(n, dtype=np.uint32))
        if self.n_events is not None:
            self.n_events[:n] = cols.get("n_events", np.zeros(n, dtype=np.uint32))
        self.count = n
        return self

    def view(self) -> Dict[str, np.ndarray]:
        n = self.count
        d = {c: getattr(self, c)[:n].copy() for c in COLUMNS_F}
        d["id"] = self.id[:n].copy()
        d["parent"] = self.parent[:n].copy()
        d["birth"] = self.birth[:n].copy()
        if self.n_events is not None:
            d["n_events"] = self.n_events[:n].copy()
        return d

    def _cstruct(self) -> OrStore:
        s = OrStore()
        for c in COLUMNS_F:
            setattr(s, c, getattr(self, c).ctypes.data_as(_dp))
        s.id = self.id.ctypes.data_as(_u64p)
        s.parent = self.parent.ctypes.data_as(_u64p)
        s.birth = self.birth.ctypes.data_as(_u32p)
        s.n_events = (self.n_events.ctypes.data_as(_u32p) if self.n_events is not None
                      else C.cast(None, _u32p))
        s.count = self.count
        s.capacity = self.capacity
        return s


@dataclass
class Field:
    kind: int = FIELD_UNIFORM
    e0: Sequence[float] = (0.0, 0.0, 0.0)
    b0: Sequence[float] = (0.0, 0.0, 0.0)
    amp: float = 0.0
    omega: float = 1.0
    phase: float = 0.0
    grid: Optional[List[np.ndarray]] = None  # six float32 arrays [nz, ny, nx]
    dx: Sequence[float] = (1.0, 1.0, 1.0)
    origin: Sequence[float] = (0.0, 0.0, 0.0)

    def cstruct(self) -> OrField:
        f = OrField()
        f.kind = self.kind
        f.e0 = _d3(self.e0)
        f.b0 = _d3(self.b0)
        f.amp, f.omega, f.phase = self.amp, self.omega, self.phase
        if self.grid is not None:
            for i, g in enumerate(self.grid):
                if g.dtype != np.float32 or not g.flags["C_CONTIGUOUS"]:
                    raise ValueError("grid components must be C-contiguous float32")
                f.grid[i] = g.ctypes.data_as(_fp)
            nz, ny, nx = self.grid[0].shape
            f.n = (C.c_int * 3)(nx, ny, nz)
        f.dx = _d3(self.dx)
        f.origin = _d3(self.origin)
        return f


@dataclass
class Params:
    dt: float
    eps_r: float
    kappa: float = 1.0
    t0: float = 0.0
    adaptive: int = 1
    forced_substeps: int = 0
    emission: int = 1
    pairs: int = 1
    push_photons: int = 1
    backend: int = TABLE
    seed: int = 0
    step: int = 0
    f_photon: float = 1.0  # generator factors of Sec. VI (<= 1: off)
    f_pair: float = 1.0
    same_step_generations: int = 0  # children advanced in their birth step, generations
    f_every: int = 0  # deterministic form of the generator factors (every f_g-th event)
    runs_photon: int = 1  # reverse mode of Sec. VI: N_g runs per occasion (<= 1: off)
    runs_pair: int = 1

    def cstruct(self) -> OrParams:
        p = OrParams()
        for k in ("dt", "eps_r", "kappa", "t0", "adaptive", "forced_substeps", "emission",
                  "pairs", "push_photons", "backend", "seed", "step", "f_photon", "f_pair",
                  "same_step_generations", "f_every", "runs_photon", "runs_pair"):
            setattr(p, k, getattr(self, k))
        return p


def field_at(fld: Field, x, t):
    E = (C.c_double * 3)()
    Bv = (C.c_double * 3)()
    cf = fld.cstruct()
    lib().or_field_at(C.byref(cf), _d3(x), float(t), E, Bv)
    return np.array(E[:]), np.array(Bv[:])


def step(stores: Sequence[Store], fld: Field, params: Params) -> Dict:
    """One global step n = params.step over the three species stores, in place."""
    arr = (OrStore * 3)(*[s._cstruct() for s in stores])
    cf = fld.cstruct()
    cp = params.cstruct()
    st = OrStats()
    rc = lib().or_step(C.byref(tables()), arr, C.byref(cf), C.byref(cp), C.byref(st))
    if rc != 0:
        raise RuntimeError("oracle step failed")
    for i, s in enumerate(stores):
        s.count = int(arr[i].count)
    return st.as_dict()


def schwinger(stores: Sequence["Store"], fld: "Field", dt: float, eps_r: float, weight: float,
              seed: int, step: int) -> Dict:
    """Non-perturbative pairs of Sec. V.B from a Yee-grid field, one step, appended to the
    electron and positron stores in place."""
    arr = (OrStore * 3)(*[s._cstruct() for s in stores])
    cf = fld.cstruct()
    rec = OrSchwingerRecord()
    lib().or_schwinger(arr, C.byref(cf), float(dt), float(eps_r), float(weight), int(seed),
                       int(step), C.byref(rec))
    for i, s in enumerate(stores):
        s.count = int(arr[i].count)
    return {k: getattr(rec, k) for k, _ in OrSchwingerRecord._fields_}


def thin(store: "Store", trigger: int, target: int, seed: int, step: int) -> Dict:
    """Thinning by global even redistribution (Sec. VI) of one store, in place."""
    cs = store._cstruct()
    rec = OrThinRecord()
    rc = lib().or_thin(C.byref(cs), int(trigger), int(target), int(seed), int(step),
                       C.byref(rec))
    if rc < 0:
        raise RuntimeError("oracle thinning failed")
    store.count = int(cs.count)
    return {k: getattr(rec, k) for k, _ in OrThinRecord._fields_} | {"thinned": rc == 1}


def thin_children(store: "Store", is_photon: bool, max_per_parent: int, seed: int,
                  step: int) -> Dict:
    """The cap on the children one parent made in the last step (Sec. VII), in place;
    `step` is the step counter after that step."""
    cs = store._cstruct()
    rec = OrThinChildrenRecord()
    rc = lib().or_thin_children(C.byref(cs), 1 if is_photon else 0, int(max_per_parent),
                                int(seed), int(step), C.byref(rec))
    if rc < 0:
        raise RuntimeError("oracle thinning per parent failed")
    store.count = int(cs.count)
    return {k: getattr(rec, k) for k, _ in OrThinChildrenRecord._fields_} | {"thinned": rc == 1}


def thin_cells(store: "Store", is_photon: bool, n, dx, origin, max_per_cell: int, seed: int,
               step: int) -> Dict:
    """Thinning per block of grid cells (Sec. VI's redistribution within each cell block
    holding more than max_per_cell particles), in place; the store ends in block order."""
    cs = store._cstruct()
    rec = OrThinCellsRecord()
    rc = lib().or_thin_cells(C.byref(cs), 1 if is_photon else 0, (C.c_int * 3)(*n),
                             (C.c_double * 3)(*dx), (C.c_double * 3)(*origin),
                             int(max_per_cell), int(seed), int(step), C.byref(rec))
    if rc < 0:
        raise RuntimeError("oracle thinning per cell failed")
    store.count = int(cs.count)
    return {k: getattr(rec, k) for k, _ in OrThinCellsRecord._fields_} | {"thinned": rc == 1}


def run(stores: Sequence[Store], fld: Field, params: Params, n_steps: int,
        first_step: int = 0, stop_on_drop: bool = True) -> List[Dict]:
    """Advance n_steps global steps; stop after the first step that drops children."""
    out = []
    for n in range(first_step, first_step + n_steps):
        params.step = n
        s = step(stores, fld, params)
        s["step"] = n
        s["counts"] = [st.count for st in stores]
        out.append(s)
        if stop_on_drop and s["dropped"] > 0:
            break
    return out
