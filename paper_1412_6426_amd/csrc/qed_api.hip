// qed_api.hip -- extern "C" entry points of libqed: argument validation, launch geometry
// and the host-side constants of the rate tables.  No entry point allocates device memory
// or synchronises the host.
#include <math.h>

#include <mutex>

#include "qed_internal.h"

using namespace qedk;

// Fixed workspace of qed_step_noalloc: every GPU the library runs on holds its own copy
// until the process ends.  In host code this name is a stand-in, not a device address:
// only the address resolved by scratch_on_current_device() may reach a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[QED_STEP_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kScratchDevices];  // device address of `scratch` per device, once resolved

// The address of `scratch` on the current device, resolved (with that device current) on
// the first call for the device and kept.
hipError_t scratch_on_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int g_cu_count[kMaxDevices];
// [precision][field mode][kernel: photon, lepton, extended lepton, reverse-mode lepton]
// resident 256-thread blocks per CU
int g_occ[kMaxDevices][2][3][4];

bool device_geometry(int* cus, int precision, int fmode, int kernel, int block, int* per_cu) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_cu_count[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      return false;
    g_cu_count[dev] = n;
  }
  *cus = g_cu_count[dev];
  if (fmode < 0 || fmode > 2 || kernel < 0 || kernel > 3) return false;
  if (block == 256) {
    int& o = g_occ[dev][precision == QED_MIXED ? 1 : 0][fmode][kernel];
    if (o == 0) o = step_blocks_per_cu(precision, fmode, kernel, 256);
    *per_cu = o;
  } else {
    *per_cu = step_blocks_per_cu(precision, fmode, kernel, block);
  }
  return true;
}

bool soa_ok(const qed_soa& s, bool need_events) {
  return s.x && s.y && s.z && s.px && s.py && s.pz && s.w && s.id && s.parent && s.birth &&
         (!need_events || s.n_events);
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

}  // namespace

extern "C" {

size_t qed_table_bytes(void) { return sizeof(DevTables); }

qed_status qed_build_tables(void* d_tables, size_t bytes, void* stream) {
  if (!d_tables || bytes < sizeof(DevTables) || (reinterpret_cast<uintptr_t>(d_tables) & 255u))
    return QED_ERR_ARG;
  // Small-z series of K_{2/3} and int_z^inf K_{1/3} (from K_nu = (1/2)Gamma(nu)(z/2)^-nu(...)
  // + (1/2)Gamma(-nu)(z/2)^nu(...), DLMF 10.27.4, and int_0^inf K_{1/3} = pi/sqrt 3):
  //   K_{2/3} = b0 z^-2/3 + b1 z^2/3 + (3/4) b0 z^4/3,  int K_{1/3} = c0 - c1 z^2/3 - c2 z^4/3.
  Series64 s;
  s.b0 = 0.5 * tgamma(2.0 / 3.0) * exp2(2.0 / 3.0);
  s.b1 = 0.5 * tgamma(-2.0 / 3.0) * exp2(-2.0 / 3.0);
  s.c0 = kPi / sqrt(3.0);
  s.c1 = 0.75 * tgamma(1.0 / 3.0) * exp2(1.0 / 3.0);
  s.c2 = 0.375 * tgamma(-1.0 / 3.0) * exp2(-1.0 / 3.0);
  const hipError_t e =
      launch_build_tables(static_cast<DevTables*>(d_tables), s, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

size_t qed_work_bytes(int n_instances, int64_t photon_slots, int64_t arena_records,
                      int same_step) {
  if (n_instances < 1 || photon_slots < 0 || arena_records < 0) return 0;
  return WorkLayout::make(n_instances, photon_slots, arena_records, same_step != 0).total;
}

namespace {

// Column pointers of a child arena inside the workspace, as seen by a producing kernel of
// `waves` wavefronts: with a pool, half the records are the wavefronts' equal shares and
// the rest a pool of chunks; without, all are shares.  same_step: the layout has the
// same-step columns; use_same_step: point at them (else they stay null).
ChildArena arena_at(uint8_t* w, size_t cols, size_t cnt, size_t nrec, size_t base, size_t chain,
                    long long cap, bool pair, int waves, bool same_step, bool use_same_step,
                    bool pool) {
  ChildArena A{};
  if (cap <= 0 || waves <= 0) return A;
  const size_t col8 = ((size_t)cap * 8 + 255) & ~(size_t)255;
  const size_t col4 = ((size_t)cap * 4 + 255) & ~(size_t)255;
  uint8_t* p = w + cols;
  double** dcols[8] = {&A.x, &A.y, &A.z, &A.px, &A.py, &A.pz, &A.w, &A.r1};
  for (int c = 0; c < (pair ? 8 : 7); ++c) {
    *dcols[c] = reinterpret_cast<double*>(p);
    p += col8;
  }
  A.parent = reinterpret_cast<unsigned long long*>(p);
  p += col8;
  A.sub = reinterpret_cast<unsigned int*>(p);
  p += col4;
  A.inst = reinterpret_cast<unsigned int*>(p);
  p += col4;
  if (same_step && use_same_step) {
    A.tau = reinterpret_cast<double*>(p);
    p += col8;
    A.fe = reinterpret_cast<double*>(p);
    p += 6 * col8;
    A.slot = reinterpret_cast<long long*>(p);
    p += col8;
    if (pair) A.slot2 = reinterpret_cast<long long*>(p);
  }
  A.cap = cap;
  A.cnt = reinterpret_cast<unsigned int*>(w + cnt);
  A.nrec = reinterpret_cast<unsigned int*>(w + nrec);
  A.base = reinterpret_cast<long long*>(w + base);
  A.used = reinterpret_cast<unsigned int*>(w + chain);
  A.first = reinterpret_cast<unsigned int*>(w + chain + 256);
  A.next = reinterpret_cast<unsigned int*>(w + chain + 256 +
                                           ((sizeof(unsigned int) * kMaxWaves + 255) & ~(size_t)255));
  A.waves = waves;
  const ArenaGeometry g = arena_geometry(cap, waves, pool);
  A.per_wave = g.per_wave;
  A.pool0 = g.pool0;
  A.nchunks = g.nchunks;
  return A;
}

}  // namespace

qed_status qed_step_noalloc(const void* d_tables, const qed_stores* stores,
                            const qed_field* field, const qed_params* params, int64_t* d_step,
                            qed_stats* d_stats, void* stream) {
  if (!stores || !params) return QED_ERR_ARG;
  if (stores->n_instances < 1 || stores->slots[QED_PHOTON] < 0) return QED_ERR_ARG;
  const int ss = params->same_step_generations > 0 ? 1 : 0;
  const size_t need = qed_work_bytes(stores->n_instances, stores->slots[QED_PHOTON], 0, ss);
  if (need == 0 || need > (size_t)QED_STEP_SCRATCH_BYTES) return QED_ERR_SCRATCH;
  void* w = nullptr;
  if (scratch_on_current_device(&w) != hipSuccess) return QED_ERR_HIP;
  return qed_step(d_tables, stores, field, params, d_step, d_stats, w,
                  (size_t)QED_STEP_SCRATCH_BYTES, stream);
}

qed_status qed_step(const void* d_tables, const qed_stores* stores, const qed_field* field,
                    const qed_params* params, int64_t* d_step, qed_stats* d_stats, void* d_work,
                    size_t work_bytes, void* stream) {
  if (!d_tables || !stores || !field || !params || !d_step || !d_stats || !d_work)
    return QED_ERR_ARG;
  const qed_params& P = *params;
  const int ni = stores->n_instances;
  if (ni < 1 || !stores->d_instances) return QED_ERR_ARG;
  if (stores->slots[0] < 0 || stores->slots[1] < 0 || stores->slots[2] < 0) return QED_ERR_ARG;
  const int G = P.same_step_generations;
  if (G < 0 || G > kMaxGenerations) return QED_ERR_ARG;
  const int ss = G > 0 ? 1 : 0;
  if (work_bytes < qed_work_bytes(ni, stores->slots[QED_PHOTON], 0, ss) ||
      (reinterpret_cast<uintptr_t>(d_work) & 255u))
    return QED_ERR_ARG;
  if (!soa_ok(stores->species[QED_ELECTRON], true) || !soa_ok(stores->species[QED_POSITRON], true))
    return QED_ERR_ARG;
  const bool run_photons = P.pairs || P.push_photons;
  if ((P.emission || run_photons) && !soa_ok(stores->species[QED_PHOTON], false))
    return QED_ERR_ARG;
  if (!isfinite(P.f_photon) || !isfinite(P.f_pair)) return QED_ERR_ARG;
  // the forms of Sec. VI that do not combine, and the limits of the run index and phase
  if ((P.f_photon > 1.0 && P.runs_photon > 1) || (P.f_pair > 1.0 && P.runs_pair > 1) ||
      P.runs_photon > kMaxRuns || P.runs_pair > kMaxRuns)
    return QED_ERR_ARG;
  if (P.refill_min < 0 || P.refill_min > 64) return QED_ERR_ARG;
  if (P.f_every && ((P.f_photon > 1.0 && (P.f_photon != floor(P.f_photon) ||
                                          P.f_photon > 2147483647.0)) ||
                    (P.f_pair > 1.0 && (P.f_pair != floor(P.f_pair) ||
                                        P.f_pair > 2147483647.0))))
    return QED_ERR_ARG;
  if (!finite_pos(P.dt) || !finite_pos(P.eps_r) || !finite_pos(P.kappa) || !isfinite(P.t0))
    return QED_ERR_ARG;
  if (P.precision != QED_FP64 && P.precision != QED_MIXED) return QED_ERR_ARG;
  if (P.forced_substeps < 0 || P.forced_substeps > QED_NSUB_MAX) return QED_ERR_ARG;
  if (P.tile < 0 || P.grid_blocks < 0 || P.grid_blocks > kMaxGridBlocks) return QED_ERR_ARG;
  const int block = P.block == 0 ? 256 : P.block;
  if (block < 64 || block > 256 || (block & 63)) return QED_ERR_ARG;

  StepArgs a{};
  for (int s = 0; s < 3; ++s) a.sp[s] = stores->species[s];
  a.inst = stores->d_instances;
  a.n_inst = ni;
  a.tables = static_cast<const DevTables*>(d_tables);
  a.field.kind = field->kind;
  switch (field->kind) {
    case QED_FIELD_UNIFORM:
      for (int d = 0; d < 3; ++d) {
        if (!isfinite(field->e0[d]) || !isfinite(field->b0[d])) return QED_ERR_ARG;
        a.e0[d] = field->e0[d];
        a.b0[d] = field->b0[d];
      }
      break;
    case QED_FIELD_ROTATING_E:
    case QED_FIELD_CP_STANDING:
    case QED_FIELD_LP_STANDING:
      if (!isfinite(field->amp) || !isfinite(field->omega) || !isfinite(field->phase))
        return QED_ERR_ARG;
      break;
    case QED_FIELD_YEE:
      for (int c = 0; c < 6; ++c)
        if (!field->grid[c]) return QED_ERR_ARG;
      for (int d = 0; d < 3; ++d) {
        if (field->n[d] < 2 || !finite_pos(field->dx[d]) || !isfinite(field->origin[d]))
          return QED_ERR_ARG;
        a.field.n[d] = field->n[d];
        a.field.inv_dx[d] = 1.0 / field->dx[d];
        a.field.origin[d] = field->origin[d];
      }
      // node offsets are 32-bit: fewer than 2^31 values per component
      if ((long long)field->n[0] * field->n[1] * field->n[2] > 2147483647ll) return QED_ERR_ARG;
      for (int c = 0; c < 6; ++c) a.field.grid[c] = field->grid[c];
      break;
    default:
      return QED_ERR_ARG;
  }
  a.field.amp = field->amp;
  a.field.omega = field->omega;
  a.field.phase = field->phase;
  a.field.tn = 0.0;  // filled per step on the device for the position-dependent kinds
  a.dt = P.dt;
  a.t0 = P.t0;
  a.eps_r = P.eps_r;
  a.inv_lep_scale = 1.0 / (P.kappa * 28.0 * kPi * P.eps_r);
  a.inv_pho_scale = 1.0 / (P.kappa * 260.0 * kPi * P.eps_r);
  a.dtfac_per_h = kAlpha / P.eps_r;
  a.fg_photon = P.f_photon > 1.0 ? P.f_photon : 1.0;
  a.inv_fg_photon = 1.0 / a.fg_photon;
  a.fg_pair = P.f_pair > 1.0 ? P.f_pair : 1.0;
  a.inv_fg_pair = 1.0 / a.fg_pair;
  a.every_photon = (P.f_every && P.f_photon > 1.0) ? (unsigned)P.f_photon : 0u;
  a.every_pair = (P.f_every && P.f_pair > 1.0) ? (unsigned)P.f_pair : 0u;
  a.runs_photon = P.runs_photon > 1 ? P.runs_photon : 1;
  a.runs_pair = P.runs_pair > 1 ? P.runs_pair : 1;
  a.adaptive = P.adaptive;
  a.forced = P.forced_substeps;
  a.emission = P.emission;
  a.pairs = P.pairs;
  a.push_photons = P.push_photons;
  a.freeze_on_drop = P.freeze_on_drop;
  a.tile = P.tile;
  // the largest child arena the workspace holds (sizes are monotonic in the record count)
  long long arena = 0;
  if (ni <= kArenaMaxInstances &&
      work_bytes >= qed_work_bytes(ni, stores->slots[QED_PHOTON], 1024, ss)) {
    long long lo = 1024, hi = 1024;
    // record offsets are 32-bit: at most 2^31 records per arena
    while (work_bytes >= qed_work_bytes(ni, stores->slots[QED_PHOTON], hi * 2, ss) &&
           hi < (1ll << 30))
      hi *= 2;
    long long top = hi * 2;
    while (top - lo > 1) {  // largest r in [lo, top) with work_bytes >= size(r)
      const long long mid = lo + (top - lo) / 2;
      if (work_bytes >= qed_work_bytes(ni, stores->slots[QED_PHOTON], mid, ss)) lo = mid;
      else top = mid;
    }
    arena = lo;
  }
  // same-step processing moves children through the arenas
  if (G > 0 && arena == 0) return QED_ERR_UNSUPPORTED;
  const WorkLayout L = WorkLayout::make(ni, stores->slots[QED_PHOTON], arena, ss != 0);
  uint8_t* w = static_cast<uint8_t*>(d_work);
  a.hdr = reinterpret_cast<WorkHdr*>(w);
  a.n0 = reinterpret_cast<long long*>(w + L.n0);
  a.lep_pref = reinterpret_cast<long long*>(w + L.lep_pref);
  a.pho_pref = reinterpret_cast<long long*>(w + L.pho_pref);
  a.eb = reinterpret_cast<double*>(w + L.eb);
  a.lep_part = reinterpret_cast<unsigned long long*>(w + L.lep_part);
  a.pho_part = reinterpret_cast<unsigned long long*>(w + L.pho_part);
  a.ex_part = reinterpret_cast<unsigned long long*>(w + L.ex_part);
  a.cand = reinterpret_cast<unsigned long long*>(w + L.cand);
  a.cand_cap = stores->slots[QED_PHOTON] > 0 ? stores->slots[QED_PHOTON] : 1;
  a.candw = reinterpret_cast<unsigned long long*>(w + L.candw);
  a.candn = reinterpret_cast<unsigned int*>(w + L.candn);
  a.stats = d_stats;
  a.d_step = reinterpret_cast<long long*>(d_step);
  for (int i = 0; i < 4; ++i) a.events[i] = static_cast<hipEvent_t>(P.events[i]);

  int cus = 0, lep_per_cu = 0, pho_per_cu = 0;
  const int fmode = field_mode(field->kind);
  // the lepton kernel's extended form runs with same-step processing, a photon generator
  // factor or its reverse mode (the launch makes the same choice)
  const bool lep_ext = G > 0 || P.f_photon > 1.0 || P.runs_photon > 1;
  const int lep_kernel = P.runs_photon > 1 ? 3 : lep_ext ? 2 : 1;
  if (P.refill_min > 0)
    a.refill_min = P.refill_min;
  else
    a.refill_min = !lep_ext && (field->kind == QED_FIELD_YEE ||
                                field->kind == QED_FIELD_ROTATING_E) ? kRefillMin : 1;
  if (!device_geometry(&cus, P.precision, fmode, lep_kernel, block, &lep_per_cu) ||
      !device_geometry(&cus, P.precision, fmode, 0, block, &pho_per_cu))
    return QED_ERR_HIP;
  LaunchShape lep{P.grid_blocks > 0 ? P.grid_blocks : cus * lep_per_cu, block};
  LaunchShape pho{P.grid_blocks > 0 ? P.grid_blocks : cus * pho_per_cu, block};
  if (lep.grid > kMaxGridBlocks) lep.grid = kMaxGridBlocks;
  if (pho.grid > kMaxGridBlocks) pho.grid = kMaxGridBlocks;
  a.lep_grid = lep.grid;
  a.pho_grid = run_photons ? pho.grid : 0;
  a.ex_grid = (run_photons && P.pairs) ? kExactGridBlocks : 0;
  const int lep_waves = lep.grid * (block / 64);
  const int pho_waves = pho.grid * (block / 64);
  a.pho_waves = run_photons ? pho_waves : 0;
  a.cand_per_wave = cand_list_entries(stores->slots[QED_PHOTON], pho_waves);
  if (arena > 0) {
    const bool on = G > 0;
    // the lepton kernel continues in the pool only in its extended form (same-step
    // processing, a generator factor or its reverse mode); the pair and generation
    // producers always do
    const bool lep_pool = lep_ext;
    a.pa = arena_at(w, L.ph_cols[0], L.ph_cnt[0], L.ph_nrec[0], L.ph_base[0], L.ph_chain[0],
                    L.ph_cap, false, lep_waves, L.same_step, on, lep_pool);
    if (a.ex_grid > 0)
      a.qa = arena_at(w, L.pr_cols[0], L.pr_cnt[0], L.pr_nrec[0], L.pr_base[0], L.pr_chain[0],
                      L.pr_cap, true, a.ex_grid * 4, L.same_step, on, true);
    if (on) {
      a.generations = G;
      a.gen_grid = kGenGridBlocks;
      a.gen_part = reinterpret_cast<unsigned long long*>(w + L.gen_part);
      const int gen_waves = kGenGridBlocks * 4;
      for (int s2 = 0; s2 < 2; ++s2) {
        a.gpa[s2] = arena_at(w, L.ph_cols[s2], L.ph_cnt[s2], L.ph_nrec[s2], L.ph_base[s2],
                             L.ph_chain[s2], L.ph_cap, false, gen_waves, true, true, true);
        a.gqa[s2] = arena_at(w, L.pr_cols[s2], L.pr_cnt[s2], L.pr_nrec[s2], L.pr_base[s2],
                             L.pr_chain[s2], L.pr_cap, true, gen_waves, true, true, true);
      }
    }
  }
  const hipError_t e =
      launch_step(a, P.precision, lep, pho, run_photons, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

size_t qed_sort_work_bytes(int n_instances, int64_t species_slots) {
  if (n_instances < 1 || species_slots < 0) return 0;
  return SortLayout::make(n_instances, species_slots).total;
}

size_t qed_thin_cells_work_bytes(int n_instances, int64_t species_slots) {
  if (n_instances < 1 || species_slots < 0) return 0;
  return ThinCellsLayout::make(n_instances, species_slots).total;
}

// Shared argument checks of qed_sort_cells and qed_thin_cells.
static qed_status check_cell_args(const qed_stores* stores, int species,
                                  const qed_field* field, void* d_work) {
  if (!stores || !field || !d_work || !stores->d_instances) return QED_ERR_ARG;
  if (species < 0 || species >= QED_NSPECIES || stores->n_instances < 1) return QED_ERR_ARG;
  if (field->kind != QED_FIELD_YEE) return QED_ERR_ARG;
  const long long slots = stores->slots[species];
  if (slots < 0) return QED_ERR_ARG;
  if (slots >= (1ll << 32)) return QED_ERR_UNSUPPORTED;
  for (int d = 0; d < 3; ++d)
    if (field->n[d] < 1 || !finite_pos(field->dx[d]) || !isfinite(field->origin[d]))
      return QED_ERR_ARG;
  if (!soa_ok(stores->species[species], false)) return QED_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(d_work) & 255u) return QED_ERR_ARG;
  return QED_OK;
}

qed_status qed_thin_cells(const qed_stores* stores, int species, const qed_field* field,
                          int64_t max_per_cell, const int64_t* d_step,
                          qed_thin_cells_record* d_records, void* d_work, size_t work_bytes,
                          void* stream) {
  const qed_status c = check_cell_args(stores, species, field, d_work);
  if (c != QED_OK) return c;
  if (max_per_cell < 1 || !d_step || !d_records) return QED_ERR_ARG;
  const long long slots = stores->slots[species];
  if (work_bytes < qed_thin_cells_work_bytes(stores->n_instances, slots)) return QED_ERR_ARG;
  const hipError_t e = launch_thin_cells(
      stores->species[species], species, stores->d_instances, stores->n_instances, slots,
      field->n, field->dx, field->origin, (long long)max_per_cell,
      reinterpret_cast<const long long*>(d_step), d_records, d_work,
      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

size_t qed_thin_children_work_bytes(int n_instances, int64_t species_slots) {
  if (n_instances < 1 || species_slots < 0) return 0;
  return ThinChildrenLayout::make(n_instances, species_slots).total;
}

qed_status qed_thin_children(const qed_stores* stores, int species, int64_t max_per_parent,
                             const int64_t* d_step, qed_thin_children_record* d_records,
                             void* d_work, size_t work_bytes, void* stream) {
  if (!stores || !d_work || !stores->d_instances || !d_step || !d_records) return QED_ERR_ARG;
  if (species < 0 || species >= QED_NSPECIES || stores->n_instances < 1) return QED_ERR_ARG;
  if (max_per_parent < 1) return QED_ERR_ARG;
  const long long slots = stores->slots[species];
  if (slots < 0) return QED_ERR_ARG;
  // hash-table entries are 32-bit indices of tables of twice the capacity; instances are
  // the y dimension of the grids
  if (slots >= (1ll << 31) || stores->n_instances > 65535) return QED_ERR_UNSUPPORTED;
  if (!soa_ok(stores->species[species], false)) return QED_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(d_work) & 255u) return QED_ERR_ARG;
  if (work_bytes < qed_thin_children_work_bytes(stores->n_instances, slots)) return QED_ERR_ARG;
  const hipError_t e = launch_thin_children(
      stores->species[species], species, stores->d_instances, stores->n_instances, slots,
      (long long)max_per_parent, reinterpret_cast<const long long*>(d_step), d_records, d_work,
      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

qed_status qed_sort_cells(const qed_stores* stores, int species, const qed_field* field,
                          void* d_work, size_t work_bytes, void* stream) {
  const qed_status c = check_cell_args(stores, species, field, d_work);
  if (c != QED_OK) return c;
  const long long slots = stores->slots[species];
  const qed_soa& s = stores->species[species];
  if (work_bytes < qed_sort_work_bytes(stores->n_instances, slots)) return QED_ERR_ARG;
  const hipError_t e = launch_sort_cells(s, species, stores->d_instances, stores->n_instances,
                                         slots, field->n, field->dx, field->origin, d_work,
                                         static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

qed_status qed_schwinger(const qed_stores* stores, const qed_field* field, double dt,
                         double eps_r, double weight, const int64_t* d_step,
                         qed_schwinger_record* d_record, void* stream) {
  if (!stores || !field || !d_step || !d_record || !stores->d_instances) return QED_ERR_ARG;
  if (stores->n_instances < 1 || field->kind != QED_FIELD_YEE) return QED_ERR_ARG;
  if (!finite_pos(dt) || !finite_pos(eps_r) || !finite_pos(weight)) return QED_ERR_ARG;
  for (int c = 0; c < 3; ++c)
    if (!field->grid[c]) return QED_ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (field->n[d] < 1 || !finite_pos(field->dx[d]) || !isfinite(field->origin[d]))
      return QED_ERR_ARG;
  // cell indices are 32-bit in the kernel's index arithmetic
  if ((long long)field->n[0] * field->n[1] * field->n[2] > 2147483647ll) return QED_ERR_ARG;
  if (!soa_ok(stores->species[QED_ELECTRON], false) || !soa_ok(stores->species[QED_POSITRON], false))
    return QED_ERR_ARG;
  const hipError_t e = launch_schwinger(*stores, field->grid, field->n, field->dx, field->origin,
                                        dt, eps_r, weight, reinterpret_cast<const long long*>(d_step),
                                        d_record, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

size_t qed_generator_work_bytes(int generator, double chi, double delta_min) {
  if (generator == QED_GEN_MODIFIED || generator == QED_GEN_ALTERNATIVE) return 0;
  if (generator != QED_GEN_STANDARD || !finite_pos(chi) || !(delta_min > 0.0 && delta_min < 1.0))
    return 0;
  double u0, k0;
  const long long panels = standard_panels(chi, delta_min, &u0, &k0);
  if (panels > generator_max_panels()) return 0;
  return generator_work_bytes(panels);
}

qed_status qed_generator_trials(const void* d_tables, int generator, double chi, double gamma,
                                double dtfac, double delta_min, uint64_t key, int64_t first,
                                int64_t n, double* d_delta, void* d_work, size_t work_bytes,
                                void* stream) {
  if (!d_tables || (reinterpret_cast<uintptr_t>(d_tables) & 255u)) return QED_ERR_ARG;
  if (n < 0 || first < 0 || n > INT64_MAX - first || (n > 0 && !d_delta)) return QED_ERR_ARG;
  if (!finite_pos(chi) || !(gamma >= 1.0) || !isfinite(gamma) || !(dtfac >= 0.0) ||
      !isfinite(dtfac))
    return QED_ERR_ARG;
  if (generator != QED_GEN_MODIFIED && generator != QED_GEN_ALTERNATIVE &&
      generator != QED_GEN_STANDARD)
    return QED_ERR_ARG;
  if (generator == QED_GEN_STANDARD) {
    const size_t need = qed_generator_work_bytes(generator, chi, delta_min);
    if (need == 0 || !d_work || (reinterpret_cast<uintptr_t>(d_work) & 255u) ||
        work_bytes < need)
      return QED_ERR_ARG;
  }
  const hipError_t e = launch_generator_trials(
      static_cast<const DevTables*>(d_tables), generator, chi, gamma, dtfac, delta_min, key,
      first, n, d_delta, d_work, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

qed_status qed_standard_w_table(const void* d_tables, double chi_min, double chi_max, int n,
                                double delta_min, double* d_w, void* stream) {
  if (!d_tables || (reinterpret_cast<uintptr_t>(d_tables) & 255u) || !d_w) return QED_ERR_ARG;
  if (n < 1 || n > 65535 || !finite_pos(chi_min) || !isfinite(chi_max) || chi_max < chi_min)
    return QED_ERR_ARG;
  if (!(delta_min > 0.0 && delta_min < 1.0)) return QED_ERR_ARG;
  const hipError_t e =
      launch_standard_w_table(static_cast<const DevTables*>(d_tables), chi_min, chi_max, n,
                              delta_min, d_w, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

size_t qed_thin_work_bytes(int n_instances, int64_t species_slots) {
  if (n_instances < 1 || species_slots < 0) return 0;
  return ThinLayout::make(n_instances, species_slots).total;
}

qed_status qed_thin(const qed_stores* stores, int species, int64_t trigger, int64_t target,
                    const int64_t* d_step, qed_thin_record* d_records, void* d_work,
                    size_t work_bytes, void* stream) {
  if (!stores || !d_step || !d_records || !d_work || !stores->d_instances) return QED_ERR_ARG;
  if (species < QED_ELECTRON || species > QED_PHOTON || trigger < 0 || target < 1)
    return QED_ERR_ARG;
  const int ni = stores->n_instances;
  const int64_t slots = stores->slots[species];
  if (ni < 1 || ni > 65535 || slots < 0) return QED_ERR_ARG;  // instances are grid rows
  if (slots >= (1ll << 32)) return QED_ERR_UNSUPPORTED;
  if (work_bytes < qed_thin_work_bytes(ni, slots) || (reinterpret_cast<uintptr_t>(d_work) & 255u))
    return QED_ERR_ARG;
  if (!soa_ok(stores->species[species], species != QED_PHOTON)) return QED_ERR_ARG;
  const hipError_t e = launch_thin(stores->species[species], species, stores->d_instances, ni,
                                   (long long)slots, (long long)trigger, (long long)target,
                                   reinterpret_cast<const long long*>(d_step), d_records, d_work,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

qed_status qed_append_stats(const qed_stats* d_stats, qed_stats* d_log, int64_t log_capacity,
                            int64_t* d_log_count, void* stream) {
  if (!d_stats || !d_log || !d_log_count || log_capacity < 0) return QED_ERR_ARG;
  const hipError_t e =
      launch_append_stats(d_stats, d_log, (long long)log_capacity,
                          reinterpret_cast<long long*>(d_log_count), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

qed_status qed_photon_spectrum(const qed_stores* stores, double lo, double hi, int bins,
                               double* d_hist, void* stream) {
  if (!stores || !d_hist || !stores->d_instances || stores->n_instances < 1 ||
      stores->n_instances > 65535 || bins < 1 || !finite_pos(lo) || !finite_pos(hi) || hi <= lo)
    return QED_ERR_ARG;
  if (!soa_ok(stores->species[QED_PHOTON], false)) return QED_ERR_ARG;
  const hipError_t e = launch_spectrum(stores->species[QED_PHOTON], stores->d_instances,
                                       stores->n_instances, lo, hi, bins, d_hist,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

qed_status qed_fill_standing_wave(float* const d_grid[6], const int n[3], const double dx[3],
                                  const double origin[3], double amp, double omega,
                                  double phase, double t, void* stream) {
  if (!d_grid || !n || !dx || !origin) return QED_ERR_ARG;
  for (int c = 0; c < 6; ++c)
    if (!d_grid[c]) return QED_ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || !finite_pos(dx[d]) || !isfinite(origin[d])) return QED_ERR_ARG;
  if (!isfinite(amp) || !isfinite(omega) || !isfinite(phase) || !isfinite(t)) return QED_ERR_ARG;
  const hipError_t e = launch_fill_standing(d_grid, n, dx, origin, amp, omega, phase, t,
                                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QED_OK : QED_ERR_HIP;
}

const char* qed_status_string(qed_status s) {
  switch (s) {
    case QED_OK: return "ok";
    case QED_ERR_ARG: return "invalid argument";
    case QED_ERR_HIP: return "HIP runtime or launch failure";
    case QED_ERR_UNSUPPORTED: return "unsupported";
    case QED_ERR_SCRATCH: return "the request needs more workspace than the fixed scratch holds";
  }
  return "unknown status";
}

int qed_version(void) { return 100; }

}  // extern "C"
