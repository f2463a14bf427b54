// qed_internal.h -- shared declarations between the host entry points and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qed.h"
#include "qed_device.h"

namespace qedk {

// Upper bound of workgroups per persistent kernel (the workspace holds one partial stats
// record per workgroup).
constexpr int kMaxGridBlocks = 4096;
// Upper bound of wavefronts per kernel (workgroups of at most 256 threads).
constexpr int kMaxWaves = kMaxGridBlocks * 4;
// Workgroups of the exact pair-decision kernel (a grid-stride loop over the candidates).
constexpr int kExactGridBlocks = 512;
// Child arenas are used for up to this many instances (their count matrices hold one
// word per (instance, wavefront)); above it every append reserves store slots directly.
constexpr int kArenaMaxInstances = 1024;
// Workgroups of the generation kernel (same-step processing of children).
constexpr int kGenGridBlocks = 512;  // 2 wavefronts per SIMD on 256 CUs
// Candidate entries per photon wavefront beyond its even share of the photon slots.
constexpr int kCandSlack = 64;

// Entries of each of `pho_waves` photon wavefronts' candidate lists: an even share of the
// workspace's photon_slots + kMaxWaves kCandSlack entries (pho_waves <= kMaxWaves).
inline long long cand_list_entries(long long photon_slots, int pho_waves) {
  const long long slots = photon_slots > 0 ? photon_slots : 1;
  return pho_waves > 0 ? (slots + (long long)kMaxWaves * kCandSlack) / pho_waves : 0;
}

// Per-workgroup partial stats: 64-bit words, stored field-major ([field][block]) so that
// the finalize kernel reduces each field with coalesced loads.
enum PartialField : int {
  kPfSubsteps = 0, kPfEvents, kPfSaturated, kPfNear, kPfNonfinite, kPfNearInt, kPfClamped,
  kPfDropped, kPfEarly, kPfAdv0, kPfAdv1, kPfWaveIters, kPfLowOcc,
  kPfPairs,     // pairs created by the generation kernel (its kPfEvents are photons)
  kPfChildren,  // children advanced in their birth step
  kPfDeferred,  // children with time left in the step that wait for the next step
  kPfRefined,   // lepton sub-steps taken again at half the length
  kPfEnergy,  // double bits
  kPfMaxP,    // double bits: largest probability (emission; pairs in the photon kernels)
  kPfMaxQ,    // double bits: largest pair probability of the generation kernel
  kPfNsub,    // QED_NSUB_HIST words
  kPfHist = kPfNsub + QED_NSUB_HIST,  // QED_SPECTRUM_BINS words
  kPfCount = kPfHist + QED_SPECTRUM_BINS
};

// Header of the qed_step workspace; followed by the arrays laid out by WorkLayout.
struct alignas(64) WorkHdr {
  long long lep_total;         // leptons (e- and e+, all instances) alive at the step start
  long long pho_total;         // photon slots to visit (0 when the photon kernel does not run)
  long long step;              // global step index n
  double tn;                   // field time t0 + n dt
  unsigned long long n_cand;   // photons recorded for the exact pair decision this step
  uint32_t tables_ok;
  uint32_t reserved[5];
};

// Deferred children: a wavefront writes each child it creates into its own share of
// `per_wave` records (no reservation on a shared counter) and, once that is full, into
// chunks of kArenaChunk records taken from a pool with one atomic per chunk and chained
// (`first`, `next`); it counts its records per instance.  After the step's particle kernels
// a scan turns the counts into store offsets and a copy kernel moves the records into the
// stores, in (instance, wavefront, creation) order.  Structure of arrays, `cap` records:
// the shares [0, pool0), then the pool.
// With same-step processing the records also carry the time left in the step, the parent's
// frozen fields and (written by the copy kernel) the store slots the children landed in.
struct ChildArena {
  double *x, *y, *z, *px, *py, *pz, *w;  // position; momentum (photon) or k (pair record)
  double* r1;                            // pair records: electron share of k
  unsigned long long* parent;            // id of the emitting lepton / converting photon
  unsigned int* sub;                     // sub-step of the event
  unsigned int* inst;                    // instance of the event
  double* tau;        // same-step: time left in the step after the event (else null)
  double* fe;         // same-step, space-dependent fields: Ex..Bz of the parent, [6][cap]
  long long* slot;    // same-step: store slot of the (electron) child, -1 if dropped
  long long* slot2;   // same-step, pair records: store slot of the positron
  long long cap;      // records (row length of fe)
  unsigned int* cnt;    // [n_inst][waves]: records per (instance, wavefront); offsets after the scan
  unsigned int* nrec;   // [waves]: records written by each wavefront
  long long* base;      // [n_inst][2]: store counts before the append (photon or e-, e+)
  unsigned int* first;  // [waves]: a wavefront's first pool chunk
  unsigned int* next;   // [nchunks]: the chunk after this one in its wavefront's chain
  unsigned int* used;   // pool chunks handed out (zeroed before each producing kernel)
  long long per_wave;   // share of each wavefront (records)
  long long pool0;      // first pool record (waves * per_wave)
  long long nchunks;    // pool chunks
  int waves;            // wavefronts of the producing kernel (row length of cnt); 0: arena off
};
constexpr long long kArenaChunk = 256;  // records per pool chunk (a multiple of 64)

// How an arena of `cap` records is cut for `waves` producing wavefronts: with a pool, half
// the records are the wavefronts' equal shares and the rest chunks of kArenaChunk records
// taken on demand; without, all are shares.  Records [0, pool0) are the shares, the pool
// chunks follow and end at pool0 + nchunks kArenaChunk <= cap.
struct ArenaGeometry {
  long long per_wave, pool0, nchunks;
};
inline ArenaGeometry arena_geometry(long long cap, int waves, bool pool) {
  ArenaGeometry g{};
  if (cap <= 0 || waves <= 0) return g;
  g.per_wave = (pool ? cap / 2 : cap) / waves;
  g.pool0 = g.per_wave * waves;
  g.nchunks = (cap - g.pool0) / kArenaChunk;
  return g;
}

// Upper bound of generations advanced in their birth step (qed_params.same_step_generations).
constexpr int kMaxGenerations = 64;
constexpr int kMaxRuns = 64;  // runs of the reverse mode of Sec. VI (the run sits in one byte)

// The lepton kernel's default refill threshold (qed_params.refill_min = 0).  Each refill is a
// round of dependent loads (the columns, and on a grid the 24 CIC gathers) that the
// wavefront waits for; taking them in batches of at least kRefillMin idle lanes costs some
// idle lanes in the sub-steps in between and saves most of those rounds where particles take
// few sub-steps a step.  On the 256^3 grid cascade the lepton kernel took 197 ms with a
// refill for every idle lane and 155-160 ms with thresholds of 24 to 56 (157 ms at 40); on
// the rotating-field cascade 274.8 ms per job against 270.4 at 40.  Where particles take
// hundreds of sub-steps a step (the large-step shower and avalanche, same-step children)
// idle lanes wait long and the threshold costs 4-22%, so the default is 1 there: the plain
// kernel on a Yee grid or a rotating field gets kRefillMin, every other case 1.
constexpr int kRefillMin = 40;

struct WorkLayout {
  size_t n0;        // long long [n_inst * 3]: live slots at step start (0 when frozen)
  size_t lep_pref;  // long long [2 n_inst + 1]: particle prefix over (instance, e-/e+)
  size_t pho_pref;  // long long [n_inst + 1]: particle prefix over instances
  size_t eb;        // double [n_inst * 6]: E, B of space-independent fields at t_n
  size_t lep_part;  // uint64 [kPfCount][kMaxGridBlocks]
  size_t pho_part;  // uint64 [kPfCount][kMaxGridBlocks]
  size_t ex_part;   // uint64 [kPfCount][kMaxGridBlocks]
  size_t candn;     // uint32 [kMaxWaves]: candidates per photon wavefront
  size_t candw;     // uint64 [photon slots + kMaxWaves kCandSlack]: per-wavefront lists
  size_t cand;      // uint64 [photon slots]: overflow list, (photon index << 16) | sub-step
  size_t gen_part;  // uint64 [kPfCount][kMaxGridBlocks]: the generation kernel's partials
  // child arenas (present when arena_records > 0 and n_inst <= kArenaMaxInstances); set 1
  // only with same-step processing (generations alternate between the two sets)
  size_t ph_cols[2], ph_cnt[2], ph_nrec[2], ph_base[2], ph_chain[2];  // photons from leptons
  size_t pr_cols[2], pr_cnt[2], pr_nrec[2], pr_base[2], pr_chain[2];  // pair records
  long long ph_cap, pr_cap;
  bool same_step;
  size_t total;
  static WorkLayout make(int n_inst, long long photon_slots, long long arena_records,
                         bool same_step = false) {
    WorkLayout L{};
    size_t off = (sizeof(WorkHdr) + 255) & ~(size_t)255;  // every region 256-byte aligned
    auto take = [&off](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    const size_t slots = (size_t)(photon_slots > 0 ? photon_slots : 1);
    L.n0 = take(sizeof(long long) * 3 * (size_t)n_inst);
    L.lep_pref = take(sizeof(long long) * (2 * (size_t)n_inst + 1));
    L.pho_pref = take(sizeof(long long) * ((size_t)n_inst + 1));
    L.eb = take(sizeof(double) * 6 * (size_t)n_inst);
    L.lep_part = take(sizeof(unsigned long long) * kPfCount * kMaxGridBlocks);
    L.pho_part = take(sizeof(unsigned long long) * kPfCount * kMaxGridBlocks);
    L.ex_part = take(sizeof(unsigned long long) * kPfCount * kMaxGridBlocks);
    L.candn = take(sizeof(unsigned int) * kMaxWaves);
    L.candw = take(sizeof(unsigned long long) * (slots + (size_t)kMaxWaves * kCandSlack));
    L.cand = take(sizeof(unsigned long long) * slots);
    L.same_step = same_step;
    if (arena_records > 0 && n_inst <= kArenaMaxInstances) {
      L.ph_cap = arena_records;
      L.pr_cap = arena_records / 4 > 4096 ? arena_records / 4 : 4096;
      const size_t mat = sizeof(unsigned int) * (size_t)n_inst * kMaxWaves;
      for (int s = 0; s < (same_step ? 2 : 1); ++s) {
        L.ph_cols[s] = take(ChildArenaBytes(L.ph_cap, false, same_step));
        L.ph_cnt[s] = take(mat);
        L.ph_nrec[s] = take(sizeof(unsigned int) * kMaxWaves);
        L.ph_base[s] = take(sizeof(long long) * 2 * (size_t)n_inst);
        L.ph_chain[s] = take(ChainBytes(L.ph_cap));
        L.pr_cols[s] = take(ChildArenaBytes(L.pr_cap, true, same_step));
        L.pr_cnt[s] = take(mat);
        L.pr_nrec[s] = take(sizeof(unsigned int) * kMaxWaves);
        L.pr_base[s] = take(sizeof(long long) * 2 * (size_t)n_inst);
        L.pr_chain[s] = take(ChainBytes(L.pr_cap));
      }
      if (same_step)
        L.gen_part = take(sizeof(unsigned long long) * kPfCount * kMaxGridBlocks);
    }
    L.total = off;
    return L;
  }
  // Column block of an arena: 7 (+1 for pairs) doubles, parent, sub, inst per record, and
  // with same-step processing tau, six field components and one (two for pairs) slots; each
  // column 256-byte aligned.
  // Pool bookkeeping: `used` (256 bytes), `first` per wavefront, `next` per chunk.
  static size_t ChainBytes(long long cap) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 256 + al(sizeof(unsigned int) * kMaxWaves) +
           al(sizeof(unsigned int) * ((size_t)cap / kArenaChunk + 1));
  }
  static size_t ChildArenaBytes(long long cap, bool pair, bool same_step) {
    auto col = [cap](size_t b) { return ((size_t)cap * b + 255) & ~(size_t)255; };
    size_t n = col(8) * (pair ? 8 : 7) + col(8) + col(4) * 2;
    if (same_step) n += col(8) * (1 + 6 + (pair ? 2 : 1));
    return n;
  }
};

// Thinning (qed_thin): ranges (workgroups) per instance and the workspace layout.  An
// instance's segment is cut into nb ranges of about kThinSlotsPerRange slots of the mean
// segment (slots / n_inst), at most kThinBlocks.
constexpr int kThinBlocks = 2048;  // a multiple of the 256 threads of the plan kernels
constexpr long long kThinSlotsPerRange = 8192;
struct ThinLayout {
  int nb;
  size_t plan, part_n, part_w, hole_off, surv_off, holes, total;
  static int ranges(int n_inst, long long slots) {
    const long long seg = n_inst > 0 ? (slots + n_inst - 1) / n_inst : 0;
    const long long want = (seg + kThinSlotsPerRange - 1) / kThinSlotsPerRange;
    return (int)(want < 1 ? 1 : want > kThinBlocks ? kThinBlocks : want);
  }
  static ThinLayout make(int n_inst, long long slots) {
    ThinLayout L{};
    size_t off = 0;
    auto take = [&off](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    L.nb = ranges(n_inst, slots);
    const size_t nb = (size_t)n_inst * L.nb;
    L.plan = take(64 * (size_t)n_inst);
    L.part_n = take(8 * nb);
    L.part_w = take(8 * nb);
    L.hole_off = take(8 * nb);
    L.surv_off = take(8 * nb);
    L.holes = take(4 * (size_t)(slots > 0 ? slots : 1));
    L.total = off;
    return L;
  }
};

// Cell sort (qed_sort_cells): tiles of kSortTile slots, keys of 8, 16 or 24 bits (cell
// blocks; removed photons get the largest key), and the workspace layout.
constexpr int kSortTile = 4096;
constexpr int kSortMaxPasses = 3;
struct SortGeometry {
  int shift;      // blocks of 2^shift cells per axis
  int passes;     // 8-bit digit passes: keys of 8 * passes bits
  unsigned dead;  // key of a removed photon: 2^(8 passes) - 1; non-finite positions dead - 1
  long long nb[3];
};
struct alignas(64) SortHdr {
  long long n;       // live slots of the species, all instances
  long long tiles;   // tiles of the instance-ordered tile list
  long long groups;  // qed_thin_cells: groups (runs of one key), removed photons' included
  long long kept;    // qed_thin_cells: survivors, all instances
  long long nbig;    // qed_thin_cells: groups handed to the workgroup-per-group pass
  long long reserved[3];
};
struct SortLayout {
  size_t hdr, gpref, tpref, key[2], val[2], cnt, sums, cols, total;
  long long tiles_max, cap;
  static SortLayout make(int n_inst, long long slots) {
    SortLayout L{};
    size_t off = 0;
    auto take = [&off](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    L.cap = slots > 0 ? slots : 1;
    // each instance's last tile may be partial: one more tile per instance at most
    L.tiles_max = (L.cap + kSortTile - 1) / kSortTile + n_inst;
    const size_t cap = (size_t)L.cap;
    L.hdr = take(sizeof(SortHdr));
    L.gpref = take(sizeof(long long) * ((size_t)n_inst + 1));
    L.tpref = take(sizeof(long long) * ((size_t)n_inst + 1));
    for (int k = 0; k < 2; ++k) {
      L.key[k] = take(sizeof(unsigned) * cap);
      L.val[k] = take(sizeof(unsigned) * cap);
    }
    L.cnt = take(sizeof(unsigned) * 256 * (size_t)L.tiles_max);
    L.sums = take(sizeof(unsigned) * (((size_t)L.tiles_max * 256 + 4095) / 4096));
    const size_t col8 = (cap * 8 + 255) & ~(size_t)255, col4 = (cap * 4 + 255) & ~(size_t)255;
    L.cols = take(col8 * 9 + col4 * 2);  // x..w, id, parent; birth, n_events
    L.total = off;
    return L;
  }
};

// qed_thin_cells: the sort's workspace, then per group (at most one per live slot) its first
// item, weight factor, weight before and after, and survivors, and the list of large groups;
// per instance the group and survivor prefixes.  The sort's second key and index arrays hold each item's group and its
// survivor rank within its tile, its first index array the survival flags, and the count
// array's first and second tiles_max words the per-tile group and survivor counts.
struct ThinCellsLayout {
  SortLayout sort;
  size_t gstart, gfac, gw, gwa, gkept, big, gpfx, kpref, total;
  static ThinCellsLayout make(int n_inst, long long slots) {
    ThinCellsLayout L{};
    L.sort = SortLayout::make(n_inst, slots);
    size_t off = L.sort.total;
    auto take = [&off](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    const size_t cap = (size_t)L.sort.cap;
    L.gstart = take(sizeof(unsigned) * (cap + 1));
    L.gfac = take(sizeof(double) * cap);
    L.gw = take(sizeof(double) * cap);
    L.gwa = take(sizeof(double) * cap);
    L.gkept = take(sizeof(unsigned) * cap);
    L.big = take(sizeof(unsigned) * cap);
    L.gpfx = take(sizeof(long long) * ((size_t)n_inst + 1));
    L.kpref = take(sizeof(long long) * ((size_t)n_inst + 1));
    L.total = off;
    return L;
  }
};

struct StepArgs {
  qed_soa sp[3];
  qed_instance* inst;
  int n_inst;
  const DevTables* tables;
  FieldArgs field;
  double e0[3], b0[3];
  double dt, t0, eps_r;
  double inv_lep_scale;  // 1 / (kappa 28 pi eps_r)
  double inv_pho_scale;  // 1 / (kappa 260 pi eps_r)
  double dtfac_per_h;    // alpha / eps_r
  // generator factors (Sec. VI): fg = f_g when f_g > 1, else 1 (off); inv_fg = 1 / f_g
  double fg_photon, inv_fg_photon, fg_pair, inv_fg_pair;
  // deterministic form (Sec. VI): every_* = F when the factor is taken once every F events,
  // else 0; runs_* = N_g of the reverse mode (1: off)
  unsigned every_photon, every_pair;
  int runs_photon, runs_pair;
  int refill_min;  // a lepton wavefront refills idle lanes once this many are idle (or all)
  int adaptive, forced, emission, pairs, push_photons, freeze_on_drop;
  int generations;  // children advanced in their birth step: generations (0: none)
  long long tile;  // particles per work chunk (0: one chunk per wavefront)
  WorkHdr* hdr;
  long long* n0;
  long long* lep_pref;
  long long* pho_pref;
  double* eb;
  unsigned long long* lep_part;
  unsigned long long* pho_part;
  unsigned long long* ex_part;
  unsigned long long* cand;  // overflow candidate list
  long long cand_cap;
  unsigned long long* candw;  // per-wavefront candidate lists
  unsigned int* candn;
  long long cand_per_wave;
  ChildArena pa;  // photons emitted by the lepton kernel
  ChildArena qa;  // pair records of the exact kernel
  // same-step processing: both arena sets as written by the generation kernel (gen_waves
  // producing wavefronts), and its partial stats
  ChildArena gpa[2], gqa[2];
  unsigned long long* gen_part;
  int gen_grid;
  int lep_grid, pho_grid, ex_grid;  // workgroups of the lepton, photon and exact-pair kernels
  int pho_waves;                    // wavefronts of the photon kernel
  qed_stats* stats;
  long long* d_step;
  hipEvent_t events[4];
};

struct LaunchShape {
  int grid;
  int block;
};

// Kernel launchers (qed_step.hip / qed_tables.hip).
hipError_t launch_step(const StepArgs& a, int precision, LaunchShape lep, LaunchShape pho,
                       bool run_photons, hipStream_t s);
hipError_t launch_build_tables(DevTables* t, const Series64& s, hipStream_t st);
hipError_t launch_append_stats(const qed_stats* src, qed_stats* log, long long cap,
                               long long* cnt, hipStream_t s);
hipError_t launch_spectrum(const qed_soa& ph, qed_instance* inst, int n_inst, double lo,
                           double hi, int bins, double* hist, hipStream_t s);
hipError_t launch_fill_standing(float* const g[6], const int n[3], const double dx[3],
                                const double org[3], double amp, double omega, double phase,
                                double t, hipStream_t s);
hipError_t launch_thin(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                       long long slots, long long trigger, long long target,
                       const long long* d_step, qed_thin_record* rec, void* work,
                       hipStream_t st);
hipError_t launch_schwinger(const qed_stores& st, const float* const grid[3], const int n[3],
                            const double dx[3], const double origin[3], double dt, double eps_r,
                            double weight, const long long* d_step, qed_schwinger_record* rec,
                            hipStream_t s);
hipError_t launch_sort_cells(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                             long long slots, const int n[3], const double dx[3],
                             const double origin[3], void* work, hipStream_t st);
// The key geometry of an n[0] x n[1] x n[2] grid: the smallest shift that leaves at most
// 2^24 - 2 blocks, and the fewest 8-bit passes whose keys hold every block and the two
// reserved keys.
SortGeometry sort_geometry(const int n[3]);
// The cap on the children of one parent in one step (qed_thin_children): per-instance hash
// tables of 2 x capacity entries, range partials and a column copy.
struct ThinChildrenLayout {
  int nb;
  size_t hdr, part, off, tkey, tn, tk, tk2, tmin, ent, keep, cd, cu, cb, total;
  static ThinChildrenLayout make(int n_inst, long long slots);
};
hipError_t launch_thin_children(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                                long long slots, long long max_per_parent,
                                const long long* d_step, qed_thin_children_record* rec,
                                void* work, hipStream_t st);
hipError_t launch_thin_cells(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                             long long slots, const int n[3], const double dx[3],
                             const double origin[3], long long max_per_cell,
                             const long long* d_step, qed_thin_cells_record* rec, void* work,
                             hipStream_t st);
// Emission generators as trials (qed_generators.hip).
long long standard_panels(double chi, double delta_min, double* u0, double* k0);
size_t generator_work_bytes(long long panels);
long long generator_max_panels();
hipError_t launch_standard_w_table(const DevTables* tables, double chi_min, double chi_max,
                                   int n, double delta_min, double* out, hipStream_t s);
hipError_t launch_generator_trials(const DevTables* tables, int generator, double chi,
                                   double gamma, double dtfac, double delta_min, uint64_t key,
                                   long long first, long long n, double* out, void* work,
                                   hipStream_t s);
// Persistent-grid sizing: resident workgroups per CU for the step kernels.
// Resident workgroups per CU of the step kernel that a launch uses: the photon kernel, or
// the lepton kernel in its plain or extended form (EXT), for a field mode (field_mode).
int step_blocks_per_cu(int precision, int fmode, int kind, int block);
int field_mode(int kind);

}  // namespace qedk
