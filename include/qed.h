/*
 * qed.h -- C ABI of the MI355X (gfx950) strong-field QED step library (libqed.so).
 *
 * The library implements, on the GPU, the per-particle QED step that the extended PIC
 * scheme of Gonoskov et al., "Extended PIC schemes for physics in ultra-strong laser
 * fields: review and developments" (arXiv:1412.6426) adds to every time step:
 *   - field acquisition at the particle (analytic fields, or CIC from a Yee grid; Appendix A),
 *   - the quantum parameter chi (Sec. IV.C, Eqs. (3), (4), (6); photons Eqs. (31), (32)),
 *   - the adaptive sub-division of dt (Sec. IV.H, Eq. (29); photons Eq. (33)),
 *   - the Boris push (Appendix A),
 *   - the modified event generator for photon emission (Sec. IV.G, Eqs. (24), (25)),
 *   - the Breit-Wheeler pair generator (Sec. V.A, Eq. (30)),
 *   - the append of the new particles into structure-of-arrays stores.
 *
 * Conventions shared by every entry point
 *   - Units: time 1/w_r, length c/w_r, momentum m c, energy m c^2, fields m c w_r / e, with
 *     eps_r = hbar w_r / (m c^2).  The Sauter-Schwinger field is 1/eps_r.
 *   - Species: 0 electron (charge -1), 1 positron (+1), 2 photon (p holds hbar k / (m c)).
 *   - Every pointer named d_* or held in a qed_soa / qed_instance is DEVICE memory owned by
 *     the caller; structs passed by pointer (qed_stores, qed_field, qed_params) are HOST
 *     memory read during the call only.  The library never allocates device memory and
 *     keeps no pointer after a call returns.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call only enqueues work on
 *     it: no host synchronisation, no allocation, no memset node -- so a sequence of calls
 *     can be captured into a hipGraph and replayed.  Kernel arguments are frozen at capture;
 *     everything that changes from step to step (step index, counts) lives in device memory.
 *   - Errors: the return value reports argument validation and launch failures only.  What
 *     happens on the device (children dropped for lack of capacity, non-finite values,
 *     probabilities >= 1) never aborts; it is counted in the qed_stats record and in the
 *     instance descriptors, readable once the stream has synchronised.
 *   - Calls are reentrant; concurrent calls must not share stores, stats or work buffers.
 */
#ifndef QED_H
#define QED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QED_OK = 0,
  QED_ERR_ARG = 1,          /* invalid argument (null pointer, size, unknown enum value) */
  QED_ERR_HIP = 2,          /* a HIP runtime call or kernel launch failed */
  QED_ERR_UNSUPPORTED = 3,  /* valid request the library does not implement */
  QED_ERR_SCRATCH = 4       /* qed_step_noalloc: the step needs more workspace than its
                               fixed scratch buffer holds */
} qed_status;

typedef enum { QED_FP64 = 0, QED_MIXED = 1 } qed_precision;

enum { QED_ELECTRON = 0, QED_POSITRON = 1, QED_PHOTON = 2, QED_NSPECIES = 3 };

typedef enum {
  QED_FIELD_UNIFORM = 0,     /* E = e0*amp_i, B = b0*amp_i */
  QED_FIELD_ROTATING_E = 1,  /* E = amp*amp_i (cos phi, sin phi, 0), B = 0, phi = omega t + phase */
  QED_FIELD_CP_STANDING = 2, /* E = 2 a cos(omega x) (0, cos phi, sin phi),
                                B = 2 a sin(omega x) (0, cos phi, sin phi), a = amp*amp_i */
  QED_FIELD_YEE = 3,         /* CIC (trilinear) gather from a periodic FP32 Yee grid */
  QED_FIELD_LP_STANDING = 4  /* plane standing wave of two counter-propagating linearly
                                polarised waves: E = a (0, sin(omega x) cos phi, 0),
                                B = a (0, 0, -cos(omega x) sin phi), a = amp*amp_i,
                                phi = omega t + phase (Sec. VII avalanche) */
} qed_field_kind;

#define QED_TABLE_N 4096
#define QED_ID_DEAD 0xFFFFFFFFFFFFFFFFull   /* id of a photon removed by pair creation */
#define QED_NO_PARENT 0xFFFFFFFFFFFFFFFFull /* parent id of a seed particle */
#define QED_NSUB_MAX 16383
#define QED_NSUB_HIST 32
#define QED_SPECTRUM_BINS 130               /* 10 bins per decade of eps/mc^2 from 1e-8 */

/* status bits of qed_stats.status */
#define QED_STATUS_DROPPED 1u
#define QED_STATUS_NONFINITE 2u
#define QED_STATUS_SATURATED 4u
#define QED_STATUS_NSUB_CLAMPED 8u
#define QED_STATUS_NO_TABLES 16u  /* d_tables was not filled by qed_build_tables: nothing done */

/* ---------------------------------------------------------------------------------------
 * Rate tables (Sec. IV.F: the rates are tabulated once and interpolated during the step).
 *
 * Three functions of z are tabulated, from which the emission rate of Eq. (24) and the
 * pair rate of Eq. (30) follow once their explicit delta and chi factors are pulled out:
 *   A(z) = int_z^inf K_{5/3},  B(z) = K_{2/3}(z),  C(z) = int_z^inf K_{1/3}.
 * Nodes: z_i = 2^(-20 + 27 i / 4095), i = 0..4095; stored value e^z F(z), computed in FP64
 * by trapezoid quadrature of DLMF 10.32.9; FP32 copies for QED_MIXED.  Below z = 2^-20 the
 * small-z series is used, above z = 2^7 the functions are taken as zero.  Also holds a
 * per-octave upper bound of the pair rate used to settle most photon decisions early.
 * --------------------------------------------------------------------------------------- */

/* Layout of the tables buffer (byte offsets):
 *        0  double[4096][2]  (e^z A, e^z B) at node i
 *    65536  double[4096][2]  (e^z B, e^z C)
 *   131072  float[4096][2]   FP32 copy of the first block
 *   163840  float[4096][2]   FP32 copy of the second block
 *   196608  double[2048]     pair bound: sup over delta_e of the bracket of Eq. (30) for
 *                            chi_gamma < (1/2 + (j+1)/32) 2^(e-64), entry 16 e + j,
 *                            e = 0..127, j = 0..15
 *   212992  float[2048]      FP32 copy
 *   221184  double[8]        b0, b1, c0, c1, c2 (small-z series), 0, 0, 0
 *   221248  uint32           0x51454454 once built
 * Size in bytes of the device buffer qed_build_tables fills: */
size_t qed_table_bytes(void);

/* Fill d_tables (device, qed_table_bytes() bytes, 256-byte aligned) on `stream`.
 * QED_ERR_ARG if d_tables is NULL, misaligned or bytes is too small. */
qed_status qed_build_tables(void *d_tables, size_t bytes, void *stream);

/* ---------------------------------------------------------------------------------------
 * Particle stores.  One structure-of-arrays per species; all columns have the same length
 * (the store's total capacity) and are indexed by slot.  Instance i owns the slots
 * [base[s], base[s] + capacity[s]) of species s; its live slots are the first count[s].
 * --------------------------------------------------------------------------------------- */
typedef struct {
  double *x, *y, *z;      /* position */
  double *px, *py, *pz;   /* momentum (photons: hbar k / m c) */
  double *w;              /* statistical weight; children copy the parent's (Sec. V.A) */
  uint64_t *id;           /* particle id; seeds 0..N-1, children a hash with the top bit set */
  uint64_t *parent;       /* id of the parent, QED_NO_PARENT for seeds */
  uint32_t *birth;        /* (step+1) << 14 | sub-step of creation; 0 for seeds */
  uint32_t *n_events;     /* leptons: photons emitted so far; may be NULL for photons */
} qed_soa;

/* Per-instance descriptor (device array of n_instances, initialised by the caller).
 * count[] and dropped are updated by the library; frozen is set by it when
 * freeze_on_drop is on. */
typedef struct {
  int64_t base[3];      /* first slot of the instance's segment in each species store */
  int64_t capacity[3];  /* slots in the segment */
  int64_t count[3];     /* live slots (removed photons keep their slot, id = QED_ID_DEAD) */
  int64_t dropped;      /* children not stored for lack of capacity, cumulative */
  uint64_t seed;        /* random stream of the instance */
  double amp;           /* field amplitude multiplier of the instance (analytic fields) */
  int32_t frozen;       /* nonzero: the instance is skipped */
  int32_t reserved;
} qed_instance;

typedef struct {
  qed_soa species[3];
  int64_t slots[3];           /* length of every column of each species store */
  qed_instance *d_instances;
  int n_instances;
} qed_stores;

typedef struct {
  int kind;                 /* qed_field_kind */
  double e0[3], b0[3];      /* QED_FIELD_UNIFORM */
  double amp, omega, phase; /* QED_FIELD_ROTATING_E / QED_FIELD_CP_STANDING / _LP_STANDING */
  const float *grid[6];     /* QED_FIELD_YEE: device Ex, Ey, Ez, Bx, By, Bz, each n[2]*n[1]*n[0]
                               floats, x fastest; component c sits at origin + (i + off_c) dx,
                               off = (1/2,0,0) (0,1/2,0) (0,0,1/2) (0,1/2,1/2) (1/2,0,1/2) (1/2,1/2,0) */
  int n[3];
  double dx[3], origin[3];
} qed_field;

typedef struct {
  double dt;            /* global time step */
  double eps_r;         /* hbar w_r / m c^2 */
  double kappa;         /* sub-step safety factor: dt_q = kappa * bound of Eq. (29) / (33) */
  double t0;            /* time of step 0; step n evaluates fields at t0 + n dt */
  int adaptive;         /* 1: sub-divide dt per particle (Sec. IV.H) */
  int forced_substeps;  /* > 0: every particle uses exactly this many sub-steps */
  int emission;         /* photon emission on/off */
  int pairs;            /* pair creation on/off */
  int push_photons;     /* photons advance at c along k */
  int precision;        /* qed_precision */
  int freeze_on_drop;   /* 1: an instance that dropped children is frozen from the next step */
  int tile;             /* work split: each wavefront takes chunks of `tile` consecutive
                           particles, dealt round-robin, so that at any moment the
                           wavefronts stream through neighbouring memory; 0 = 128.  A tile of
                           at least N / wavefronts gives one contiguous chunk per wavefront */
  int block;            /* threads per workgroup (64..256, multiple of 64); 0 = 256 */
  int grid_blocks;      /* persistent workgroups per kernel (<= 4096); 0 = resident
                           workgroups per CU times the CU count */
  void *events[4];      /* optional hipEvent_t recorded on `stream` right before/after the
                           lepton kernel ([0], [1]) and the photon bound kernel ([2], [3]),
                           for timing those two kernels alone; NULL entries are skipped.
                           Owned by the caller. */
  double f_photon;      /* tunable generator factors f_g of Sec. VI for photon emission and */
  double f_pair;        /* pair creation; a value <= 1 means off.  An event still acts on its
                           parent every time it fires (the lepton recoils, the photon decays);
                           its children are created only with probability 1/f_g (a Philox draw
                           keyed by the parent id, counter (step, sub-step | p << 16, seed),
                           p = 5 for photons, 6 for pairs; first two words as the uniform u,
                           created iff u < 1/f_g) and carry f_g times the parent's weight.
                           Must be finite. */
  int same_step_generations; /* children in their birth step (Sec. IV.H: several events per
                           step).  0: children join the stores and are first advanced at
                           step n+1.  G in 1..64: a child born at sub-step k of a parent
                           advanced through T in n_sub sub-steps is advanced in the same step
                           through tau = (n_sub - k - 1) (T / n_sub), with the parent's
                           frozen E, B and its own n_sub over tau; its children likewise, up
                           to G generations (generation G + 1 waits for step n+1).  Needs
                           child arenas (at most 1024 instances, arena space in the
                           workspace, sized with same_step set in qed_work_bytes). */
  int f_every;          /* the deterministic form of f_g (Sec. VI: the generator run once
                           every f_g occasions).  Nonzero: a factor f_g > 1 must be an
                           integer F <= 2^31 - 1, and the children of a parent's event number
                           e are created iff (e + phi) mod F == 0.  e is the parent's event
                           count before the event (a lepton's n_events, or 0 at the step start
                           if its store has no n_events column; 0 for a photon, whose one
                           event is its decay); phi = (o0 F) >> 32 for the first word o0 of
                           the Philox draw keyed by the parent id with counter
                           (0, 12 << 16, seed), so the phase is the parent's for life. */
  int runs_photon;      /* the reverse mode N_g of Sec. VI for emission and for pair          */
  int runs_pair;        /* creation: the generator runs N_g times at every sub-step, run r
                           drawing with counter (step, sub-step | r << 24, seed) (run 0 is the
                           ordinary draw) and naming its children with purpose p | r << 8.
                           Emission: each run that fires makes a photon of weight w / N_g
                           from the lepton's momentum before the sub-step's events, and the
                           lepton then loses the sum of those photon momenta divided by N_g.
                           Pairs: the photon stands for N_g copies of weight w / N_g; each
                           run that fires makes a pair of that weight; after m firings in a
                           sub-step the photon keeps weight (w / N_g) (N_g - m) and goes on,
                           and it is removed when all N_g fire.  A value <= 1 means off; at
                           most 64; not with a factor f_g > 1 on the same generator
                           (QED_ERR_ARG). */
  int refill_min;       /* work queue of the lepton kernel: a wavefront takes new particles
                           into its idle lanes once at least refill_min of its 64 lanes are
                           idle (or all of them); 1 refills every idle lane at once.  0: 40 on
                           a Yee grid or a rotating field when no generator factor, reverse
                           mode or same-step processing is on, else 1.  0..64; results do not
                           depend on it (only the order of the children in the stores). */
} qed_params;

/* Per-step record written by qed_step (device memory). */
typedef struct {
  int64_t step;                 /* global step index n */
  int64_t n_start[3];           /* live slots per species at the step start (all instances) */
  int64_t advanced[3];          /* particles advanced this step (removed photons excluded) */
  int64_t emitted;              /* photon emissions */
  int64_t pairs;                /* pair creations */
  int64_t dropped;              /* children not stored (capacity) */
  int64_t saturated;            /* decisions with probability >= 1 */
  int64_t near_threshold;       /* decisions with |r2 - P| < 1e-12 */
  int64_t nsub_near_int;        /* dt/dt_q within 1e-12 (relative) of an integer, at the
                                   step start or when a sub-step is checked for refinement */
  int64_t nsub_clamped;         /* n_sub capped at QED_NSUB_MAX */
  int64_t nonfinite;            /* NaN/Inf met in chi, rates or momenta */
  int64_t substeps;             /* particle sub-steps executed */
  int64_t wave_iters;           /* lepton-kernel wavefront iterations */
  int64_t low_occupancy_iters;  /* of which fewer than half the lanes held a particle */
  int64_t early_out;            /* photon decisions settled by the pair-rate bound */
  int64_t children_advanced;    /* children advanced in their birth step (time left > 0) */
  int64_t deferred;             /* children with time left in their birth step that wait
                                   for the next step: generation G + 1, or children whose
                                   wavefront's arena share was full */
  int64_t nsub_refined;         /* lepton sub-steps taken again at half the length: Sec. IV.H
                                   wants every sub-interval to satisfy Eq. (29), and a lepton's
                                   effective field can grow within the step (the field slows
                                   it down, or it has radiated most of its energy), so a
                                   sub-step of length h is kept only if h <= dt_q in the state
                                   it ends in; otherwise the rest of the step is cut into
                                   twice as many sub-steps of half the length (at most
                                   QED_NSUB_MAX in all; a refinement beyond that is skipped
                                   and counted in nsub_clamped) */
  double photon_energy;         /* sum of w * eps over the emissions (every event, also those
                                   whose photon a generator factor did not create) */
  double max_p_emit;            /* largest emission probability evaluated */
  double max_p_pair;            /* largest pair probability among the decisions that made a
                                   pair (every probability >= 1 makes one) */
  int64_t nsub_hist[QED_NSUB_HIST];          /* leptons alive at the step start per n_sub at
                                                the step start (last bin: >= 31) */
  int64_t photon_hist[QED_SPECTRUM_BINS];    /* emissions per photon-energy bin: bin b holds
                                                floor(10 (log10(eps) + 8)) = b, eps = delta
                                                gamma in m c^2, evaluated in FP64 */
  uint32_t status;              /* QED_STATUS_* bits */
  uint32_t reserved;
} qed_stats;

/* Size of a qed_step workspace for n_instances instances, a photon store of photon_slots
 * slots and child arenas of arena_records records.  The workspace holds the per-step lists
 * of photons whose pair decision needs the exact rate (at most one entry per photon) and,
 * when arena_records > 0 and n_instances <= 1024, the child arenas: each wavefront writes
 * the photons (and pair records, a quarter of arena_records) it creates into its own share
 * of an arena, and after the particle kernels a scan and a copy kernel move them into the
 * stores, so no wavefront reserves store slots on a shared counter.  A wavefront whose
 * share is full reserves slots directly (correct, slower).  same_step nonzero adds what
 * same-step processing of children needs: per record the time left in the step, the
 * parent's fields and the children's slots (64 more bytes a photon record, 72 a pair
 * record), a second set of arenas for alternating generations, and partial statistics.
 * arena_records = 0 gives the smallest valid workspace.  Returns 0 for n_instances < 1 or
 * negative sizes. */
size_t qed_work_bytes(int n_instances, int64_t photon_slots, int64_t arena_records,
                      int same_step);

/* One global step n = *d_step of every non-frozen instance (Sec. IV.H):
 *   for each lepton and photon alive at the step start: fields at the start position
 *   (once per step), chi, n_sub, then n_sub times {push, chi, one event decision}; children
 *   are appended at the end of their instance's segment and are processed from step n+1,
 *   or, with params->same_step_generations > 0, also through the rest of step n.
 * Increments *d_step and overwrites *d_stats.  d_work: at least
 * qed_work_bytes(n_instances, stores->slots[QED_PHOTON], 0, same_step) bytes, 256-byte
 * aligned, same_step = (params->same_step_generations > 0); the largest child arena that
 * fits in work_bytes is used.  QED_ERR_UNSUPPORTED for same-step processing without child
 * arenas (more than 1024 instances, or no arena space).  The order in which children land
 * in a store follows the work distribution (instance, wavefront, creation order) and does
 * not depend on timing when the arenas are in use.
 * QED_ERR_ARG on null or inconsistent arguments.  If d_tables does not hold built tables
 * the kernels do nothing and set QED_STATUS_NO_TABLES. */
qed_status qed_step(const void *d_tables, const qed_stores *stores, const qed_field *field,
                    const qed_params *params, int64_t *d_step, qed_stats *d_stats, void *d_work,
                    size_t work_bytes, void *stream);

/* qed_step without a workspace argument, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid allocation).
 * The workspace is a fixed buffer of QED_STEP_SCRATCH_BYTES inside the library, one per
 * GPU, held from the first call on that GPU until the process ends; the call itself
 * allocates nothing.  Same arguments and results as qed_step with that buffer as d_work
 * (the largest child arena that fits in it is used).  Returns QED_ERR_SCRATCH, before any
 * launch, when qed_work_bytes(n_instances, photon slots, 0, same_step) exceeds
 * QED_STEP_SCRATCH_BYTES (about 1.4 * 10^6 photon slots for one instance without
 * same-step processing); QED_ERR_HIP if the buffer's address cannot be resolved.  The
 * buffer belongs to the device current at the call, and `stream` must belong to that
 * device.  Every call on a GPU shares its buffer (each call sets what it reads before
 * reading it), so calls that overlap on one GPU -- concurrent streams or threads -- race
 * and must be serialised by the caller.  The first call on a device resolves the buffer's
 * address and should not be made under stream capture. */
#define QED_STEP_SCRATCH_BYTES (64u << 20)
qed_status qed_step_noalloc(const void *d_tables, const qed_stores *stores,
                            const qed_field *field, const qed_params *params, int64_t *d_step,
                            qed_stats *d_stats, void *stream);

/* Result of qed_thin for one instance (device memory, one record per instance).  A store
 * at or below the trigger is not examined: all fields 0, factor 1. */
typedef struct {
  int64_t live_before;   /* live particles of the store before (removed photons excluded) */
  int64_t kept;          /* live particles after */
  double weight_before;  /* sum of w over the live particles before (= after, up to rounding) */
  double factor;         /* factor applied to the survivors' weights (1 if not thinned) */
  int32_t thinned;       /* 1 if the store was thinned */
  int32_t reserved;
} qed_thin_record;

/* Workspace size of qed_thin for n_instances instances and a species store of
 * species_slots slots (a hole list of 4 bytes per slot and per-instance partial sums). */
size_t qed_thin_work_bytes(int n_instances, int64_t species_slots);

/* Thinning by global even redistribution (Sec. VI), for one species of every instance.
 * An instance whose segment holds more than `trigger` slots (live particles and removed
 * photons) and more than `target` live particles is thinned: each live particle survives
 * with probability q = target / live, decided by the Philox draw keyed by its id with
 * counter (*d_step, 4 << 16, instance seed lo, hi), survival iff the first two words as a
 * uniform in (0, 1) are below q; the survivors' weights are multiplied by the live weight
 * over the surviving weight (sum f / (sum f - f_r)), which conserves the total weight; the
 * segment is compacted (survivors past the new count fill the holes below it; removed
 * photons go too) and its count set to the number of survivors.  Instances at or below the
 * trigger are left as they are.  d_records[n_instances] receives one record per instance.
 * Graph-capturable; no host synchronisation.  QED_ERR_ARG on bad arguments,
 * QED_ERR_UNSUPPORTED if the store has 2^32 or more slots. */
qed_status qed_thin(const qed_stores *stores, int species, int64_t trigger, int64_t target,
                    const int64_t *d_step, qed_thin_record *d_records, void *d_work,
                    size_t work_bytes, void *stream);

/* Workspace size of qed_sort_cells for n_instances instances and a species store of
 * species_slots slots: two 4-byte keys and two 4-byte indices per slot, a copy of the
 * columns (80 bytes per slot) and the per-tile digit counts.  0 for invalid arguments. */
size_t qed_sort_work_bytes(int n_instances, int64_t species_slots);

/* Reorders the live slots [0, count) of every instance's segment of one species store by
 * the grid cell that holds each particle, for position-dependent fields gathered from a
 * grid (Appendix A: the field of a particle comes from the eight nodes around it; Sec. IV.H:
 * this interpolation is usually the costliest part of the update).  Particles of one cell
 * then sit in neighbouring slots and a wavefront's gathers share cache lines; children are
 * appended in their parents' order, so sorting the lepton stores also orders the photons
 * they emit.  The key is the block of 2^s x 2^s x 2^s cells of `field` (kind QED_FIELD_YEE:
 * n, dx, origin; cell (i, j, k) = floor((x - origin) / dx) per axis, periodic) that holds
 * the particle, blocks numbered x fastest, with s the smallest shift that leaves at most
 * 2^24 - 2 blocks (s = 0 up to 16,777,214 cells; 1 for 256^3), in keys of the fewest 8-bit
 * digits that leave room for two more values: removed photons take the largest and go to
 * the end of their segment, non-finite positions the one below it.  The sort is stable
 * (particles of one block keep their order), so the result is deterministic; frozen
 * instances (which qed_step skips) are left as they are;
 * counts, contents and every particle's state are unchanged, only the slots move.  d_work:
 * qed_sort_work_bytes(n_instances, slots of the species) bytes, 256-byte aligned.
 * Asynchronous on `stream`, graph-capturable.  QED_ERR_ARG for a field that is not a Yee
 * grid, bad sizes or pointers, a missing column (n_events may be NULL); QED_ERR_UNSUPPORTED
 * for 2^32 or more slots. */
qed_status qed_sort_cells(const qed_stores *stores, int species, const qed_field *field,
                          void *d_work, size_t work_bytes, void *stream);

/* Result of qed_thin_cells for one instance (device memory, one record per instance; all
 * zero for a frozen instance). */
typedef struct {
  int64_t live_before;     /* live particles before (removed photons excluded) */
  int64_t kept;            /* live particles after */
  int64_t groups;          /* non-empty cell blocks (and the non-finite group, if any) */
  int64_t groups_thinned;  /* groups that held more than max_per_cell particles */
  double weight_before;    /* sum of w over the live particles before */
  double weight_after;     /* after (equal up to rounding: every group keeps its weight) */
} qed_thin_cells_record;

/* Workspace size of qed_thin_cells: qed_sort_work_bytes plus 36 bytes per slot of the
 * species store (per-group starts, factors, weights and survivor counts, and a list of the
 * large groups) and two 8-byte prefixes per instance.  0 for invalid arguments. */
size_t qed_thin_cells_work_bytes(int n_instances, int64_t species_slots);

/* Thinning per cell (Sec. VI's thinning with global even redistribution applied within
 * each cell block; Sec. VII's thinning that limits how many particles a cell holds), for
 * one species of every instance that is not frozen.  The store is first sorted as
 * qed_sort_cells sorts it (the same blocks of 2^s cells, with the cell of a coordinate
 * computed as floor((x - origin) / dx), periodic); a group is then a run of particles with
 * one key: one block, or the particles with a non-finite coordinate.  A group of at most
 * max_per_cell particles is kept as it is.  In a group of n > max_per_cell particles each
 * survives with probability q = max_per_cell / n, decided by the Philox draw keyed by its
 * id with counter (*d_step, 11 << 16, instance seed lo, hi), survival iff the first two
 * words as a uniform in (0, 1) are below q; if none survives, the particle with the
 * smallest draw does (the first, in store order, on a tie); the survivors' weights are
 * multiplied by the group's weight over its survivors' weight, so every group keeps its
 * weight (a group of up to 1024 particles is summed in store order; a larger one in a fixed
 * order of its own, equal to rounding).  The survivors are written back in sorted order
 * (removed photons go) and the count set to their number.  d_records[n_instances]
 * receives one record per instance.  Graph-capturable; no host synchronisation.
 * QED_ERR_ARG for a field that is not a Yee grid, max_per_cell < 1, bad sizes or pointers;
 * QED_ERR_UNSUPPORTED for 2^32 or more slots. */
qed_status qed_thin_cells(const qed_stores *stores, int species, const qed_field *field,
                          int64_t max_per_cell, const int64_t *d_step,
                          qed_thin_cells_record *d_records, void *d_work, size_t work_bytes,
                          void *stream);

/* Result of qed_thin_children for one instance (device memory, one record per instance;
 * all zero for a frozen instance). */
typedef struct {
  int64_t children;        /* children of the last step (live, with a parent) before */
  int64_t groups;          /* their parents */
  int64_t groups_thinned;  /* parents with more than max_per_parent of them */
  int64_t kept;            /* children of the last step after */
  double weight_before;    /* their weight before */
  double weight_after;     /* after (equal up to rounding where a parent's children share
                              one weight, which they do but for the pairs of one photon in
                              the reverse mode) */
} qed_thin_children_record;

/* Workspace size of qed_thin_children: 141 bytes per slot of the species store (a hash
 * table of 2 entries per slot, an entry index, a keep flag and a copy of the columns), 72
 * bytes per instance and range (ranges of about 8192 slots of the mean segment, at most
 * 2048 per instance) and 64 per instance.  0 for invalid arguments. */
size_t qed_thin_children_work_bytes(int n_instances, int64_t species_slots);

/* The cap on the children one particle generates in one iteration (Sec. VII), for one
 * species of every instance that is not frozen, after the step whose counter *d_step now
 * holds (the counter after it).  The children of that step are the live particles with
 * birth >> 14 == *d_step (birth codes (step + 1) << 14 | sub-step) and a parent other than
 * QED_NO_PARENT (Schwinger pairs have none), grouped by parent id.  A group of at most
 * max_per_parent children is kept as it is.  In a group of n > max_per_parent children
 * each survives with probability q = max_per_parent / n, decided by the Philox draw keyed by
 * its id with counter (*d_step, 13 << 16, instance seed lo, hi), survival iff the first two
 * words as a uniform in (0, 1) are below q; if none survives, those with the smallest draw
 * do; the survivors' weights are multiplied by n / K for K survivors.  Every other particle
 * (removed photons included) and the survivors keep their store order; the count becomes
 * the number left.  d_records[n_instances] receives one record per instance.
 * Graph-capturable; no host synchronisation.  QED_ERR_ARG for max_per_parent < 1, bad
 * sizes or pointers; QED_ERR_UNSUPPORTED for 2^31 or more slots or more than 65535
 * instances. */
qed_status qed_thin_children(const qed_stores *stores, int species, int64_t max_per_parent,
                             const int64_t *d_step, qed_thin_children_record *d_records,
                             void *d_work, size_t work_bytes, void *stream);

/* Counters of one qed_schwinger call (device memory; overwritten by each call). */
typedef struct {
  int64_t cells;      /* (cell, instance) pairs visited */
  int64_t pairs;      /* pairs created (dropped ones included) */
  int64_t dropped;    /* leptons beyond a store's capacity */
  int64_t saturated;  /* cells with P >= 1 (at most one pair per cell, instance and step) */
  double expected;    /* sum of min(P, 1) over the visited cells */
  int64_t reserved;
} qed_schwinger_record;

/* Non-perturbative (Schwinger) pair production of Sec. V.B for step n = *d_step, from the
 * Yee-grid field `field` (kind QED_FIELD_YEE; cells of dx[0] dx[1] dx[2] with corners at
 * origin + (i, j, k) dx).  The field of a cell is taken as constant: each E component is the
 * mean of its four staggered samples on the cell (Ex at (i + 1/2, j..j+1, k..k+1), Ey at
 * (i..i+1, j + 1/2, k..k+1), Ez at (i..i+1, j..j+1, k + 1/2), periodic); the magnetic field is
 * neglected.  With e = |E| eps_r = E / E_S, every non-frozen instance gets a pair in the
 * cell with probability P = R_S V dt, R_S = e^2 exp(-pi / e) / (4 pi^3 eps_r^4) (the reduced
 * Compton length is eps_r in units of c / omega), decided by the Philox draw keyed by the cell
 * index c = i + n0 (j + n1 k) with counter (n, 7 << 16, seed lo, seed hi) of the instance
 * (first two words as u, a pair iff u < P).  The electron and the positron start at rest at
 * origin + (i + u_x, j + u_y, k + u_z) dx, u_x..u_z = (w_m + 1/2) 2^-32 from the first three
 * words of the draw with purpose 8, with weight `weight`, no parent, birth (n + 1) << 14 and
 * ids from the key c with purposes 9 (electron) and 10 (positron); they are appended to the
 * instance's stores (beyond the capacity: dropped and counted).  Call it before qed_step of
 * the same n for the pairs to move in that step.  Writes *d_record; asynchronous on
 * `stream`.  QED_ERR_ARG for a field that is not a Yee grid, fewer than 1 cell per axis,
 * 2^31 cells or more, non-positive dt, eps_r or weight, or missing lepton columns. */
qed_status qed_schwinger(const qed_stores *stores, const qed_field *field, double dt,
                         double eps_r, double weight, const int64_t *d_step,
                         qed_schwinger_record *d_record, void *stream);

/* ---------------------------------------------------------------------------------------
 * The emission event generators of Sec. IV.G as independent trials: the setting of the
 * paper's comparison of their spectra, for one lepton state (chi, gamma) over one interval
 * whose rate prefactor is dtfac = dt e^2 m c / hbar^2 (dt alpha / eps_r in the units here).
 * P(delta) is the emission density of Eq. (24), evaluated in FP64 from the rate tables.
 * Trial j = first + i (0 <= i < n) draws (r1, r2) from Philox4x32-10 with key (key lo,
 * key hi) and counter (j lo, j hi, 0, 0), r1 from the first two words and r2 from the last
 * two (open-interval uniforms as in the step), and d_delta[i] receives the emitted photon's
 * energy fraction delta, or 0 when the trial emits nothing:
 *   QED_GEN_MODIFIED     Eq. (25): delta = r1^3, emission iff r2 < 3 r1^2 P(r1^3) (the
 *                        decision qed_step makes)
 *   QED_GEN_ALTERNATIVE  Eq. (24): delta = r1, emission iff r2 < P(r1)
 *   QED_GEN_STANDARD     Eqs. (22)-(23): emission iff r1 < W(1), delta the root of
 *                        W(delta) = r2 W(1), W(x) = int_{delta_min}^{x} P(delta) d delta
 * For the standard generator W is tabulated for the given state in d_work (at least
 * qed_generator_work_bytes(QED_GEN_STANDARD, chi, delta_min) bytes, 256-byte aligned; the
 * other generators need none and take d_work = NULL) at the ends of the rate table's
 * intervals, and each trial inverts it inside one interval.  d_delta: n doubles, device.
 * If d_tables was not filled by qed_build_tables every d_delta is NaN.  Asynchronous on
 * `stream`.  QED_ERR_ARG for NULL or misaligned (not 256-byte) tables, a NULL output with
 * n > 0, n < 0, first < 0, first + n beyond INT64_MAX, chi <= 0, gamma < 1, dtfac < 0,
 * non-finite parameters, an unknown generator, or (standard) delta_min outside (0, 1), a
 * cutoff that needs more than 2^22 table intervals, or a workspace that is missing,
 * misaligned or too small.  qed_generator_work_bytes returns 0 for the generators that
 * need no workspace and for invalid arguments. */
#define QED_GEN_MODIFIED 0
#define QED_GEN_ALTERNATIVE 1
#define QED_GEN_STANDARD 2
size_t qed_generator_work_bytes(int generator, double chi, double delta_min);
qed_status qed_generator_trials(const void *d_tables, int generator, double chi, double gamma,
                                double dtfac, double delta_min, uint64_t key, int64_t first,
                                int64_t n, double *d_delta, void *d_work, size_t work_bytes,
                                void *stream);

/* The standard generator's total emission probability tabulated over chi, as the paper
 * suggests for that generator (Sec. IV.G, Eq. (23) at x = 1): d_w[i] = W(1) gamma / dtfac,
 * which depends on chi and the cutoff only, for chi_i = chi_min (chi_max / chi_min)^(i/(n-1))
 * (chi_0 = chi_min when n = 1), i < n, integrated over the rate table's intervals in log2 z
 * like qed_generator_trials.  d_w: n doubles, device; NaN everywhere if d_tables was not
 * filled by qed_build_tables.  Asynchronous on `stream`.  QED_ERR_ARG for NULL or misaligned
 * tables, NULL d_w, n < 1 or n > 65535, chi_min <= 0, chi_max < chi_min, non-finite chi,
 * or delta_min outside (0, 1). */
qed_status qed_standard_w_table(const void *d_tables, double chi_min, double chi_max, int n,
                                double delta_min, double *d_w, void *stream);

/* Append the record *d_stats to d_log[*d_log_count] and increment *d_log_count, unless
 * *d_log_count >= log_capacity (then the record is discarded and the count still grows,
 * so the caller sees the overflow).  Graph-capturable. */
qed_status qed_append_stats(const qed_stats *d_stats, qed_stats *d_log, int64_t log_capacity,
                            int64_t *d_log_count, void *stream);

/* Diagnostics and harness helpers (not part of the step). */

/* Weighted histogram of eps = |k| (m c^2) of live photons of all instances into
 * d_hist[bins] (log10-spaced over [lo, hi); under/overflow not counted).  Accumulates. */
qed_status qed_photon_spectrum(const qed_stores *stores, double lo, double hi, int bins,
                               double *d_hist, void *stream);

/* Sample the QED_FIELD_CP_STANDING wave of amplitude amp (frequency omega, phase) at time t
 * onto a periodic Yee grid: d_grid[6] device arrays laid out as in qed_field.  Stands in
 * for a field solver in the standing-wave workload. */
qed_status qed_fill_standing_wave(float *const d_grid[6], const int n[3], const double dx[3],
                                  const double origin[3], double amp, double omega,
                                  double phase, double t, void *stream);

const char *qed_status_string(qed_status s);
int qed_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QED_H */
