// qed_step.hip -- the per-step kernels of the QED step (Sec. IV.H adaptive event generator
// of Gonoskov et al., arXiv:1412.6426, with the Sec. V.A pair generator).
//
// One step is up to eight launches on the caller's stream (plus three per same-step
// generation):
//   prep     (1 + k wgs)    snapshot live counts, particle prefix sums over the
//                           (instance, species) segments, space-independent fields at t_n,
//                           zero the stats record and the arenas' count matrices;
//   leptons  (persistent)   electrons and positrons: push, chi, emission; emitted photons
//                           go to the wavefront's share of the photon arena;
//   photons  (persistent)   photons: push, chi_gamma, pair-rate bound; draws below the
//                           bound go to the wavefront's candidate list for
//   exact    (grid-stride)  the exact pair decision; pair records go to the pair arena;
//   scan     (1 wg/instance) arena counts -> store offsets, instance counts raised and
//                           clamped to the capacities;
//   copy     (1 wave/source wave) arena records -> photon, electron, positron stores;
//   reduce   (1 wave/field) per-workgroup partial stats -> the stats record (status bits
//                           set with the counters they report);
//   finalize (1 workgroup)  clamp counts, step index + 1.
// Where the copy is the step's last producer (arenas on, no same-step children), its launch
// also takes the reduce jobs and the step index, and the step is six launches.
// Children land after the step-start counts, so they are first processed at step n+1.
//
// Work distribution: the particles alive at the step start form one index space per kernel
// (segments of all instances laid end to end).  Each wavefront owns fixed chunks of it --
// no queue, no atomics -- and keeps its 64 lanes busy by refilling any lane whose particle
// has finished all of its sub-steps from the next particles of its chunk ("per-wavefront
// work queue"): one wavefront iteration advances every active lane by one sub-step, so
// lanes with n_sub = 1 and n_sub = 20 share a wavefront without idling.
//
// Appends: a wavefront writes the children it creates into its own share of an arena in
// the workspace (ballot + prefix popcount for the positions, no shared counter) and tallies
// them per instance; a scan per instance turns the tallies into store offsets and a copy
// kernel writes the children to the stores in (instance, wavefront, creation) order.  A
// device-wide counter takes one atomic per reservation and serialises every wavefront of
// the GPU on one address; the arenas avoid that.  Without arena space (or with more than
// kArenaMaxInstances instances) children are staged per wavefront in LDS and reserved in
// batches of up to 32 with one atomic per (batch, instance, species).  Statistics are
// reduced per workgroup in LDS and written as partials; the finalize kernel sums them.
#include "qed_internal.h"

namespace qedk {

constexpr int kWavesPerBlock = 4;  // launch bound 256 threads
constexpr int kStageCap = 32;      // staged photon children per wavefront
// Default work chunk: 128 particles dealt round-robin, so the wavefronts of the GPU read
// neighbouring 512-byte pieces of every column at any moment (measured faster than one
// contiguous range per wavefront, which scatters the reads over the whole store).
constexpr long long kDefaultTile = 128;

// ------------------------------------------------------------------------------------
// prep / finalize
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) prep_kernel(StepArgs a, int run_photons) {
  __shared__ int s_ok;
  if (blockIdx.x > 0) {
    // workgroups 1.. clear the per-(instance, wavefront) child counts of the arenas and
    // their pool counters
    const long long n1 = a.pa.waves > 0 ? (long long)a.n_inst * a.pa.waves : 0;
    const long long n2 = a.qa.waves > 0 ? (long long)a.n_inst * a.qa.waves : 0;
    const long long stride = (long long)(gridDim.x - 1) * blockDim.x;
    for (long long i = (long long)(blockIdx.x - 1) * blockDim.x + threadIdx.x; i < n1 + n2;
         i += stride) {
      if (i < n1) a.pa.cnt[i] = 0u;
      else a.qa.cnt[i - n1] = 0u;
    }
    if (blockIdx.x == 1 && threadIdx.x == 0) {
      if (a.pa.waves > 0) *a.pa.used = 0u;
      if (a.qa.waves > 0) *a.qa.used = 0u;
    }
    return;
  }
  WorkHdr* hdr = a.hdr;
  const long long n = *a.d_step;
  const double tn = a.t0 + (double)n * a.dt;
  if (threadIdx.x == 0) s_ok = (a.tables->magic == kTableMagic) ? 1 : 0;
  __syncthreads();
  const int ok = s_ok;
  for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) {
    qed_instance& I = a.inst[i];
    if (a.freeze_on_drop && I.dropped > 0) I.frozen = 1;
    for (int s = 0; s < 3; ++s) {
      long long c = I.count[s];
      if (c > I.capacity[s]) c = I.capacity[s];
      if (c < 0) c = 0;
      I.count[s] = c;
      a.n0[i * 3 + s] = (I.frozen || !ok) ? 0 : c;
    }
    double* eb = a.eb + 6 * i;
    const double amp = I.amp;
    if (a.field.kind == QED_FIELD_UNIFORM) {
      for (int d = 0; d < 3; ++d) {
        eb[d] = a.e0[d] * amp;
        eb[3 + d] = a.b0[d] * amp;
      }
    } else if (a.field.kind == QED_FIELD_ROTATING_E) {
      double sph, cph;
      sincos(a.field.omega * tn + a.field.phase, &sph, &cph);
      const double e = a.field.amp * amp;
      eb[0] = e * cph;
      eb[1] = e * sph;
      eb[2] = eb[3] = eb[4] = eb[5] = 0.0;
    }
  }
  unsigned long long* sw = reinterpret_cast<unsigned long long*>(a.stats);
  for (int w = threadIdx.x; w < (int)(sizeof(qed_stats) / 8); w += blockDim.x) sw[w] = 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long lp = 0, pp = 0, ns[3] = {0, 0, 0};
    a.lep_pref[0] = 0;
    a.pho_pref[0] = 0;
    for (int i = 0; i < a.n_inst; ++i) {
      for (int s = 0; s < 2; ++s) {
        const long long c = a.n0[i * 3 + s];
        lp += c;
        a.lep_pref[2 * i + s + 1] = lp;
        ns[s] += c;
      }
      const long long c = a.n0[i * 3 + 2];
      if (run_photons) pp += c;
      a.pho_pref[i + 1] = pp;
      ns[2] += c;
    }
    hdr->lep_total = lp;
    hdr->pho_total = pp;
    hdr->n_cand = 0ull;
    hdr->step = n;
    hdr->tn = tn;
    hdr->tables_ok = (uint32_t)ok;
    a.stats->step = n;
    for (int s = 0; s < 3; ++s) a.stats->n_start[s] = ns[s];
    if (!ok) a.stats->status = QED_STATUS_NO_TABLES;
  }
}

__device__ __forceinline__ void stats_add(int64_t* p, unsigned long long v) {
  if (v) atomicAdd(reinterpret_cast<unsigned long long*>(p), v);
}

// Partial-stats reduction: one wavefront per (partial set, field).  The lepton and
// generation sets have all kPfCount fields; the photon and exact-pair sets only the
// counters below kPfNsub (their histogram fields stay zero).  Sums go into the zeroed stats
// record with atomics.
constexpr int kReduceJobs = 2 * kPfCount + 2 * kPfNsub;
constexpr int kReduceBlocks = (kReduceJobs + 3) / 4;  // workgroups of 4 wavefronts

__device__ __forceinline__ void reduce_job(const StepArgs& a, int job, int lane) {
  if (job >= kReduceJobs) return;
  int kind, f;  // kind 0 leptons, 1 photons, 2 exact pairs, 3 generations
  if (job < kPfCount) {
    kind = 0;
    f = job;
  } else if (job < kPfCount + 2 * kPfNsub) {
    kind = 1 + (job - kPfCount) / kPfNsub;
    f = (job - kPfCount) % kPfNsub;
  } else {
    kind = 3;
    f = job - kPfCount - 2 * kPfNsub;
  }
  const bool pho = kind == 1 || kind == 2;
  const int G = kind == 0 ? a.lep_grid
                          : (kind == 1 ? a.pho_grid : (kind == 2 ? a.ex_grid : a.gen_grid));
  if (G <= 0) return;
  const unsigned long long* part =
      kind == 0 ? a.lep_part : (kind == 1 ? a.pho_part : (kind == 2 ? a.ex_part : a.gen_part));
  const unsigned long long* col = part + (size_t)f * kMaxGridBlocks;
  qed_stats* st = a.stats;
  if (f == kPfEnergy || f == kPfMaxP || f == kPfMaxQ) {
    double v = 0.0;
    for (int b = lane; b < G; b += 64) {
      const double x = __longlong_as_double((long long)col[b]);
      v = (f == kPfEnergy) ? v + x : fmax(v, x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(v, o, 64);
      v = (f == kPfEnergy) ? v + y : fmax(v, y);
    }
    if (lane == 0 && v != 0.0) {
      if (f == kPfEnergy) {
        if (!pho) atomicAdd(&st->photon_energy, v);
      } else {
        atomic_max_nonneg((pho || f == kPfMaxQ) ? &st->max_p_pair : &st->max_p_emit, v);
      }
    }
    return;
  }
  unsigned long long v = 0ull;
#pragma unroll 4
  for (int b = lane; b < G; b += 64) v += col[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane != 0 || v == 0ull) return;
  switch (f) {
    case kPfSubsteps: stats_add(&st->substeps, v); break;
    case kPfEvents: stats_add(pho ? &st->pairs : &st->emitted, v); break;
    case kPfSaturated:
      stats_add(&st->saturated, v);
      atomicOr(&st->status, QED_STATUS_SATURATED);
      break;
    case kPfNear: stats_add(&st->near_threshold, v); break;
    case kPfNonfinite:
      stats_add(&st->nonfinite, v);
      atomicOr(&st->status, QED_STATUS_NONFINITE);
      break;
    case kPfNearInt: stats_add(&st->nsub_near_int, v); break;
    case kPfClamped:
      stats_add(&st->nsub_clamped, v);
      atomicOr(&st->status, QED_STATUS_NSUB_CLAMPED);
      break;
    case kPfDropped:
      stats_add(&st->dropped, v);
      atomicOr(&st->status, QED_STATUS_DROPPED);
      break;
    case kPfEarly: stats_add(&st->early_out, v); break;
    case kPfAdv0: stats_add(&st->advanced[pho ? QED_PHOTON : QED_ELECTRON], v); break;
    case kPfAdv1: stats_add(&st->advanced[QED_POSITRON], v); break;
    case kPfWaveIters: stats_add(&st->wave_iters, v); break;
    case kPfLowOcc: stats_add(&st->low_occupancy_iters, v); break;
    case kPfPairs: stats_add(&st->pairs, v); break;
    case kPfChildren: stats_add(&st->children_advanced, v); break;
    case kPfDeferred: stats_add(&st->deferred, v); break;
    case kPfRefined: stats_add(&st->nsub_refined, v); break;
    default:
      if (f >= kPfNsub && f < kPfNsub + QED_NSUB_HIST)
        stats_add(&st->nsub_hist[f - kPfNsub], v);
      else if (f >= kPfHist)
        stats_add(&st->photon_hist[f - kPfHist], v);
  }
}

__global__ void __launch_bounds__(256) reduce_kernel(StepArgs a) {
  const int job = (int)blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
  reduce_job(a, job, (int)(threadIdx.x & 63u));
}

// The end of a step whose last launch is not the arena copy: counts clamped to the
// capacities, step + 1.  (The status bits are set where their counters are raised.)
__global__ void __launch_bounds__(256) finalize_kernel(StepArgs a) {
  for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) {
    qed_instance& I = a.inst[i];
    for (int s = 0; s < 3; ++s)
      if (I.count[s] > I.capacity[s]) I.count[s] = I.capacity[s];
  }
  if (threadIdx.x == 0) *a.d_step = a.hdr->step + 1;
}

// ------------------------------------------------------------------------------------
// shared pieces of the persistent kernels
// ------------------------------------------------------------------------------------
// Field modes the persistent kernels are specialised for.
enum FieldMode : int {
  kFieldEB = 0,     // space-independent E and B, evaluated once per instance (uniform field)
  kFieldE = 1,      // space-independent E, B = 0 (rotating electric field)
  kFieldLocal = 2   // evaluated at each particle (CP standing wave, Yee-grid CIC)
};

// Per-lane accumulators (few, to keep registers for the hot path); wavefront-uniform
// counts (sub-steps, events, particles advanced) are kept in scalar registers, and rare
// events (saturation, non-finite values, near-threshold decisions, clamps, drops) go
// straight into the workgroup's LDS record.
struct BlockStats;
__device__ __forceinline__ void block_count(BlockStats& bs, int field);

struct LaneCounters {
  BlockStats* bs = nullptr;
  int early = 0, subs = 0;
  double energy = 0.0, maxp = 0.0;

  // One decision r2 < P.  `fold`: P counts for the largest probability of the step (every
  // emission decision; only the pair decisions that make a pair, which include every P >= 1).
  __device__ __forceinline__ void note(double P, double r2, bool fold = true) {
    if (!isfinite(P)) {
      block_count(*bs, kPfNonfinite);
      return;
    }
    if (fold) maxp = fmax(maxp, P);
    if (P >= 1.0) block_count(*bs, kPfSaturated);
    if (fabs(r2 - P) < kNearThreshold) block_count(*bs, kPfNear);
  }
};

// Wavefront-uniform counts.
struct WaveCounters {
  long long substeps = 0, events = 0, adv0 = 0, adv1 = 0, wave_iters = 0, low_occ = 0;
  long long pairs = 0, children = 0, deferred = 0;  // same-step processing
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Workgroup-level partial stats in LDS.
struct BlockStats {
  unsigned long long w[kPfCount];
  double energy, maxp, maxq;  // maxq: pair decisions of a kernel that also has emissions
};

__device__ __forceinline__ void block_count(BlockStats& bs, int field) {
  atomicAdd(&bs.w[field], 1ull);
}

// Sub-step refinement (Sec. IV.H asks every sub-interval to satisfy Eq. (29)): a sub-step of
// length h that ends in the state (chi, gamma^2 = 1 + p2) is taken again at half the length
// if h > dt_q there, i.e. if hs3 chi^2 > gamma^2 with hs3 = (h / (kappa 28 pi eps_r))^3 --
// unless that would make more than QED_NSUB_MAX sub-steps (then it is kept and counted as
// clamped).  h / dt_q within 1e-12 of 1 is counted with the near-integer sub-step ratios.
__device__ __forceinline__ bool refine_substep(double hs3, double chi, double p2, double g,
                                               double h, double inv_lep_scale, int k, int left,
                                               BlockStats& bs) {
  const double lhs = hs3 * (chi * chi), rhs = 1.0 + p2;
  if (fabs(lhs - rhs) <= 4e-12 * rhs &&
      fabs(substep_ratio_lepton(h, chi, g, inv_lep_scale) - 1.0) <= 1e-12)
    block_count(bs, kPfNearInt);
  if (!(lhs > rhs)) return false;
  if (k + 2 * left > QED_NSUB_MAX) {
    block_count(bs, kPfClamped);
    return false;
  }
  block_count(bs, kPfRefined);
  return true;
}

__device__ __forceinline__ void block_stats_init(BlockStats& bs) {
  for (int i = threadIdx.x; i < kPfCount; i += blockDim.x) bs.w[i] = 0ull;
  if (threadIdx.x == 0) {
    bs.energy = 0.0;
    bs.maxp = 0.0;
    bs.maxq = 0.0;
  }
}

// Wave totals of the counters into the workgroup's LDS record; `pc` holds the pair decisions
// of a kernel that also makes emission decisions (their largest probability is kept apart).
__device__ void wave_to_block(BlockStats& bs, const LaneCounters& c, const WaveCounters& wc,
                              const LaneCounters* pc = nullptr) {
  const long long early = wave_sum((long long)c.early);
  const long long subs = wave_sum((long long)c.subs);
  const double en = wave_sum(c.energy);
  const double mp = wave_max(c.maxp);
  const double mq = pc ? wave_max(pc->maxp) : 0.0;
  if (lane_id() == 0) {
    const long long vals[10] = {wc.substeps + subs, wc.events, wc.adv0, wc.adv1,
                                wc.wave_iters, wc.low_occ, early, wc.pairs, wc.children,
                                wc.deferred};
    const int fields[10] = {kPfSubsteps, kPfEvents, kPfAdv0, kPfAdv1, kPfWaveIters, kPfLowOcc,
                            kPfEarly, kPfPairs, kPfChildren, kPfDeferred};
    for (int i = 0; i < 10; ++i)
      if (vals[i]) atomicAdd(&bs.w[fields[i]], (unsigned long long)vals[i]);
    if (en != 0.0) atomicAdd(&bs.energy, en);
    if (mp > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(&bs.maxp),
                (unsigned long long)__double_as_longlong(mp));
    if (mq > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(&bs.maxq),
                (unsigned long long)__double_as_longlong(mq));
  }
}

// After a __syncthreads: store the workgroup's record as column blockIdx.x of `part`.
__device__ __forceinline__ void block_stats_store(const BlockStats& bs, unsigned long long* part) {
  for (int i = threadIdx.x; i < kPfCount; i += blockDim.x) {
    unsigned long long v = bs.w[i];
    if (i == kPfEnergy) v = (unsigned long long)__double_as_longlong(bs.energy);
    if (i == kPfMaxP) v = (unsigned long long)__double_as_longlong(bs.maxp);
    if (i == kPfMaxQ) v = (unsigned long long)__double_as_longlong(bs.maxq);
    part[(size_t)i * kMaxGridBlocks + blockIdx.x] = v;
  }
}

// The same, added to what earlier launches of the kernel stored (first: store).
__device__ __forceinline__ void block_stats_accumulate(const BlockStats& bs,
                                                       unsigned long long* part, bool first) {
  for (int i = threadIdx.x; i < kPfCount; i += blockDim.x) {
    const size_t at = (size_t)i * kMaxGridBlocks + blockIdx.x;
    const unsigned long long old = first ? 0ull : part[at];
    unsigned long long v;
    if (i == kPfEnergy) {
      v = (unsigned long long)__double_as_longlong(
          bs.energy + (first ? 0.0 : __longlong_as_double((long long)old)));
    } else if (i == kPfMaxP || i == kPfMaxQ) {
      const double m = i == kPfMaxP ? bs.maxp : bs.maxq;
      v = (unsigned long long)__double_as_longlong(
          first ? m : fmax(m, __longlong_as_double((long long)old)));
    } else {
      v = bs.w[i] + old;
    }
    part[at] = v;
  }
}

// Append one child per flagged lane to species SP of the lane's instance: one ballot, a
// prefix popcount and one atomic reservation per instance present among the flagged lanes.
// write(store, slot) fills the child's columns.  Must be called by all 64 lanes.
template <int SP, class Writer>
__device__ __forceinline__ void wave_append(const StepArgs& a, bool flag, int inst,
                                            LaneCounters& cnt, Writer&& write) {
  uint64_t m = wave_ballot(flag);
  const uint64_t below = lanes_below();
  while (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int li = wave_bcast(inst, leader);
    const bool mine = flag && inst == li;
    const uint64_t same = wave_ballot(mine);
    long long base = 0;
    if (lane_id() == leader)
      base = (long long)atomicAdd(reinterpret_cast<unsigned long long*>(&a.inst[li].count[SP]),
                                  (unsigned long long)__popcll(same));
    base = wave_bcast(base, leader);
    const long long cap = a.inst[li].capacity[SP];
    const long long pos = base + __popcll(same & below);
    const bool fits = pos < cap;
    if (mine && fits) write(a.sp[SP], a.inst[li].base[SP] + pos);
    // children beyond the capacity are dropped and counted, once per wavefront
    const uint64_t lost = wave_ballot(mine && !fits);
    if (lost != 0 && lane_id() == leader) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.inst[li].dropped),
                (unsigned long long)__popcll(lost));
      atomicAdd(&cnt.bs->w[kPfDropped], (unsigned long long)__popcll(lost));
    }
    m &= ~same;
  }
}

// A wavefront-uniform 64-bit value moved to scalar registers (lane 0's copy).
__device__ __forceinline__ long long wave_uniform(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Wavefront index within the launch (wavefront-uniform).
__device__ __forceinline__ int wave_index() {
  return (int)blockIdx.x * (int)(blockDim.x >> 6) +
         __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Per-wavefront tally of arena records per instance.  Records are counted for the instance
// `cur` in a register; when another instance shows up the tally goes to the wavefront's own
// word of the count matrix (a private address, so the add never waits on other waves).
struct ArenaTally {
  int cur = -1;
  unsigned n = 0;
  __device__ __forceinline__ void flush(const ChildArena& A, int wid) {
    if (n != 0 && lane_id() == 0)
      atomicAdd(&A.cnt[(size_t)cur * A.waves + wid], n);
    n = 0;
  }
  // Count the flagged lanes (mask m) by instance.  All lanes call it.
  __device__ __forceinline__ void add(const ChildArena& A, int wid, uint64_t m, bool flag,
                                      int inst) {
    while (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      const int li = wave_bcast(inst, leader);
      const uint64_t same = wave_ballot(flag && inst == li);
      if (li != cur) {
        flush(A, wid);
        cur = li;
      }
      n += (unsigned)__popcll(same);
      m &= ~same;
    }
  }
};

// A producing wavefront's position in an arena: records written, and the pool chunk it
// fills once its share is full.
struct ArenaCursor {
  long long n = 0;
  unsigned cur = 0xFFFFFFFFu;  // current pool chunk (none yet)
  unsigned fill = (unsigned)kArenaChunk;
};

// Where the ranks of one ballot go: [0, k0) to the share from `share`, [k0, k1) to the
// current chunk from c0, [k1, n) to a new chunk from c1.
struct ArenaSpan {
  long long share, c0, c1;
  int k0, k1;
  __device__ __forceinline__ long long at(int rank) const {
    return rank < k0 ? share + rank : (rank < k1 ? c0 + (rank - k0) : c1 + (rank - k1));
  }
};

// Reserve n_new (1..64) records for one ballot of wavefront wid: the rest of its share,
// then its current chunk, then one new chunk from the pool (one atomic).  False, with
// nothing reserved, when the pool is exhausted.  Wavefront-uniform arguments; all lanes call.
__device__ __forceinline__ bool arena_reserve(const ChildArena& A, int wid, ArenaCursor& c,
                                              int n_new, ArenaSpan& s) {
  const long long room_share = A.per_wave > c.n ? A.per_wave - c.n : 0;
  s.share = (long long)wid * A.per_wave + c.n;
  if (n_new <= room_share) {
    s.k0 = s.k1 = n_new;
    s.c0 = s.c1 = 0;
    c.n += n_new;
    return true;
  }
  s.k0 = (int)room_share;
  const int rest = n_new - s.k0;
  const int room = (int)(kArenaChunk - c.fill);
  s.c0 = A.pool0 + (long long)c.cur * kArenaChunk + c.fill;  // used only if room > 0
  if (rest <= room) {
    s.k1 = n_new;
    s.c1 = 0;
    c.fill += (unsigned)rest;
    c.n += n_new;
    return true;
  }
  unsigned long long nc = 0;
  if (lane_id() == 0) nc = atomicAdd(A.used, 1u);
  nc = (unsigned long long)wave_bcast((long long)nc, 0);
  if (nc >= (unsigned long long)A.nchunks) return false;
  if (lane_id() == 0) {
    if (c.cur == 0xFFFFFFFFu) A.first[wid] = (unsigned)nc;
    else A.next[c.cur] = (unsigned)nc;
  }
  s.k1 = s.k0 + room;
  s.c1 = A.pool0 + (long long)nc * kArenaChunk;
  c.cur = (unsigned)nc;
  c.fill = (unsigned)(rest - room);
  c.n += n_new;
  return true;
}

// The share-only form: false once the ballot does not fit in the rest of the share.
__device__ __forceinline__ bool share_reserve(const ChildArena& A, int wid, ArenaCursor& c,
                                              int n_new, ArenaSpan& s) {
  if (c.n + n_new > A.per_wave) return false;
  s.share = (long long)wid * A.per_wave + c.n;
  s.k0 = s.k1 = n_new;
  s.c0 = s.c1 = 0;
  c.n += n_new;
  return true;
}

// Record indices of producing wavefront sw's records, read in batches [j0, j0 + m) with
// m <= 64 and j0 increasing: advance() (wavefront-uniform) moves to the pool chunk that
// holds the batch's first pool record; index() gives a lane's record j of the batch (below
// n, the wavefront's record count), which lies in the share, that chunk or the next one.
struct ArenaWalk {
  unsigned chunk = 0xFFFFFFFFu;
  long long start = 0;  // the chunk holds pool records [start, start + kArenaChunk) of sw
  __device__ __forceinline__ void advance(const ChildArena& A, int sw, long long j0, long long m,
                                          long long n) {
    if (n <= A.per_wave || j0 + m <= A.per_wave) return;  // the batch is all in the share
    const long long jp = j0 > A.per_wave ? j0 - A.per_wave : 0;
    if (chunk == 0xFFFFFFFFu) {
      chunk = A.first[sw];
      start = 0;
    }
    while (jp >= start + kArenaChunk) {
      chunk = A.next[chunk];
      start += kArenaChunk;
    }
  }
  __device__ __forceinline__ long long index(const ChildArena& A, int sw, long long j) const {
    if (j < A.per_wave) return (long long)sw * A.per_wave + j;
    const long long jp = j - A.per_wave;
    if (jp < start + kArenaChunk) return A.pool0 + (long long)chunk * kArenaChunk + (jp - start);
    return A.pool0 + (long long)A.next[chunk] * kArenaChunk + (jp - start - kArenaChunk);
  }
};

// Current piece of a wavefront's work: slots [cur, end) of one (instance, species) segment.
struct TileCursor {
  long long cur = 0, end = 0;  // slots
  long long g = 0;             // index of slot `cur` in the kernel's particle index space
  int inst = 0, species = 0;
};

// A wavefront's share of the index space [0, N): chunks chunk, chunk + W, ... of T particles.
struct WaveRange {
  long long g, gend, chunk, T, W, N;

  __device__ __forceinline__ void init(long long n, long long tile) {
    const long long wpb = blockDim.x >> 6;
    W = (long long)gridDim.x * wpb;
    const long long wv = (long long)blockIdx.x * wpb +
                         __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    N = n;
    T = tile > 0 ? tile : kDefaultTile;
    if (T < 1) T = 1;
    chunk = wv - W;
    g = gend = 0;
  }
  // Next piece within one segment; false once the wavefront's share is exhausted.
  __device__ __forceinline__ bool next(const StepArgs& a, const long long* pref, int nseg,
                                       bool lepton, TileCursor& tc) {
    while (g >= gend) {
      chunk += W;
      const long long s = chunk * T;
      if (s >= N) return false;
      g = s;
      gend = min(s + T, N);
    }
    int lo = 0, hi = nseg;  // pref[lo] <= g < pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= g) lo = mid;
      else hi = mid;
    }
    const int inst = lepton ? (lo >> 1) : lo;
    const int sp = lepton ? (lo & 1) : QED_PHOTON;
    const long long piece_end = min(gend, pref[lo + 1]);
    const long long base = a.inst[inst].base[sp];
    tc.cur = base + (g - pref[lo]);
    tc.end = tc.cur + (piece_end - g);
    tc.g = g;
    tc.inst = inst;
    tc.species = sp;
    g = piece_end;
    return true;
  }
};

// Does this workgroup own any work?  (its first wavefront's first chunk starts below N)
__device__ __forceinline__ bool block_has_work(long long N, long long tile) {
  const long long wpb = blockDim.x >> 6;
  long long T = tile > 0 ? tile : kDefaultTile;
  if (T < 1) T = 1;
  return (long long)blockIdx.x * wpb * T < N;
}

template <bool MIXED>
struct TabType {
  using T = double2;
};
template <>
struct TabType<true> {
  using T = float2;
};

// Emission decision of the modified generator (Sec. IV.G, Eqs. (24), (25)) for draw o:
// delta = r1^3, emit iff r2 < 3 r1^2 P(r1^3).  The mixed form evaluates the rate and the
// comparison in FP32.
template <bool MIXED>
__device__ __forceinline__ bool emission_decision(const typename TabType<MIXED>::T* tab,
                                                  const Series64& ser64, const Series32& ser32,
                                                  const uint4& o, double chi, double g,
                                                  double dtfac, LaneCounters& cnt,
                                                  double& delta) {
  if (MIXED) {
    const float r1 = uniform32(o.y), r2 = uniform32(o.w);
    const float d = r1 * r1 * r1, omd = 1.0f - d;
    const float z = (2.0f / 3.0f) * d / (omd * (float)chi);
    const float P = 3.0f * r1 * r1 * ((float)(dtfac * kInvSqrt3Pi) / (float)g) *
                    emission_bracket32(reinterpret_cast<const float2*>(tab), ser32, z,
                                       d * d / omd);
    cnt.note((double)P, (double)r2);
    delta = (double)d;
    return r2 < P;
  }
  const double r1 = uniform64(o.x, o.y), r2 = uniform64(o.z, o.w);
  const double d = r1 * r1 * r1, omd = 1.0 - d;
  const double z = (2.0 / 3.0) * d / (omd * chi);
  const double P = 3.0 * r1 * r1 * (dtfac * kInvSqrt3Pi / g) *
                   emission_bracket64(reinterpret_cast<const double2*>(tab), ser64, z,
                                      d * d / omd);
  cnt.note(P, r2);
  delta = d;
  return r2 < P;
}

// The photon of an emission: energy delta gamma m c^2 along p (Sec. IV.F), as the factor
// f = |k| / |p|.  Counts the event's spectrum bin and radiated energy; false (and a
// non-finite count) if p = 0.
__device__ __forceinline__ bool emission_photon(const V3& p, double g, double delta, double wgt,
                                                BlockStats& bs, LaneCounters& cnt, double& f) {
  const double pabs = sqrt(dot(p, p));
  if (!(pabs > 0.0)) {
    block_count(bs, kPfNonfinite);
    return false;
  }
  const double eps = delta * g;
  f = eps / pabs;
  // bin floor(10 (log10 eps + 8)), in FP64 in both precisions (an emission is rare next to
  // the sub-steps, and the bins then agree with an FP64 count of the same photons)
  const double lb = floor(10.0 * (log10(eps) + 8.0));
  if (lb >= 0.0 && lb < (double)QED_SPECTRUM_BINS) atomicAdd(&bs.w[kPfHist + (int)lb], 1ull);
  cnt.energy += wgt * eps;
  return true;
}

// Same-step processing: the time a child has left in the step and its parent's fields,
// stored with its arena record r (the fields only where they depend on position).
template <int FMODE>
__device__ __forceinline__ void record_same_step(const ChildArena& A, long long r, double tau,
                                                 const V3& E, const V3& B) {
  A.tau[r] = tau;
  if (FMODE == kFieldLocal) {
    const long long c = A.cap;
    double* f = A.fe;
    f[r] = E.x;
    f[c + r] = E.y;
    f[2 * c + r] = E.z;
    f[3 * c + r] = B.x;
    f[4 * c + r] = B.y;
    f[5 * c + r] = B.z;
  }
}

// Column pointer of electrons or positrons without indexing the kernel-argument array.
#define LEPTON_COL(col, sp) ((sp) == QED_ELECTRON ? a.sp[QED_ELECTRON].col : a.sp[QED_POSITRON].col)

// Per-wavefront LDS staging of emitted photons.
struct PhotonStage {
  double x[kStageCap], y[kStageCap], z[kStageCap];
  double px[kStageCap], py[kStageCap], pz[kStageCap], w[kStageCap];
  unsigned long long id[kStageCap], parent[kStageCap];
  unsigned int birth[kStageCap];
  int inst[kStageCap];
};

// Reserve slots for the `staged` records and copy them out (lane j takes record j).
__device__ __forceinline__ void flush_stage(const StepArgs& a, PhotonStage& sg, int staged,
                                            LaneCounters& cnt) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int lane = lane_id();
  const bool has = lane < staged;
  const int j = has ? lane : 0;
  const int rinst = has ? sg.inst[j] : -1;
  wave_append<QED_PHOTON>(a, has, rinst, cnt, [&](const qed_soa& o, long long s) {
    o.x[s] = sg.x[j];
    o.y[s] = sg.y[j];
    o.z[s] = sg.z[j];
    o.px[s] = sg.px[j];
    o.py[s] = sg.py[j];
    o.pz[s] = sg.pz[j];
    o.w[s] = sg.w[j];
    o.id[s] = sg.id[j];
    o.parent[s] = sg.parent[j];
    o.birth[s] = sg.birth[j];
    if (o.n_events) o.n_events[s] = 0u;
  });
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Per-wavefront LDS staging of pair creations (one record -> an electron and a positron).
struct PairStage {
  double x[kStageCap], y[kStageCap], z[kStageCap];
  double kx[kStageCap], ky[kStageCap], kz[kStageCap], r1[kStageCap], w[kStageCap];
  unsigned long long parent[kStageCap];
  unsigned int sub[kStageCap];
  int inst[kStageCap];
};

__device__ __forceinline__ void flush_pairs(const StepArgs& a, PairStage& sg, int staged,
                                            uint32_t step, LaneCounters& cnt) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int lane = lane_id();
  const bool has = lane < staged;
  const int j = has ? lane : 0;
  const int rinst = has ? sg.inst[j] : -1;
  const uint64_t seed = has ? a.inst[rinst].seed : 0ull;
  const double r1 = sg.r1[j];
  // electron takes r1 of the photon momentum, positron the rest (Sec. V.A)
  wave_append<QED_ELECTRON>(a, has, rinst, cnt, [&](const qed_soa& o, long long s) {
    o.x[s] = sg.x[j];
    o.y[s] = sg.y[j];
    o.z[s] = sg.z[j];
    o.px[s] = r1 * sg.kx[j];
    o.py[s] = r1 * sg.ky[j];
    o.pz[s] = r1 * sg.kz[j];
    o.w[s] = sg.w[j];
    o.id[s] = child_id(sg.parent[j], seed, step, sg.sub[j], kElectronChild);
    o.parent[s] = sg.parent[j];
    o.birth[s] = birth_code(step, sg.sub[j]);
    if (o.n_events) o.n_events[s] = 0u;
  });
  wave_append<QED_POSITRON>(a, has, rinst, cnt, [&](const qed_soa& o, long long s) {
    const double r1c = 1.0 - r1;
    o.x[s] = sg.x[j];
    o.y[s] = sg.y[j];
    o.z[s] = sg.z[j];
    o.px[s] = r1c * sg.kx[j];
    o.py[s] = r1c * sg.ky[j];
    o.pz[s] = r1c * sg.kz[j];
    o.w[s] = sg.w[j];
    o.id[s] = child_id(sg.parent[j], seed, step, sg.sub[j], kPositronChild);
    o.parent[s] = sg.parent[j];
    o.birth[s] = birth_code(step, sg.sub[j]);
    if (o.n_events) o.n_events[s] = 0u;
  });
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// ------------------------------------------------------------------------------------
// leptons
// ------------------------------------------------------------------------------------
// EXT: the extensions are compiled in -- the generator factor, and same-step processing
// (children also get their time left and the parent's fields; a full share continues in
// pool chunks).  Without them a full share falls back to direct reservation, and the plain
// step's kernel stays lean.
//
// The emission table goes to LDS (64 KB in FP64, 32 KB in FP32), except in the plain FP64
// kernel for a space-independent E with B = 0: there it is read from the L2-resident copy,
// and without the 64 KB of LDS per workgroup the kernel fits three wavefronts per SIMD (the
// compiler holds it to 168 VGPRs with a few spilled), 8% faster on the rotating-field
// cascade.  With a B field the Boris rotation's registers make that bound cost more spills
// than the third wavefront gains (3% slower on 10^4 electrons in a uniform B), and with a
// grid field far more (1.9 times slower), so those kernels keep the LDS table at two
// wavefronts per SIMD.
template <bool MIXED, int FMODE, bool EXT>
struct LeptonShape {
  static constexpr bool global_table = !MIXED && FMODE == kFieldE && !EXT;
  static constexpr int min_waves = global_table ? 3 : 1;
};

// RUNS: the reverse mode of Sec. VI (runs_photon > 1) is compiled in (with EXT).
template <bool MIXED, int FMODE, bool EXT, bool RUNS>
__device__ __forceinline__ void lepton_step(const StepArgs& a) {
  using Tab = typename TabType<MIXED>::T;
  constexpr bool kGlobalTab = LeptonShape<MIXED, FMODE, EXT>::global_table;
  __shared__ Tab tab_lds[kGlobalTab ? 1 : kTableN];
  __shared__ BlockStats bs;
  __shared__ PhotonStage stage[kWavesPerBlock];
  WorkHdr* hdr = a.hdr;
  const long long N = hdr->lep_total;
  const int wid = wave_index();
  block_stats_init(bs);
  if (!block_has_work(N, a.tile)) {
    if (a.pa.waves > 0 && lane_id() == 0) a.pa.nrec[wid] = 0u;
    __syncthreads();
    block_stats_store(bs, a.lep_part);
    return;
  }
  const Tab* src = MIXED ? reinterpret_cast<const Tab*>(a.tables->ab32)
                         : reinterpret_cast<const Tab*>(a.tables->ab64);
  if (!kGlobalTab)
    for (int i = threadIdx.x; i < kTableN; i += blockDim.x) tab_lds[i] = src[i];
  const Tab* tab = kGlobalTab ? src : tab_lds;
  __syncthreads();

  const Series64 ser64 = {a.tables->series[0], a.tables->series[1], a.tables->series[2],
                          a.tables->series[3], a.tables->series[4]};
  const Series32 ser32 = {(float)ser64.b0, (float)ser64.b1, (float)ser64.c0, (float)ser64.c1,
                          (float)ser64.c2};
  const uint32_t step = (uint32_t)hdr->step;
  const int nseg = 2 * a.n_inst;
  FieldArgs fld = a.field;
  fld.tn = hdr->tn;
  const uint64_t below = lanes_below();
  PhotonStage& sg = stage[threadIdx.x >> 6];

  LaneCounters cnt;
  cnt.bs = &bs;
  WaveCounters wc;
  TileCursor tc;
  WaveRange wr;
  wr.init(N, a.tile);
  bool open = true;
  int staged = 0;
  // arena: this wavefront's share, then pool chunks
  const ChildArena& pa = a.pa;
  ArenaCursor acur;
  ArenaTally tally;

  // lane state: sub-step k of the particle in `slot`, `left` sub-steps of length h to go
  // (the current one included)
  long long slot = -1;
  int inst = 0, sp = 0, k = 0, left = 0;
  V3 x{}, p{}, E{}, B{};
  uint64_t id = 0, seed = 0;
  uint32_t nev = 0;
  double qh2 = 0.0, h = 0.0, dtfac = 0.0, wgt = 0.0, hs3 = 0.0;
  const bool refine = a.forced <= 0 && a.adaptive;

  while (true) {
    // ---- refill idle lanes from the wavefront's share, once enough of them are idle ----
    uint64_t freem = wave_ballot(slot < 0);
    if (__popcll(freem) < a.refill_min && ~freem != 0ull) freem = 0ull;
    while (freem != 0 && open) {
      if (tc.cur >= tc.end) {
        open = wr.next(a, a.lep_pref, nseg, true, tc);
        continue;
      }
      const int nfree = __popcll(freem);
      const long long avail = tc.end - tc.cur;
      const int take = (int)(avail < nfree ? avail : nfree);
      const int rank = __popcll(freem & below);
      if (slot < 0 && rank < take) {
        slot = tc.cur + rank;
        inst = tc.inst;
        sp = tc.species;
        x = {LEPTON_COL(x, sp)[slot], LEPTON_COL(y, sp)[slot], LEPTON_COL(z, sp)[slot]};
        p = {LEPTON_COL(px, sp)[slot], LEPTON_COL(py, sp)[slot], LEPTON_COL(pz, sp)[slot]};
        id = LEPTON_COL(id, sp)[slot];
        wgt = LEPTON_COL(w, sp)[slot];
        uint32_t* ne = LEPTON_COL(n_events, sp);
        nev = ne ? ne[slot] : 0u;
        seed = a.inst[inst].seed;
        if (FMODE == kFieldLocal) {
          field_at_position(fld, a.inst[inst].amp, x, E, B);
        } else {
          const double* eb = a.eb + 6 * inst;
          E = {eb[0], eb[1], eb[2]};
          if (FMODE == kFieldEB) B = {eb[3], eb[4], eb[5]};
        }
        // chi and the number of sub-steps, once per step from the step-start state
        const double g = sqrt(1.0 + dot(p, p));
        const double chi = chi_of(p, g, E, FMODE == kFieldE ? V3{0.0, 0.0, 0.0} : B, a.eps_r);
        // (FP64 in both precisions: n_sub is no part of the FP32 rate evaluation)
        int nsub = 1;
        if (a.forced > 0) {
          nsub = a.forced;
        } else if (a.adaptive && chi > 0.0) {
          const NsubInfo ni = nsub_from_ratio(substep_ratio_lepton(a.dt, chi, g, a.inv_lep_scale));
          nsub = ni.n;
          if (ni.near_int) block_count(bs, kPfNearInt);
          if (ni.clamped) block_count(bs, kPfClamped);
        }
        if (!isfinite(chi)) block_count(bs, kPfNonfinite);
        atomicAdd(&bs.w[kPfNsub + (nsub < QED_NSUB_HIST ? nsub : QED_NSUB_HIST - 1)], 1ull);
        h = a.dt / (double)nsub;
        dtfac = h * a.dtfac_per_h;
        qh2 = (sp == QED_ELECTRON ? -0.5 : 0.5) * h;
        hs3 = substep_cube(h, a.inv_lep_scale);
        k = 0;
        left = nsub;
      }
      if (tc.species == QED_ELECTRON) wc.adv0 += take;
      else wc.adv1 += take;
      tc.cur += take;
      freem = wave_ballot(slot < 0);
    }
    const uint64_t act = wave_ballot(slot >= 0);
    if (act == 0) break;
    ++wc.wave_iters;
    wc.low_occ += (__popcll(act) < 32);

    // ---- one sub-step: push, chi, emission decision (Sec. IV.G) ----
    // A sub-step whose end state breaks Eq. (29) is taken again from its start at half the
    // length (rare: such lanes repeat the push while the others wait).
    bool emit = false;
    double f = 0.0, g = 1.0, chi = 0.0;
    // the weight of an event's photon before any factor: w, or w / N_g in the reverse mode
    // of Sec. VI, whose runs beyond the first follow the first below
    const double wrun = RUNS ? wgt / (double)a.runs_photon : wgt;
    if (slot >= 0) {
      const V3 p0 = p;
      for (;;) {
        if (FMODE == kFieldE) {
          // B = 0: the Boris rotation is the identity and the push is p += q h E
          p = {p0.x + 2.0 * qh2 * E.x, p0.y + 2.0 * qh2 * E.y, p0.z + 2.0 * qh2 * E.z};
        } else {
          p = p0;
          boris(p, qh2, E, B);
        }
        const double p2 = dot(p, p);
        g = sqrt(1.0 + p2);
        chi = chi_of(p, g, E, FMODE == kFieldE ? V3{0.0, 0.0, 0.0} : B, a.eps_r);
        if (!(refine && chi > 0.0) ||
            !refine_substep(hs3, chi, p2, g, h, a.inv_lep_scale, k, left, bs))
          break;
        h *= 0.5;
        qh2 *= 0.5;
        dtfac *= 0.5;
        hs3 *= 0.125;
        left *= 2;
      }
      const double hg = h / g;
      x = {x.x + hg * p.x, x.y + hg * p.y, x.z + hg * p.z};
      if (a.emission) {
        const uint4 o = draw_words(id, seed, step, (uint32_t)k, kDraw);
        double delta;
        emit = emission_decision<MIXED>(tab, ser64, ser32, o, chi, g, dtfac, cnt, delta);
        if (emit) {
          emit = emission_photon(p, g, delta, wrun, bs, cnt, f);
          if (emit) ++nev;
        }
      }
    }

    // ---- emitted photons: into the wavefront's arena share, else staged and reserved ----
    // With a generator factor f_g (Sec. VI) the photon of an event is created with
    // probability 1 / f_g, or for every f_g-th event of the lepton in the deterministic
    // form, and carries f_g times the lepton's weight; the recoil below happens at every
    // event.
    wc.substeps += __popcll(act);
    bool child = emit;
    if (EXT && emit) {
      if (a.every_photon) child = generator_every(id, seed, nev - 1u, a.every_photon);
      else if (a.fg_photon > 1.0)
        child = generator_runs(id, seed, step, (uint32_t)k, kGenPhoton, a.inv_fg_photon);
    }
    const double cw = RUNS ? wrun : EXT ? wgt * a.fg_photon : wgt;
    const bool ss = EXT && a.generations > 0;
    const uint64_t em = wave_ballot(child);
    ArenaSpan span;
    if (em && pa.waves > 0 &&
        (EXT ? arena_reserve(pa, wid, acur, __popcll(em), span)
             : share_reserve(pa, wid, acur, __popcll(em), span))) {
      const int n_new = __popcll(em);
      wc.events += n_new;
      tally.add(pa, wid, em, child, inst);
      if (child) {
        const long long r = span.at(__popcll(em & below));
        pa.x[r] = x.x;
        pa.y[r] = x.y;
        pa.z[r] = x.z;
        pa.px[r] = f * p.x;
        pa.py[r] = f * p.y;
        pa.pz[r] = f * p.z;
        pa.w[r] = cw;
        pa.parent[r] = id;
        pa.sub[r] = (unsigned)k;
        pa.inst[r] = (unsigned)inst;
        if (ss) record_same_step<FMODE>(pa, r, (double)(left - 1) * h, E, B);
      }
    } else if (em) {
      const int n_new = __popcll(em);
      wc.events += n_new;
      // reserved directly in the stores: not advanced in this step
      if (ss) wc.deferred += __popcll(wave_ballot(child && left > 1));
      if (staged + n_new > kStageCap) {
        flush_stage(a, sg, staged, cnt);
        staged = 0;
      }
      if (n_new > kStageCap) {
        wave_append<QED_PHOTON>(a, child, inst, cnt, [&](const qed_soa& o, long long s) {
          o.x[s] = x.x;
          o.y[s] = x.y;
          o.z[s] = x.z;
          o.px[s] = f * p.x;
          o.py[s] = f * p.y;
          o.pz[s] = f * p.z;
          o.w[s] = cw;
          o.id[s] = child_id(id, seed, step, (uint32_t)k, kPhotonChild);
          o.parent[s] = id;
          o.birth[s] = birth_code(step, (uint32_t)k);
          if (o.n_events) o.n_events[s] = 0u;
        });
      } else {
        if (child) {
          const int r = staged + __popcll(em & below);
          sg.x[r] = x.x;
          sg.y[r] = x.y;
          sg.z[r] = x.z;
          sg.px[r] = f * p.x;
          sg.py[r] = f * p.y;
          sg.pz[r] = f * p.z;
          sg.w[r] = cw;
          sg.id[r] = child_id(id, seed, step, (uint32_t)k, kPhotonChild);
          sg.parent[r] = id;
          sg.birth[r] = birth_code(step, (uint32_t)k);
          sg.inst[r] = inst;
        }
        staged += n_new;
      }
    }
    if constexpr (RUNS) {
      // reverse mode: runs 1 .. N_g - 1 of the generator on the same state, each photon
      // appended as above; the lepton then recoils by the mean of the runs' photons
      V3 rec = {0.0, 0.0, 0.0};
      if (emit) rec = {f * p.x, f * p.y, f * p.z};
      bool fired = emit;
      for (int run = 1; run < a.runs_photon; ++run) {
        const uint32_t sc = sub_code(k, run);
        bool e2 = false;
        double f2 = 0.0;
        if (slot >= 0 && a.emission) {
          const uint4 o = draw_words(id, seed, step, sc, kDraw);
          double delta;
          e2 = emission_decision<MIXED>(tab, ser64, ser32, o, chi, g, dtfac, cnt, delta);
          if (e2) {
            e2 = emission_photon(p, g, delta, wrun, bs, cnt, f2);
            if (e2) ++nev;
          }
        }
        const uint64_t em2 = wave_ballot(e2);
        if (em2) {
          const int n_new = __popcll(em2);
          wc.events += n_new;
          ArenaSpan span2;
          if (pa.waves > 0 && arena_reserve(pa, wid, acur, n_new, span2)) {
            tally.add(pa, wid, em2, e2, inst);
            if (e2) {
              const long long r = span2.at(__popcll(em2 & below));
              pa.x[r] = x.x;
              pa.y[r] = x.y;
              pa.z[r] = x.z;
              pa.px[r] = f2 * p.x;
              pa.py[r] = f2 * p.y;
              pa.pz[r] = f2 * p.z;
              pa.w[r] = wrun;
              pa.parent[r] = id;
              pa.sub[r] = sc;
              pa.inst[r] = (unsigned)inst;
              if (ss) record_same_step<FMODE>(pa, r, (double)(left - 1) * h, E, B);
            }
          } else {
            // reserved directly in the stores: not advanced in this step
            if (ss) wc.deferred += __popcll(wave_ballot(e2 && left > 1));
            wave_append<QED_PHOTON>(a, e2, inst, cnt, [&](const qed_soa& o, long long s) {
              o.x[s] = x.x;
              o.y[s] = x.y;
              o.z[s] = x.z;
              o.px[s] = f2 * p.x;
              o.py[s] = f2 * p.y;
              o.pz[s] = f2 * p.z;
              o.w[s] = wrun;
              o.id[s] = child_id(id, seed, step, sc, kPhotonChild);
              o.parent[s] = id;
              o.birth[s] = birth_code(step, (uint32_t)k);
              if (o.n_events) o.n_events[s] = 0u;
            });
          }
        }
        if (e2) {
          rec = {rec.x + f2 * p.x, rec.y + f2 * p.y, rec.z + f2 * p.z};
          fired = true;
        }
      }
      if (fired) {
        const double R = (double)a.runs_photon;
        p = {p.x - rec.x / R, p.y - rec.y / R, p.z - rec.z / R};
      }
      emit = false;  // the recoil is done
    }
    if (emit) {
      // recoil: the lepton keeps p - k (momentum conservation, Sec. IV.F)
      const V3 kq = {f * p.x, f * p.y, f * p.z};
      p = {p.x - kq.x, p.y - kq.y, p.z - kq.z};
    }

    // ---- lanes whose particle has done all its sub-steps write back and go idle ----
    if (slot >= 0 && (++k, --left == 0)) {
      LEPTON_COL(x, sp)[slot] = x.x;
      LEPTON_COL(y, sp)[slot] = x.y;
      LEPTON_COL(z, sp)[slot] = x.z;
      LEPTON_COL(px, sp)[slot] = p.x;
      LEPTON_COL(py, sp)[slot] = p.y;
      LEPTON_COL(pz, sp)[slot] = p.z;
      uint32_t* ne = LEPTON_COL(n_events, sp);
      if (ne) ne[slot] = nev;
      slot = -1;
    }
  }
  if (staged > 0) flush_stage(a, sg, staged, cnt);
  if (pa.waves > 0) {
    tally.flush(pa, wid);
    if (lane_id() == 0) pa.nrec[wid] = (unsigned)acur.n;
  }

  wave_to_block(bs, cnt, wc);
  __syncthreads();
  block_stats_store(bs, a.lep_part);
}

template <bool MIXED, int FMODE, bool EXT>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(LeptonShape<MIXED, FMODE, EXT>::min_waves)))
    lepton_kernel(StepArgs a) {
  lepton_step<MIXED, FMODE, EXT, false>(a);
}

// The reverse mode of Sec. VI in a kernel of its own: its extra runs hold more registers,
// which the other forms would pay for in occupancy.  Held to two wavefronts per SIMD (a few
// spilled registers) rather than one.
template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    lepton_runs_kernel(StepArgs a) {
  lepton_step<MIXED, FMODE, true, true>(a);
}

// ------------------------------------------------------------------------------------
// photons
// ------------------------------------------------------------------------------------
// Photons keep chi_gamma fixed over the step (fields frozen, k unchanged), almost always
// need a single sub-step, and are mostly far from pair threshold: a per-octave bound of
// the pair probability settles those decisions from r2 alone.  Two kernels:
//   photon_kernel -- each lane takes the next photon of the wavefront's chunk: fields,
//             chi_gamma, n_sub, then for each sub-step the push and the draw; a draw with
//             r2 below the bound makes the photon a candidate -- its index and sub-step go
//             to a list in the workspace -- and its processing stops there;
//   photon_exact_kernel -- each lane re-derives one candidate's state from the stores (same
//             arithmetic, same draws), evaluates the pair probability of Eq. (30) at the
//             recorded sub-step, finishes the photon's sub-steps and stages the pairs.
// The table lookups, logarithms and exponentials stay out of the bulk kernel, whose small
// register footprint lets many wavefronts stay resident to hide HBM latency.

struct PhotonSetup {
  double chi, h, hk, pref, pbound;
  int nsub;
};

// chi_gamma, n_sub and the rate prefactors of one photon in the fields E, B (identical in
// both photon kernels).  `bound` holds the per-octave pair-rate bounds (staged in LDS).
template <bool MIXED>
__device__ __forceinline__ PhotonSetup photon_setup(const StepArgs& a, const V3& E, const V3& B,
                                                    const V3& kv, double kabs,
                                                    const double* bound, BlockStats* bs) {
  PhotonSetup ps;
  const double inv_k = 1.0 / kabs;
  // chi_gamma (Eqs. (31), (32))
  ps.chi = chi_of(kv, kabs, E, B, a.eps_r);
  ps.nsub = 1;
  if (a.forced > 0) {
    ps.nsub = a.forced;
  } else if (a.adaptive && ps.chi > 0.0) {
    // dt / dt_q with dt_q = kappa 130 (2 pi eps_r) |k| / chi_gamma (Eq. (33))
    const NsubInfo ni = nsub_from_ratio(a.dt * (ps.chi * inv_k) * a.inv_pho_scale);
    ps.nsub = ni.n;
    if (bs) {
      if (ni.near_int) block_count(*bs, kPfNearInt);
      if (ni.clamped) block_count(*bs, kPfClamped);
    }
  }
  if (bs && !isfinite(ps.chi)) block_count(*bs, kPfNonfinite);
  const double h = ps.nsub == 1 ? a.dt : a.dt / (double)ps.nsub;
  ps.h = h;
  ps.hk = h * inv_k;
  ps.pref = h * (a.dtfac_per_h * kInvSqrt3Pi) * inv_k;
  // upper bound of the pair probability over delta_e for this chi's sub-octave
  ps.pbound = 0.0;
  if (ps.chi > 0.0) {
    int e2;
    const double m = frexp(ps.chi, &e2);  // chi = m 2^e2, m in [1/2, 1)
    const int oi = e2 + kBoundOffset;
    if (oi >= kBoundOctaves) {
      ps.pbound = __builtin_inf();
    } else if (oi >= 0) {
      int j = (int)((2.0 * m - 1.0) * kBoundSub);  // exact: chi < (1/2 + (j+1)/32) 2^e2
      j = j < kBoundSub - 1 ? j : kBoundSub - 1;
      ps.pbound = ps.pref * bound[oi * kBoundSub + j];
    }
  }
  return ps;
}

// The per-octave pair-rate bounds into LDS (FP32 values widened in the mixed form).
template <bool MIXED>
__device__ __forceinline__ void stage_bounds(const StepArgs& a, double* sb) {
  for (int i = threadIdx.x; i < kBoundEntries; i += blockDim.x)
    sb[i] = MIXED ? (double)a.tables->pair_bound32[i] : a.tables->pair_bound64[i];
}

// Space-independent fields of a (wavefront-uniform) instance.
template <int FMODE>
__device__ __forceinline__ void instance_fields(const StepArgs& a, int inst, V3& E, V3& B) {
  const double* eb = a.eb + 6 * inst;
  E = {eb[0], eb[1], eb[2]};
  B = FMODE == kFieldEB ? V3{eb[3], eb[4], eb[5]} : V3{0.0, 0.0, 0.0};
}

// Can a draw fall below the bound at all?  The smallest uniform is 2^-53 in FP64 and 2^-24
// in FP32, so a smaller bound settles the decision without drawing.
template <bool MIXED>
__device__ __forceinline__ bool bound_reachable(double pbound) {
  if (MIXED) return (float)pbound > 0x1p-24f;
  return pbound > 0x1p-53;
}

// Below the bound?  (the mixed path compares in FP32, as its exact evaluation does)
template <bool MIXED>
__device__ __forceinline__ bool below_bound(const uint4& o, double pbound) {
  if (MIXED) return uniform32(o.w) < (float)pbound;
  return uniform64(o.z, o.w) < pbound;
}

// Exact pair decision of Eq. (30) for draw o; returns r1 through *r1out.
template <bool MIXED>
__device__ __forceinline__ bool pair_decision(const StepArgs& a, const Series64& s64,
                                              const Series32& s32, const uint4& o, double chi,
                                              double pref, LaneCounters& cnt, double* r1out) {
  if (MIXED) {
    const float r1 = uniform32(o.y), r2 = uniform32(o.w);
    const float omd = 1.0f - r1;
    const float z = (2.0f / 3.0f) / ((float)chi * r1 * omd);
    const float P = (float)pref * pair_bracket32(a.tables->bc32, s32, z, r1 / omd + omd / r1);
    cnt.note((double)P, (double)r2, r2 < P);
    *r1out = (double)r1;
    return r2 < P;
  }
  const double r1 = uniform64(o.x, o.y), r2 = uniform64(o.z, o.w);
  const double omd = 1.0 - r1;
  const double z = (2.0 / 3.0) / (chi * r1 * omd);
  const double P = pref * pair_bracket64(a.tables->bc64, s64, z, r1 / omd + omd / r1);
  cnt.note(P, r2, r2 < P);
  *r1out = r1;
  return r2 < P;
}

// Columns of up to 64 photon slots [base, end) for one wavefront (lane i takes base + i;
// lanes past the end get a dead id).  `base` is wavefront-uniform, so every column is
// addressed by one scalar base and a lane offset.
struct PhotonIn {
  uint64_t id;
  V3 x, k;
};
__device__ __forceinline__ PhotonIn load_photons(const qed_soa& S, long long base, long long end,
                                                 int lane) {
  PhotonIn r{QED_ID_DEAD, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  if (lane < end - base) {
    // the columns this kernel only reads are streamed past the caches (non-temporal): 3%
    // faster; the positions, which it writes back, are slower read that way
    r.id = __builtin_nontemporal_load(&S.id[base + lane]);
    r.x = {S.x[base + lane], S.y[base + lane], S.z[base + lane]};
    r.k = {__builtin_nontemporal_load(&S.px[base + lane]),
           __builtin_nontemporal_load(&S.py[base + lane]),
           __builtin_nontemporal_load(&S.pz[base + lane])};
  }
  return r;
}

template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) photon_kernel(StepArgs a) {
  __shared__ BlockStats bs;
  __shared__ double sbound[kBoundEntries];
  WorkHdr* hdr = a.hdr;
  const long long N = hdr->pho_total;
  const int wid = wave_index();
  block_stats_init(bs);
  stage_bounds<MIXED>(a, sbound);
  __syncthreads();
  if (!block_has_work(N, a.tile)) {
    if (lane_id() == 0) a.candn[wid] = 0u;
    block_stats_store(bs, a.pho_part);
    return;
  }
  const uint32_t step = (uint32_t)hdr->step;
  FieldArgs fld = a.field;
  fld.tn = hdr->tn;
  const uint64_t below = lanes_below();
  const int lane = lane_id();
  const qed_soa& S = a.sp[QED_PHOTON];
  // this wavefront's candidate list; a full list spills to the shared overflow list
  unsigned long long* clist = a.candw + (size_t)wid * a.cand_per_wave;
  long long ncand = 0;

  LaneCounters cnt;
  cnt.bs = &bs;
  WaveCounters wc;
  TileCursor tc;
  WaveRange wr;
  wr.init(N, a.tile);

  // Software pipeline: the next 64 photons' columns (in this piece or the next one) are
  // requested before the current ones are processed, so each wavefront keeps a load batch
  // in flight while it computes.
  bool has = wr.next(a, a.pho_pref, a.n_inst, false, tc);
  PhotonIn nxt{};
  if (has) nxt = load_photons(S, wave_uniform(tc.cur), wave_uniform(tc.end), lane);
  while (has) {
    const int inst = __builtin_amdgcn_readfirstlane(tc.inst);
    const uint64_t seed = a.inst[inst].seed;
    V3 E{}, B{};
    if (FMODE != kFieldLocal) instance_fields<FMODE>(a, inst, E, B);
    const long long cur = wave_uniform(tc.cur), end = wave_uniform(tc.end);
    const long long g0 = wave_uniform(tc.g);
    TileCursor tn;
    bool has_next = false;
    for (long long base = cur; base < end; base += 64) {
      const PhotonIn in = nxt;
      if (base + 64 < end) {
        // the next batch's loads go out at a raised wave priority, ahead of the other
        // wavefronts' arithmetic on the SIMD (265 against 267 us per launch on the
        // rotating-field cascade)
        __builtin_amdgcn_s_setprio(1);
        nxt = load_photons(S, base + 64, end, lane);
        __builtin_amdgcn_s_setprio(0);
      } else {
        has_next = wr.next(a, a.pho_pref, a.n_inst, false, tn);
        if (has_next) nxt = load_photons(S, wave_uniform(tn.cur), wave_uniform(tn.end), lane);
      }
      double* X = S.x + base;
      double* Y = S.y + base;
      double* Z = S.z + base;
      bool cand = false;
      int kcand = 0;
      const uint64_t id = in.id;
      V3 x = in.x;
      const V3 kv = in.k;
      const double kabs = sqrt(dot(kv, kv));
      const bool live = id != QED_ID_DEAD;
      const bool ok = live && kabs > 0.0 && isfinite(kabs);
      if (live && !ok) block_count(bs, kPfNonfinite);
      wc.adv0 += __popcll(wave_ballot(ok));
      if (ok) {
        if (FMODE == kFieldLocal) field_at_position<true>(fld, a.inst[inst].amp, x, E, B);
        const PhotonSetup st = photon_setup<MIXED>(a, E, B, kv, kabs, sbound, &bs);
        int k = 0;
        for (; k < st.nsub; ++k) {
          if (a.push_photons) x = {x.x + st.hk * kv.x, x.y + st.hk * kv.y, x.z + st.hk * kv.z};
          if (!a.pairs) continue;
          if (!bound_reachable<MIXED>(st.pbound)) {
            cnt.early += a.runs_pair;
            continue;
          }
          // a candidate if the draw of any run (N_g of them in the reverse mode of Sec. VI)
          // falls below the bound
          bool hit = below_bound<MIXED>(draw_words(id, seed, step, (uint32_t)k, kDraw),
                                        st.pbound);
          for (int run = 1; run < a.runs_pair && !hit; ++run)
            hit = below_bound<MIXED>(draw_words(id, seed, step, sub_code(k, run), kDraw),
                                     st.pbound);
          if (hit) {
            cand = true;
            kcand = k;
            break;
          }
          cnt.early += a.runs_pair;
        }
        if (!cand) {
          cnt.subs += st.nsub;
          if (a.push_photons) {
            // streaming stores: the positions are not read again in this step (1% faster
            // than plain stores; reading the positions non-temporally as well was slower)
            __builtin_nontemporal_store(x.x, &X[lane]);
            __builtin_nontemporal_store(x.y, &Y[lane]);
            __builtin_nontemporal_store(x.z, &Z[lane]);
          }
        } else {
          cnt.subs += kcand;  // the exact kernel counts the rest
        }
      }
      // ---- record candidates: (photon index << 16) | sub-step ----
      const uint64_t cm = wave_ballot(cand);
      if (cm) {
        const int nc = __popcll(cm);
        const unsigned long long e =
            ((unsigned long long)(g0 + (base - cur) + lane) << 16) | (unsigned long long)kcand;
        if (ncand + nc <= a.cand_per_wave) {
          if (cand) clist[ncand + __popcll(cm & below)] = e;
          ncand += nc;
        } else {
          unsigned long long pos = 0;
          if (lane == 0) pos = atomicAdd(&hdr->n_cand, (unsigned long long)nc);
          pos = wave_bcast(pos, 0) + (unsigned long long)__popcll(cm & below);
          // the overflow list holds one entry per photon slot: never full
          if (cand && pos < (unsigned long long)a.cand_cap) a.cand[pos] = e;
        }
      }
    }
    tc = tn;
    has = has_next;
  }
  if (lane == 0) a.candn[wid] = (unsigned)ncand;
  wave_to_block(bs, cnt, wc);
  __syncthreads();
  block_stats_store(bs, a.pho_part);
}

// State of one wavefront of the exact pair-decision kernel.
struct ExactCtx {
  Series64 ser64;
  Series32 ser32;
  FieldArgs fld;
  uint32_t step;
  int wid;
  int staged;
  ArenaCursor acur;  // this wavefront's place in the pair arena
  ArenaTally tally;
  const double* bound;  // per-octave pair-rate bounds (LDS)
};

// The pair records of the lanes with `make` into the wavefront's arena share or pool chunks,
// else staged and reserved in the stores (an electron and a positron each); all lanes call.
// `sub` is the sub-step code (sub-step and run), `later` whether the pair has time left in
// the step.
template <int FMODE>
__device__ __forceinline__ void exact_append(const StepArgs& a, ExactCtx& c, PairStage& ps,
                                             LaneCounters& cnt, WaveCounters& wc, bool make,
                                             const V3& x, const V3& kv, double r1, double wp,
                                             uint64_t id, uint32_t sub, int inst, double tau,
                                             const V3& Ef, const V3& Bf, bool later) {
  const uint64_t below = lanes_below();
  const uint64_t pm = wave_ballot(make);
  if (!pm) return;
  const int n_new = __popcll(pm);
  wc.events += n_new;
  const ChildArena& qa = a.qa;
  ArenaSpan span;
  if (qa.waves > 0 && arena_reserve(qa, c.wid, c.acur, n_new, span)) {
    // ---- pair records into the wavefront's arena share or pool chunks ----
    c.tally.add(qa, c.wid, pm, make, inst);
    if (make) {
      const long long r = span.at(__popcll(pm & below));
      qa.x[r] = x.x;
      qa.y[r] = x.y;
      qa.z[r] = x.z;
      qa.px[r] = kv.x;
      qa.py[r] = kv.y;
      qa.pz[r] = kv.z;
      qa.r1[r] = r1;
      qa.w[r] = wp;
      qa.parent[r] = id;
      qa.sub[r] = sub;
      qa.inst[r] = (unsigned)inst;
      if (a.generations > 0) record_same_step<FMODE>(qa, r, tau, Ef, Bf);
    }
    return;
  }
  // reserved directly in the stores: not advanced in this step (an electron and a positron)
  if (a.generations > 0) wc.deferred += 2 * __popcll(wave_ballot(later));
  // ---- else stage them and reserve e-/e+ slots once per batch ----
  if (c.staged + n_new > kStageCap) {
    flush_pairs(a, ps, c.staged, c.step, cnt);
    c.staged = 0;
  }
  if (make) {
    const int r = c.staged + __popcll(pm & below);
    ps.x[r] = x.x;
    ps.y[r] = x.y;
    ps.z[r] = x.z;
    ps.kx[r] = kv.x;
    ps.ky[r] = kv.y;
    ps.kz[r] = kv.z;
    ps.r1[r] = r1;
    ps.w[r] = wp;
    ps.parent[r] = id;
    ps.sub[r] = sub;
    ps.inst[r] = inst;
  }
  c.staged += n_new;
}

// One candidate of the photon kernel's lists, re-derived from the stores: its slot, instance,
// columns, fields and setup, and the sub-step kc its draw fell below the bound at.
struct ExactCand {
  long long s;
  int inst, kc;
  uint64_t id, seed;
  V3 x, kv, E, B;
  PhotonSetup st;
};

template <bool MIXED, int FMODE>
__device__ __forceinline__ ExactCand load_candidate(const StepArgs& a, const ExactCtx& c,
                                                    unsigned long long e) {
  const qed_soa& S = a.sp[QED_PHOTON];
  ExactCand q;
  const long long g = (long long)(e >> 16);
  q.kc = (int)(e & 0xFFFFull);
  int lo = 0, hi = a.n_inst;  // pho_pref[lo] <= g < pho_pref[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.pho_pref[mid] <= g) lo = mid;
    else hi = mid;
  }
  q.inst = lo;
  q.s = a.inst[q.inst].base[QED_PHOTON] + (g - a.pho_pref[q.inst]);
  q.id = S.id[q.s];
  q.x = {S.x[q.s], S.y[q.s], S.z[q.s]};
  q.kv = {S.px[q.s], S.py[q.s], S.pz[q.s]};
  const double kabs = sqrt(dot(q.kv, q.kv));
  q.seed = a.inst[q.inst].seed;
  if (FMODE == kFieldLocal) field_at_position<true>(c.fld, a.inst[q.inst].amp, q.x, q.E, q.B);
  else instance_fields<FMODE>(a, q.inst, q.E, q.B);
  q.st = photon_setup<MIXED>(a, q.E, q.B, q.kv, kabs, c.bound, nullptr);
  return q;
}

// Exact pair decision for the candidates list[i0 + lane] (i0 + lane < n); all lanes call.
template <bool MIXED, int FMODE>
__device__ __forceinline__ void exact_batch(const StepArgs& a, ExactCtx& c, PairStage& ps,
                                            LaneCounters& cnt, WaveCounters& wc,
                                            const unsigned long long* list, long long i0,
                                            long long n) {
  const qed_soa& S = a.sp[QED_PHOTON];
  const long long i = i0 + lane_id();
  bool pair = false, make = false;
  double r1 = 0.0, wp = 0.0, tau = 0.0;
  int kpair = 0, inst = 0, nsub = 0;
  V3 x{}, kv{}, Ef{}, Bf{};
  uint64_t id = 0;
  if (i < n) {
    const ExactCand q = load_candidate<MIXED, FMODE>(a, c, list[i]);
    const PhotonSetup& st = q.st;
    const long long s = q.s;
    inst = q.inst;
    id = q.id;
    x = q.x;
    kv = q.kv;
    int done = st.nsub;
    for (int k = 0; k < st.nsub; ++k) {
      if (a.push_photons) x = {x.x + st.hk * kv.x, x.y + st.hk * kv.y, x.z + st.hk * kv.z};
      if (k < q.kc) continue;  // settled by the bound in photon_kernel
      const uint4 o = draw_words(id, q.seed, c.step, (uint32_t)k, kDraw);
      if (k > q.kc && !below_bound<MIXED>(o, st.pbound)) {
        ++cnt.early;
        continue;
      }
      if (pair_decision<MIXED>(a, c.ser64, c.ser32, o, st.chi, st.pref, cnt, &r1)) {
        pair = true;
        kpair = k;
        done = k + 1;
        break;
      }
    }
    cnt.subs += done - q.kc;
    if (a.push_photons) {
      S.x[s] = x.x;
      S.y[s] = x.y;
      S.z[s] = x.z;
    }
    if (pair) {
      // the photon decays at every event; with a generator factor f_g (Sec. VI) the pair is
      // created with probability 1 / f_g, or for one photon in f_g in the deterministic
      // form, and carries f_g times the photon's weight
      S.id[s] = QED_ID_DEAD;
      make = a.every_pair     ? generator_every(id, q.seed, 0u, a.every_pair)
             : a.fg_pair > 1.0 ? generator_runs(id, q.seed, c.step, (uint32_t)kpair, kGenPair,
                                                a.inv_fg_pair)
                               : true;
      wp = S.w[s] * a.fg_pair;
      nsub = st.nsub;
      tau = (double)(st.nsub - kpair - 1) * st.h;
      Ef = q.E;
      Bf = q.B;
    }
  }
  exact_append<FMODE>(a, c, ps, cnt, wc, make, x, kv, r1, wp, id, (uint32_t)kpair, inst, tau,
                      Ef, Bf, make && kpair < nsub - 1);
}

// The same in the reverse mode of Sec. VI (N_g = runs_pair > 1): the photon stands for N_g
// copies of weight w / N_g.  Lanes go through their sub-steps together from the candidate's
// kc; at each, every run draws (the bound settles most), each run that fires makes a pair of
// the copies' weight, the photon keeps the weight of the copies left and is removed when all
// N_g fire.  Pairs are appended run by run, so a photon can make several.
template <bool MIXED, int FMODE>
__device__ __forceinline__ void exact_batch_runs(const StepArgs& a, ExactCtx& c, PairStage& ps,
                                                 LaneCounters& cnt, WaveCounters& wc,
                                                 const unsigned long long* list, long long i0,
                                                 long long n) {
  const qed_soa& S = a.sp[QED_PHOTON];
  const long long i = i0 + lane_id();
  const int R = a.runs_pair;
  bool live = i < n;
  ExactCand q{};
  int k = 0;
  double wcur = 0.0;
  if (live) {
    q = load_candidate<MIXED, FMODE>(a, c, list[i]);
    // the sub-steps before kc were settled by the bound: only the push remains
    if (a.push_photons)
      for (; k < q.kc; ++k)
        q.x = {q.x.x + q.st.hk * q.kv.x, q.x.y + q.st.hk * q.kv.y, q.x.z + q.st.hk * q.kv.z};
    k = q.kc;
    wcur = S.w[q.s];
  }
  while (wave_ballot(live)) {
    double wc_run = 0.0;
    if (live) {
      if (a.push_photons)
        q.x = {q.x.x + q.st.hk * q.kv.x, q.x.y + q.st.hk * q.kv.y, q.x.z + q.st.hk * q.kv.z};
      wc_run = wcur / (double)R;
    }
    int m = 0;
    const double tau = live ? (double)(q.st.nsub - k - 1) * q.st.h : 0.0;
    for (int run = 0; run < R; ++run) {
      bool make = false;
      double r1 = 0.0;
      const uint32_t sc = sub_code(k, run);
      if (live) {
        const uint4 o = draw_words(q.id, q.seed, c.step, sc, kDraw);
        if (!below_bound<MIXED>(o, q.st.pbound)) ++cnt.early;
        else make = pair_decision<MIXED>(a, c.ser64, c.ser32, o, q.st.chi, q.st.pref, cnt, &r1);
        m += make;
      }
      exact_append<FMODE>(a, c, ps, cnt, wc, make, q.x, q.kv, r1, wc_run, q.id, sc, q.inst, tau,
                          q.E, q.B, make && k < q.st.nsub - 1);
    }
    if (live) {
      ++k;
      ++cnt.subs;
      const bool dead = m == R;
      if (!dead && m > 0) wcur = wc_run * (double)(R - m);
      if (dead || k == q.st.nsub) {
        live = false;
        if (a.push_photons) {
          S.x[q.s] = q.x.x;
          S.y[q.s] = q.x.y;
          S.z[q.s] = q.x.z;
        }
        if (dead) S.id[q.s] = QED_ID_DEAD;
        else if (wcur != S.w[q.s]) S.w[q.s] = wcur;
      }
    }
  }
}

template <bool MIXED, int FMODE, bool RUNS>
__device__ __forceinline__ void exact_pass(const StepArgs& a) {
  __shared__ BlockStats bs;
  __shared__ PairStage pstage[kWavesPerBlock];
  __shared__ double sbound[kBoundEntries];
  WorkHdr* hdr = a.hdr;
  block_stats_init(bs);
  stage_bounds<MIXED>(a, sbound);
  __syncthreads();
  ExactCtx c;
  c.bound = sbound;
  c.ser64 = {a.tables->series[0], a.tables->series[1], a.tables->series[2], a.tables->series[3],
             a.tables->series[4]};
  c.ser32 = {(float)c.ser64.b0, (float)c.ser64.b1, (float)c.ser64.c0, (float)c.ser64.c1,
             (float)c.ser64.c2};
  c.fld = a.field;
  c.fld.tn = hdr->tn;
  c.step = (uint32_t)hdr->step;
  c.wid = wave_index();
  c.staged = 0;
  c.acur = ArenaCursor{};
  PairStage& ps = pstage[threadIdx.x >> 6];
  LaneCounters cnt;
  cnt.bs = &bs;
  WaveCounters wc;
  const int V = (int)gridDim.x * (int)(blockDim.x >> 6);

  // the photon kernel's per-wavefront lists, one list per wavefront at a time
  for (int sw = c.wid; sw < a.pho_waves; sw += V) {
    const long long n = (long long)a.candn[sw];
    const unsigned long long* list = a.candw + (size_t)sw * a.cand_per_wave;
    for (long long i0 = 0; i0 < n; i0 += 64) {
      if constexpr (RUNS) exact_batch_runs<MIXED, FMODE>(a, c, ps, cnt, wc, list, i0, n);
      else exact_batch<MIXED, FMODE>(a, c, ps, cnt, wc, list, i0, n);
    }
  }
  // then the overflow list
  long long n = (long long)hdr->n_cand;
  if (n > a.cand_cap) n = a.cand_cap;
  for (long long i0 = (long long)c.wid * 64; i0 < n; i0 += (long long)V * 64) {
    if constexpr (RUNS) exact_batch_runs<MIXED, FMODE>(a, c, ps, cnt, wc, a.cand, i0, n);
    else exact_batch<MIXED, FMODE>(a, c, ps, cnt, wc, a.cand, i0, n);
  }

  if (c.staged > 0) flush_pairs(a, ps, c.staged, c.step, cnt);
  if (a.qa.waves > 0) {
    c.tally.flush(a.qa, c.wid);
    if (lane_id() == 0) a.qa.nrec[c.wid] = (unsigned)c.acur.n;
  }
  wave_to_block(bs, cnt, wc);
  __syncthreads();
  block_stats_store(bs, a.ex_part);
}

template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) photon_exact_kernel(StepArgs a) {
  exact_pass<MIXED, FMODE, false>(a);
}

// The reverse mode of Sec. VI (runs_pair > 1) in a kernel of its own, for the registers,
// held to two wavefronts per SIMD.
template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    photon_exact_runs_kernel(StepArgs a) {
  exact_pass<MIXED, FMODE, true>(a);
}

// ------------------------------------------------------------------------------------
// arena append: scan of the per-(instance, wavefront) counts, then the copy into the stores
// ------------------------------------------------------------------------------------
// One workgroup per instance: exclusive prefix over the wavefronts of each arena's counts
// (in place), the store count before the append into base[], and the counts raised by the
// totals, clamped to the capacities; the copy kernel drops and counts the children that land
// beyond them.
__global__ void __launch_bounds__(1024) arena_scan_kernel(StepArgs a, ChildArena pa,
                                                          ChildArena qa) {
  __shared__ unsigned long long wsum[16];
  const int i = blockIdx.x;
  const int lane = lane_id();
  const int wv = (int)(threadIdx.x >> 6);
  const int nw = (int)(blockDim.x >> 6);
  for (int kind = 0; kind < 2; ++kind) {
    const ChildArena& A = kind == 0 ? pa : qa;
    if (A.waves <= 0) continue;
    unsigned int* row = A.cnt + (size_t)i * A.waves;
    // thread t takes the run [t k, t k + k) of the row: its sum, one scan of the thread
    // sums over the workgroup, then the run's offsets
    const int k = (A.waves + (int)blockDim.x - 1) / (int)blockDim.x;
    const int j0 = (int)threadIdx.x * k;
    const int j1 = j0 + k < A.waves ? j0 + k : A.waves;
    unsigned long long v = 0ull;
    for (int j = j0; j < j1; ++j) v += row[j];
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    unsigned long long run = x - v, carry = 0;
    for (int q = 0; q < nw; ++q) {
      if (q < wv) run += wsum[q];
      carry += wsum[q];
    }
    for (int j = j0; j < j1; ++j) {
      const unsigned c = row[j];
      row[j] = (unsigned)run;
      run += c;
    }
    __syncthreads();  // wsum is taken again for the next arena
    if (threadIdx.x == 0) {
      qed_instance& I = a.inst[i];
      if (kind == 0) {
        A.base[2 * i] = I.count[QED_PHOTON];
        I.count[QED_PHOTON] += (long long)carry;
      } else {
        A.base[2 * i] = I.count[QED_ELECTRON];
        A.base[2 * i + 1] = I.count[QED_POSITRON];
        I.count[QED_ELECTRON] += (long long)carry;
        I.count[QED_POSITRON] += (long long)carry;
      }
    }
  }
  // counts above the capacity (the copy drops and counts what lands beyond it) clamped
  if (threadIdx.x == 0) {
    qed_instance& I = a.inst[i];
    for (int s = 0; s < 3; ++s)
      if (I.count[s] > I.capacity[s]) I.count[s] = I.capacity[s];
  }
}

// Count n children dropped for lack of capacity (rare: only at a full store).
__device__ __forceinline__ void count_drops(const StepArgs& a, int inst, bool lost) {
  uint64_t m = wave_ballot(lost);
  while (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int li = wave_bcast(inst, leader);
    const uint64_t same = wave_ballot(lost && inst == li);
    if (lane_id() == leader) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.inst[li].dropped),
                (unsigned long long)__popcll(same));
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats->dropped),
                (unsigned long long)__popcll(same));
      atomicOr(&a.stats->status, QED_STATUS_DROPPED);
    }
    m &= ~same;
  }
}

// One wavefront per producing wavefront: walks its records in order and gives each the
// next store slot of its instance after the offsets of the scan (a per-instance running
// count in LDS), then writes the child (photon) or both children (pair record), and, for
// same-step processing, the slots into the record.  The launch also clears the count
// matrices of the arenas zpa, zqa (the next generation's, whose readers are done).  When
// the step has no later producer, its first reduce_blocks workgroups take the partial-stats
// reduction instead (the reduce kernel's jobs), and the launch ends the step: the scan has
// clamped the counts and the status bits are set where their counters are raised, so only
// the step counter is left to advance (no kernel of this launch reads it).
__global__ void __launch_bounds__(256) arena_copy_kernel(StepArgs a, ChildArena pa,
                                                         ChildArena qa, ChildArena zpa,
                                                         ChildArena zqa, int reduce_blocks) {
  __shared__ unsigned int lcnt[kWavesPerBlock][kArenaMaxInstances];
  if ((int)blockIdx.x < reduce_blocks) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.d_step = a.hdr->step + 1;
    reduce_job(a, (int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6), lane_id());
    return;
  }
  const int blk = (int)blockIdx.x - reduce_blocks;  // the copy's own workgroups
  const int nblk = (int)gridDim.x - reduce_blocks;
  {
    const long long n1 = zpa.waves > 0 ? (long long)a.n_inst * zpa.waves : 0;
    const long long n2 = zqa.waves > 0 ? (long long)a.n_inst * zqa.waves : 0;
    const long long stride = (long long)nblk * blockDim.x;
    for (long long i = (long long)blk * blockDim.x + threadIdx.x; i < n1 + n2; i += stride) {
      if (i < n1) zpa.cnt[i] = 0u;
      else zqa.cnt[i - n1] = 0u;
    }
    if (blk == 0 && threadIdx.x == 0) {
      if (zpa.waves > 0) *zpa.used = 0u;
      if (zqa.waves > 0) *zqa.used = 0u;
    }
  }
  unsigned int* run = lcnt[threadIdx.x >> 6];
  const uint64_t below = lanes_below();
  const int lane = lane_id();
  const uint32_t step = (uint32_t)a.hdr->step;
  const int npa = pa.waves;
  const int nqa = qa.waves;
  const int V = nblk * (int)(blockDim.x >> 6);
  const int wid = blk * (int)(blockDim.x >> 6) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int t = wid; t < npa + nqa; t += V) {
    const bool pair = t >= npa;
    const ChildArena& A = pair ? qa : pa;
    const int sw = pair ? t - npa : t;
    const long long n = (long long)A.nrec[sw];
    if (n == 0) continue;
    for (int q = lane; q < a.n_inst; q += 64) run[q] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    ArenaWalk walk;
    for (long long j0 = 0; j0 < n; j0 += 64) {
      const long long j = j0 + lane;
      const bool has = j < n;
      walk.advance(A, sw, j0, 64, n);
      const long long r = has ? walk.index(A, sw, j) : 0;
      const int li = has ? (int)A.inst[r] : -1;
      unsigned local = 0;
      uint64_t m = wave_ballot(has);
      while (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        const int lj = wave_bcast(li, leader);
        const uint64_t same = wave_ballot(has && li == lj);
        const unsigned c0 = run[lj];
        if (has && li == lj) local = c0 + (unsigned)__popcll(same & below);
        __builtin_amdgcn_wave_barrier();
        if (lane == leader) run[lj] = c0 + (unsigned)__popcll(same);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        m &= ~same;
      }
      bool lost0 = false, lost1 = false;
      if (has) {
        const qed_instance& I = a.inst[li];
        const long long off = (long long)A.cnt[(size_t)li * A.waves + sw] + local;
        const uint64_t seed = I.seed;
        // each record is read once (non-temporal loads: 20.2 to 18.4 us a launch)
        const uint32_t sub = __builtin_nontemporal_load(&A.sub[r]);
        const uint64_t parent = __builtin_nontemporal_load(&A.parent[r]);
        const double x = __builtin_nontemporal_load(&A.x[r]);
        const double y = __builtin_nontemporal_load(&A.y[r]);
        const double z = __builtin_nontemporal_load(&A.z[r]);
        const double px = __builtin_nontemporal_load(&A.px[r]);
        const double py = __builtin_nontemporal_load(&A.py[r]);
        const double pz = __builtin_nontemporal_load(&A.pz[r]);
        const double w = __builtin_nontemporal_load(&A.w[r]);
        if (!pair) {
          const long long d = A.base[2 * li] + off;
          if (d < I.capacity[QED_PHOTON]) {
            const qed_soa& o = a.sp[QED_PHOTON];
            const long long q = I.base[QED_PHOTON] + d;
            o.x[q] = x;
            o.y[q] = y;
            o.z[q] = z;
            o.px[q] = px;
            o.py[q] = py;
            o.pz[q] = pz;
            o.w[q] = w;
            o.id[q] = child_id(parent, seed, step, sub, kPhotonChild);
            o.parent[q] = parent;
            o.birth[q] = birth_code(step, sub);
            if (o.n_events) o.n_events[q] = 0u;
            if (A.slot) A.slot[r] = q;
          } else {
            lost0 = true;
            if (A.slot) A.slot[r] = -1;
          }
        } else {
          // electron takes r1 of the photon momentum, positron the rest (Sec. V.A)
          const double r1 = A.r1[r];
          const double r1c = 1.0 - r1;
          const long long de = A.base[2 * li] + off;
          if (de < I.capacity[QED_ELECTRON]) {
            const qed_soa& o = a.sp[QED_ELECTRON];
            const long long q = I.base[QED_ELECTRON] + de;
            o.x[q] = x;
            o.y[q] = y;
            o.z[q] = z;
            o.px[q] = r1 * px;
            o.py[q] = r1 * py;
            o.pz[q] = r1 * pz;
            o.w[q] = w;
            o.id[q] = child_id(parent, seed, step, sub, kElectronChild);
            o.parent[q] = parent;
            o.birth[q] = birth_code(step, sub);
            if (o.n_events) o.n_events[q] = 0u;
            if (A.slot) A.slot[r] = q;
          } else {
            lost0 = true;
            if (A.slot) A.slot[r] = -1;
          }
          const long long dp = A.base[2 * li + 1] + off;
          if (dp < I.capacity[QED_POSITRON]) {
            const qed_soa& o = a.sp[QED_POSITRON];
            const long long q = I.base[QED_POSITRON] + dp;
            o.x[q] = x;
            o.y[q] = y;
            o.z[q] = z;
            o.px[q] = r1c * px;
            o.py[q] = r1c * py;
            o.pz[q] = r1c * pz;
            o.w[q] = w;
            o.id[q] = child_id(parent, seed, step, sub, kPositronChild);
            o.parent[q] = parent;
            o.birth[q] = birth_code(step, sub);
            if (o.n_events) o.n_events[q] = 0u;
            if (A.slot2) A.slot2[r] = q;
          } else {
            lost1 = true;
            if (A.slot2) A.slot2[r] = -1;
          }
        }
      }
      if (wave_ballot(lost0 || lost1)) {
        count_drops(a, li, lost0);
        count_drops(a, li, lost1);
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// children in their birth step (same-step processing)
// ------------------------------------------------------------------------------------
// A generation pass reads the records the previous pass (or the step's particle kernels)
// wrote and the copy kernel placed in the stores, advances each child in its store slot
// through the time it has left in the step, with its parent's frozen fields, and writes the
// children it creates to the other arena set (with their own time left), from where the
// next scan and copy place them.  Generations alternate between the two sets.
struct GenArgs {
  ChildArena ipa, iqa;  // input: photon records and pair records of the previous pass
  ChildArena opa, oqa;  // output: this kernel's wavefronts write their children here
  int pass;             // 1 .. G
  int last;             // 1 on pass G: what it creates waits for the next step
};
// kernel arguments stay within the 4 KB the launch passes
static_assert(sizeof(StepArgs) + sizeof(GenArgs) <= 4096, "generation kernel arguments");
static_assert(sizeof(StepArgs) + 4 * sizeof(ChildArena) + 8 <= 4096, "copy kernel arguments");

// Fields a child inherited from its parent (record r of A).
template <int FMODE>
__device__ __forceinline__ void inherited_fields(const StepArgs& a, const ChildArena& A,
                                                 long long r, int inst, V3& E, V3& B) {
  if (FMODE == kFieldLocal) {
    const long long c = A.cap;
    const double* f = A.fe;
    E = {f[r], f[c + r], f[2 * c + r]};
    B = {f[3 * c + r], f[4 * c + r], f[5 * c + r]};
  } else {
    instance_fields<FMODE>(a, inst, E, B);
  }
}

struct GenWave {
  int wid;
  ArenaCursor cp, cq;  // this wavefront's place in opa, oqa
  ArenaTally tp, tq;
};

// A wavefront's stream of children: the records of producing wavefronts wid, wid + V, ...
// of arena A, one item per photon record or two (electron, positron) per pair record,
// handed out in pieces of consecutive items of one producing wavefront.
struct GenStream {
  int t = 0, V = 1;
  long long j = 0, n = 0;  // next item, items of producing wavefront t
  bool pair = false, open = false;
  ArenaWalk walk;
  __device__ __forceinline__ void init(const ChildArena& A, int wid, int v, bool is_pair) {
    t = wid;
    V = v;
    pair = is_pair;
    open = A.waves > 0 && t < A.waves;
    n = open ? (pair ? 2 : 1) * (long long)A.nrec[t] : 0;
    j = 0;
  }
  // The next piece [j0, j0 + take), take <= want <= 64; false once the stream is exhausted.
  // Wavefront-uniform; all lanes call.
  __device__ __forceinline__ bool next(const ChildArena& A, int want, long long& j0, int& take) {
    while (open && j >= n) {
      t += V;
      if (t >= A.waves) {
        open = false;
        break;
      }
      n = (pair ? 2 : 1) * (long long)A.nrec[t];
      j = 0;
      walk = ArenaWalk{};
    }
    if (!open) return false;
    take = (int)((long long)want < n - j ? (long long)want : n - j);
    j0 = j;
    const long long rec0 = pair ? (j0 >> 1) : j0;
    const long long rec1 = pair ? ((j0 + take + 1) >> 1) : j0 + take;
    walk.advance(A, t, rec0, rec1 - rec0, pair ? (n >> 1) : n);
    j += take;
    return true;
  }
  // Record holding item jj of the current piece.
  __device__ __forceinline__ long long record(const ChildArena& A, long long jj) const {
    return walk.index(A, t, pair ? (jj >> 1) : jj);
  }
};

// Electrons and positrons of the input pair records, each advanced through its tau; a lane
// whose lepton has done all its sub-steps takes the next one from the wavefront's stream.
template <bool MIXED, int FMODE, bool RUNS>
__device__ __forceinline__ void gen_lepton_phase(const StepArgs& a, const GenArgs& q,
                                                 GenWave& gw, int V,
                                                 const typename TabType<MIXED>::T* tab,
                                                 const Series64& ser64, const Series32& ser32,
                                                 BlockStats& bs, LaneCounters& cnt,
                                                 WaveCounters& wc) {
  const ChildArena& A = q.iqa;
  const ChildArena& O = q.opa;
  const uint64_t below = lanes_below();
  const uint32_t step = (uint32_t)a.hdr->step;
  GenStream st;
  st.init(A, gw.wid, V, true);
  long long slot = -1;
  int sp = 0, inst = 0, left = 0, k = 0;
  V3 x{}, p{}, E{}, B{};
  uint64_t id = 0, seed = 0;
  double wgt = 0.0, h = 0.0, dtfac = 0.0, qh2 = 0.0, hs3 = 0.0;
  uint32_t nev = 0;
  const bool refine = a.forced <= 0 && a.adaptive;
  while (true) {
    // ---- refill idle lanes ----
    uint64_t freem = wave_ballot(slot < 0);
    while (freem) {
      long long j0;
      int take;
      if (!st.next(A, __popcll(freem), j0, take)) break;
      const int rank = __popcll(freem & below);
      bool act = false;
      if (slot < 0 && rank < take) {
        const long long jj = j0 + rank;
        const long long r = st.record(A, jj);
        const long long sl = (jj & 1) ? A.slot2[r] : A.slot[r];
        const double tau = A.tau[r];
        if (sl >= 0 && tau > 0.0) {
          act = true;
          sp = (jj & 1) ? QED_POSITRON : QED_ELECTRON;
          inst = (int)A.inst[r];
          x = {LEPTON_COL(x, sp)[sl], LEPTON_COL(y, sp)[sl], LEPTON_COL(z, sp)[sl]};
          p = {LEPTON_COL(px, sp)[sl], LEPTON_COL(py, sp)[sl], LEPTON_COL(pz, sp)[sl]};
          id = LEPTON_COL(id, sp)[sl];
          wgt = LEPTON_COL(w, sp)[sl];
          uint32_t* ne = LEPTON_COL(n_events, sp);
          nev = ne ? ne[sl] : 0u;
          seed = a.inst[inst].seed;
          inherited_fields<FMODE>(a, A, r, inst, E, B);
          const double g = sqrt(1.0 + dot(p, p));
          const double chi = chi_of(p, g, E, FMODE == kFieldE ? V3{0.0, 0.0, 0.0} : B, a.eps_r);
          int nsub = 1;
          if (a.forced > 0) {
            nsub = a.forced;
          } else if (a.adaptive && chi > 0.0) {
            const NsubInfo ni =
                nsub_from_ratio(substep_ratio_lepton(tau, chi, g, a.inv_lep_scale));
            nsub = ni.n;
            if (ni.near_int) block_count(bs, kPfNearInt);
            if (ni.clamped) block_count(bs, kPfClamped);
          }
          if (!isfinite(chi)) block_count(bs, kPfNonfinite);
          h = tau / (double)nsub;
          dtfac = h * a.dtfac_per_h;
          qh2 = (sp == QED_ELECTRON ? -0.5 : 0.5) * h;
          hs3 = substep_cube(h, a.inv_lep_scale);
          k = 0;
          left = nsub;
          slot = sl;
        }
      }
      wc.children += __popcll(wave_ballot(act));
      freem = wave_ballot(slot < 0);
    }
    if (wave_ballot(slot >= 0) == 0) break;

    // ---- one sub-step (taken again at half the length if its end state breaks Eq. (29)) ----
    double g = 1.0, chi = 0.0;
    if (slot >= 0) {
      const V3 p0 = p;
      for (;;) {
        if (FMODE == kFieldE) {
          p = {p0.x + 2.0 * qh2 * E.x, p0.y + 2.0 * qh2 * E.y, p0.z + 2.0 * qh2 * E.z};
        } else {
          p = p0;
          boris(p, qh2, E, B);
        }
        const double p2 = dot(p, p);
        g = sqrt(1.0 + p2);
        chi = chi_of(p, g, E, FMODE == kFieldE ? V3{0.0, 0.0, 0.0} : B, a.eps_r);
        if (!(refine && chi > 0.0) ||
            !refine_substep(hs3, chi, p2, g, h, a.inv_lep_scale, k, left, bs))
          break;
        h *= 0.5;
        qh2 *= 0.5;
        dtfac *= 0.5;
        hs3 *= 0.125;
        left *= 2;
      }
      const double hg = h / g;
      x = {x.x + hg * p.x, x.y + hg * p.y, x.z + hg * p.z};
      ++cnt.subs;
    }
    // the emission generator, N_g times in the reverse mode of Sec. VI (as in lepton_kernel)
    const int runs = RUNS ? a.runs_photon : 1;
    const double wrun = wgt / (double)runs;
    V3 rec = {0.0, 0.0, 0.0};
    bool fired = false;
    for (int run = 0; run < runs; ++run) {
      const uint32_t sc = sub_code(k, run);
      bool emit = false;
      double f = 0.0;
      if (slot >= 0 && a.emission) {
        const uint4 o = draw_words(id, seed, step, sc, kDraw);
        double delta;
        emit = emission_decision<MIXED>(tab, ser64, ser32, o, chi, g, dtfac, cnt, delta);
        if (emit) {
          emit = emission_photon(p, g, delta, wrun, bs, cnt, f);
          if (emit) ++nev;
        }
      }
      bool child = emit;
      if (emit) {
        if (a.every_photon) child = generator_every(id, seed, nev - 1u, a.every_photon);
        else if (a.fg_photon > 1.0)
          child = generator_runs(id, seed, step, (uint32_t)k, kGenPhoton, a.inv_fg_photon);
      }
      const uint64_t em = wave_ballot(child);
      if (em) {
        const int n_new = __popcll(em);
        wc.events += n_new;
        const double cw = runs > 1 ? wrun : wgt * a.fg_photon;
        const bool later = child && left > 1;  // the photon has time left in the step
        ArenaSpan span;
        if (O.waves > 0 && arena_reserve(O, gw.wid, gw.cp, n_new, span)) {
          gw.tp.add(O, gw.wid, em, child, inst);
          if (child) {
            const long long rr = span.at(__popcll(em & below));
            O.x[rr] = x.x;
            O.y[rr] = x.y;
            O.z[rr] = x.z;
            O.px[rr] = f * p.x;
            O.py[rr] = f * p.y;
            O.pz[rr] = f * p.z;
            O.w[rr] = cw;
            O.parent[rr] = id;
            O.sub[rr] = sc;
            O.inst[rr] = (unsigned)inst;
            record_same_step<FMODE>(O, rr, (double)(left - 1) * h, E, B);
          }
          if (q.last) wc.deferred += __popcll(wave_ballot(later));
        } else {
          // the arena is full: reserved directly, not advanced in this step
          wave_append<QED_PHOTON>(a, child, inst, cnt, [&](const qed_soa& o, long long s2) {
            o.x[s2] = x.x;
            o.y[s2] = x.y;
            o.z[s2] = x.z;
            o.px[s2] = f * p.x;
            o.py[s2] = f * p.y;
            o.pz[s2] = f * p.z;
            o.w[s2] = cw;
            o.id[s2] = child_id(id, seed, step, sc, kPhotonChild);
            o.parent[s2] = id;
            o.birth[s2] = birth_code(step, (uint32_t)k);
            if (o.n_events) o.n_events[s2] = 0u;
          });
          wc.deferred += __popcll(wave_ballot(later));
        }
      }
      if (emit) {
        // recoil: the lepton keeps p - k (momentum conservation, Sec. IV.F)
        if (runs == 1) {
          p = {p.x - f * p.x, p.y - f * p.y, p.z - f * p.z};
        } else {
          rec = {rec.x + f * p.x, rec.y + f * p.y, rec.z + f * p.z};
          fired = true;
        }
      }
    }
    if (fired) {
      const double R = (double)runs;
      p = {p.x - rec.x / R, p.y - rec.y / R, p.z - rec.z / R};
    }
    if (slot >= 0 && (++k, --left == 0)) {
      LEPTON_COL(x, sp)[slot] = x.x;
      LEPTON_COL(y, sp)[slot] = x.y;
      LEPTON_COL(z, sp)[slot] = x.z;
      LEPTON_COL(px, sp)[slot] = p.x;
      LEPTON_COL(py, sp)[slot] = p.y;
      LEPTON_COL(pz, sp)[slot] = p.z;
      uint32_t* ne = LEPTON_COL(n_events, sp);
      if (ne) ne[slot] = nev;
      slot = -1;
    }
  }
}

// Photons of the input photon records, each advanced through its tau (lane refill as for
// the leptons).
template <bool MIXED, int FMODE, bool RUNS>
__device__ __forceinline__ void gen_photon_phase(const StepArgs& a, const GenArgs& q,
                                                 GenWave& gw, int V, const Series64& ser64,
                                                 const Series32& ser32, BlockStats& bs,
                                                 LaneCounters& cnt, LaneCounters& pcnt,
                                                 WaveCounters& wc) {
  const ChildArena& A = q.ipa;
  const ChildArena& O = q.oqa;
  const uint64_t below = lanes_below();
  const uint32_t step = (uint32_t)a.hdr->step;
  const qed_soa& S = a.sp[QED_PHOTON];
  const bool photons = a.push_photons || a.pairs;
  GenStream st;
  st.init(A, gw.wid, V, false);
  long long slot = -1;
  int inst = 0, nsub = 0, k = 0;
  uint64_t id = 0, seed = 0;
  V3 x{}, kv{}, E{}, B{};
  double chi = 0.0, h = 0.0, hk = 0.0, pref = 0.0, wcur = 0.0;
  while (true) {
    // ---- refill idle lanes ----
    uint64_t freem = wave_ballot(slot < 0);
    while (freem) {
      long long j0;
      int take;
      if (!st.next(A, __popcll(freem), j0, take)) break;
      const int rank = __popcll(freem & below);
      bool act = false;
      if (slot < 0 && rank < take) {
        const long long r = st.record(A, j0 + rank);
        const long long sl = A.slot[r];
        const double tau = A.tau[r];
        act = sl >= 0 && tau > 0.0;
        if (act && photons) {
          id = S.id[sl];
          x = {S.x[sl], S.y[sl], S.z[sl]};
          kv = {S.px[sl], S.py[sl], S.pz[sl]};
          const double kabs = sqrt(dot(kv, kv));
          if (!(kabs > 0.0) || !isfinite(kabs)) {
            block_count(bs, kPfNonfinite);
          } else {
            inst = (int)A.inst[r];
            seed = a.inst[inst].seed;
            inherited_fields<FMODE>(a, A, r, inst, E, B);
            const double inv_k = 1.0 / kabs;
            chi = chi_of(kv, kabs, E, B, a.eps_r);
            nsub = 1;
            if (a.forced > 0) {
              nsub = a.forced;
            } else if (a.adaptive && chi > 0.0) {
              // tau / dt_q with dt_q of Eq. (33)
              const NsubInfo ni = nsub_from_ratio(tau * (chi * inv_k) * a.inv_pho_scale);
              nsub = ni.n;
              if (ni.near_int) block_count(bs, kPfNearInt);
              if (ni.clamped) block_count(bs, kPfClamped);
            }
            if (!isfinite(chi)) block_count(bs, kPfNonfinite);
            h = nsub == 1 ? tau : tau / (double)nsub;
            hk = h * inv_k;
            pref = h * (a.dtfac_per_h * kInvSqrt3Pi) * inv_k;
            wcur = S.w[sl];
            k = 0;
            slot = sl;
          }
        }
      }
      wc.children += __popcll(wave_ballot(act));
      freem = wave_ballot(slot < 0);
    }
    if (wave_ballot(slot >= 0) == 0) break;

    // ---- one sub-step: the pair generator once, or N_g times in the reverse mode of
    // Sec. VI (as in the exact pass) ----
    const int R = RUNS ? a.runs_pair : 1;
    int m = 0;
    if (slot >= 0) {
      if (a.push_photons) x = {x.x + hk * kv.x, x.y + hk * kv.y, x.z + hk * kv.z};
      ++cnt.subs;
    }
    const double wc_run = R > 1 ? wcur / (double)R : wcur;
    for (int run = 0; run < R; ++run) {
      const uint32_t sc = sub_code(k, run);
      bool make = false;
      double r1 = 0.0, wp = 0.0;
      if (slot >= 0 && a.pairs) {
        const uint4 o = draw_words(id, seed, step, sc, kDraw);
        if (pair_decision<MIXED>(a, ser64, ser32, o, chi, pref, pcnt, &r1)) {
          ++m;
          // the photon decays; its pair is created with probability 1 / f_g, or for one
          // photon in f_g in the deterministic form (Sec. VI)
          make = R > 1           ? true
                 : a.every_pair  ? generator_every(id, seed, 0u, a.every_pair)
                 : a.fg_pair > 1.0 ? generator_runs(id, seed, step, (uint32_t)k, kGenPair,
                                                    a.inv_fg_pair)
                                   : true;
          wp = R > 1 ? wc_run : wcur * a.fg_pair;
        }
      }
      const uint64_t pm = wave_ballot(make);
      if (!pm) continue;
      const int n_new = __popcll(pm);
      wc.pairs += n_new;
      const bool later = make && k < nsub - 1;
      ArenaSpan span;
      if (O.waves > 0 && arena_reserve(O, gw.wid, gw.cq, n_new, span)) {
        gw.tq.add(O, gw.wid, pm, make, inst);
        if (make) {
          const long long rr = span.at(__popcll(pm & below));
          O.x[rr] = x.x;
          O.y[rr] = x.y;
          O.z[rr] = x.z;
          O.px[rr] = kv.x;
          O.py[rr] = kv.y;
          O.pz[rr] = kv.z;
          O.r1[rr] = r1;
          O.w[rr] = wp;
          O.parent[rr] = id;
          O.sub[rr] = sc;
          O.inst[rr] = (unsigned)inst;
          record_same_step<FMODE>(O, rr, (double)(nsub - k - 1) * h, E, B);
        }
        if (q.last) wc.deferred += 2 * __popcll(wave_ballot(later));
      } else {
        // the arena is full: reserved directly, not advanced in this step
        const double r1c = 1.0 - r1;
        wave_append<QED_ELECTRON>(a, make, inst, cnt, [&](const qed_soa& o, long long s2) {
          o.x[s2] = x.x;
          o.y[s2] = x.y;
          o.z[s2] = x.z;
          o.px[s2] = r1 * kv.x;
          o.py[s2] = r1 * kv.y;
          o.pz[s2] = r1 * kv.z;
          o.w[s2] = wp;
          o.id[s2] = child_id(id, seed, step, sc, kElectronChild);
          o.parent[s2] = id;
          o.birth[s2] = birth_code(step, (uint32_t)k);
          if (o.n_events) o.n_events[s2] = 0u;
        });
        wave_append<QED_POSITRON>(a, make, inst, cnt, [&](const qed_soa& o, long long s2) {
          o.x[s2] = x.x;
          o.y[s2] = x.y;
          o.z[s2] = x.z;
          o.px[s2] = r1c * kv.x;
          o.py[s2] = r1c * kv.y;
          o.pz[s2] = r1c * kv.z;
          o.w[s2] = wp;
          o.id[s2] = child_id(id, seed, step, sc, kPositronChild);
          o.parent[s2] = id;
          o.birth[s2] = birth_code(step, (uint32_t)k);
          if (o.n_events) o.n_events[s2] = 0u;
        });
        wc.deferred += 2 * __popcll(wave_ballot(later));
      }
    }
    if (slot >= 0) {
      const bool dead = m == R;  // every copy decayed
      if (!dead && m > 0) wcur = wc_run * (double)(R - m);
      if (dead || ++k == nsub) {
        if (a.push_photons) {
          S.x[slot] = x.x;
          S.y[slot] = x.y;
          S.z[slot] = x.z;
        }
        if (dead) S.id[slot] = QED_ID_DEAD;
        else if (wcur != S.w[slot]) S.w[slot] = wcur;
        slot = -1;
      }
    }
  }
}

template <bool MIXED, int FMODE, bool RUNS>
__device__ __forceinline__ void gen_pass(const StepArgs& a, const GenArgs& q) {
  using Tab = typename TabType<MIXED>::T;
  __shared__ BlockStats bs;
  __shared__ Tab tab[kTableN];  // the emission table, as in the lepton kernel
  block_stats_init(bs);
  {
    const Tab* src = MIXED ? reinterpret_cast<const Tab*>(a.tables->ab32)
                           : reinterpret_cast<const Tab*>(a.tables->ab64);
    for (int i = threadIdx.x; i < kTableN; i += blockDim.x) tab[i] = src[i];
  }
  __syncthreads();
  const Series64 ser64 = {a.tables->series[0], a.tables->series[1], a.tables->series[2],
                          a.tables->series[3], a.tables->series[4]};
  const Series32 ser32 = {(float)ser64.b0, (float)ser64.b1, (float)ser64.c0, (float)ser64.c1,
                          (float)ser64.c2};
  const int lane = lane_id();
  const int V = (int)gridDim.x * (int)(blockDim.x >> 6);
  GenWave gw;
  gw.wid = wave_index();
  LaneCounters cnt, pcnt;  // pcnt: pair decisions
  cnt.bs = &bs;
  pcnt.bs = &bs;
  WaveCounters wc;
  // photons of the previous generation, then its electrons and positrons
  gen_photon_phase<MIXED, FMODE, RUNS>(a, q, gw, V, ser64, ser32, bs, cnt, pcnt, wc);
  gen_lepton_phase<MIXED, FMODE, RUNS>(a, q, gw, V, tab, ser64, ser32, bs, cnt, wc);
  if (q.opa.waves > 0) {
    gw.tp.flush(q.opa, gw.wid);
    if (lane == 0) q.opa.nrec[gw.wid] = (unsigned)gw.cp.n;
  }
  if (q.oqa.waves > 0) {
    gw.tq.flush(q.oqa, gw.wid);
    if (lane == 0) q.oqa.nrec[gw.wid] = (unsigned)gw.cq.n;
  }
  wave_to_block(bs, cnt, wc, &pcnt);
  __syncthreads();
  block_stats_accumulate(bs, a.gen_part, q.pass == 1);
}

template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) gen_kernel(StepArgs a, GenArgs q) {
  gen_pass<MIXED, FMODE, false>(a, q);
}

// The reverse mode of Sec. VI (runs_photon or runs_pair > 1) in a kernel of its own.
template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) gen_runs_kernel(StepArgs a, GenArgs q) {
  gen_pass<MIXED, FMODE, true>(a, q);
}

#undef LEPTON_COL

// ------------------------------------------------------------------------------------
// Returns whether the arena copy took the partial-stats reduction and ended the step (no
// producer after it).
template <bool MIXED, int FMODE>
static bool launch_persistent(const StepArgs& a, LaunchShape lep, LaunchShape pho,
                              bool run_photons, hipStream_t s) {
  if (a.events[0]) (void)hipEventRecord(a.events[0], s);
  if (a.runs_photon > 1)
    hipLaunchKernelGGL((lepton_runs_kernel<MIXED, FMODE>), dim3(lep.grid), dim3(lep.block), 0,
                       s, a);
  else if (a.generations > 0 || a.fg_photon > 1.0)
    hipLaunchKernelGGL((lepton_kernel<MIXED, FMODE, true>), dim3(lep.grid), dim3(lep.block), 0,
                       s, a);
  else
    hipLaunchKernelGGL((lepton_kernel<MIXED, FMODE, false>), dim3(lep.grid), dim3(lep.block), 0,
                       s, a);
  if (a.events[1]) (void)hipEventRecord(a.events[1], s);
  if (run_photons) {
    if (a.events[2]) (void)hipEventRecord(a.events[2], s);
    hipLaunchKernelGGL((photon_kernel<MIXED, FMODE>), dim3(pho.grid), dim3(pho.block), 0, s, a);
    if (a.events[3]) (void)hipEventRecord(a.events[3], s);
    if (a.ex_grid > 0 && a.runs_pair > 1)
      hipLaunchKernelGGL((photon_exact_runs_kernel<MIXED, FMODE>), dim3(a.ex_grid), dim3(256), 0,
                         s, a);
    else if (a.ex_grid > 0)
      hipLaunchKernelGGL((photon_exact_kernel<MIXED, FMODE>), dim3(a.ex_grid), dim3(256), 0, s, a);
  }
  const int src = a.pa.waves + a.qa.waves;
  const ChildArena none{};
  const bool gen = a.generations > 0;
  const int rb = gen ? 0 : kReduceBlocks;
  if (src > 0) {
    hipLaunchKernelGGL(arena_scan_kernel, dim3(a.n_inst), dim3(1024), 0, s, a, a.pa, a.qa);
    // with same-step processing the copy also clears generation 1's count matrices
    hipLaunchKernelGGL(arena_copy_kernel,
                       dim3(rb + (src + kWavesPerBlock - 1) / kWavesPerBlock), dim3(256), 0, s,
                       a, a.pa, a.qa, gen ? a.gpa[1] : none, gen ? a.gqa[1] : none, rb);
  }
  // children through the rest of the step: generation g reads set (g - 1) % 2 (set 0 as the
  // particle kernels wrote it for g = 1) and writes set g % 2
  for (int g = 1; g <= a.generations; ++g) {
    GenArgs q;
    q.ipa = g == 1 ? a.pa : a.gpa[(g - 1) % 2];
    q.iqa = g == 1 ? a.qa : a.gqa[(g - 1) % 2];
    q.opa = a.gpa[g % 2];
    q.oqa = a.gqa[g % 2];
    q.pass = g;
    q.last = g == a.generations ? 1 : 0;
    if (a.runs_photon > 1 || a.runs_pair > 1)
      hipLaunchKernelGGL((gen_runs_kernel<MIXED, FMODE>), dim3(a.gen_grid), dim3(256), 0, s, a, q);
    else
      hipLaunchKernelGGL((gen_kernel<MIXED, FMODE>), dim3(a.gen_grid), dim3(256), 0, s, a, q);
    const int gsrc = q.opa.waves + q.oqa.waves;
    const bool more = g < a.generations;
    hipLaunchKernelGGL(arena_scan_kernel, dim3(a.n_inst), dim3(1024), 0, s, a, q.opa, q.oqa);
    hipLaunchKernelGGL(arena_copy_kernel, dim3((gsrc + kWavesPerBlock - 1) / kWavesPerBlock),
                       dim3(256), 0, s, a, q.opa, q.oqa, more ? a.gpa[(g + 1) % 2] : none,
                       more ? a.gqa[(g + 1) % 2] : none, 0);
  }
  return src > 0 && !gen;
}

int field_mode(int kind) {
  if (kind == QED_FIELD_UNIFORM) return kFieldEB;
  if (kind == QED_FIELD_ROTATING_E) return kFieldE;
  return kFieldLocal;
}

hipError_t launch_step(const StepArgs& a, int precision, LaunchShape lep, LaunchShape pho,
                       bool run_photons, hipStream_t s) {
  const long long zero_words = (long long)a.n_inst * (a.pa.waves + a.qa.waves);
  long long zb = (zero_words + 2047) / 2048;
  if (zb > 1024) zb = 1024;
  hipLaunchKernelGGL(prep_kernel, dim3(1 + (int)zb), dim3(256), 0, s, a, run_photons ? 1 : 0);
  const int fm = field_mode(a.field.kind);
  bool reduced;
  if (precision == QED_MIXED) {
    if (fm == kFieldEB) reduced = launch_persistent<true, kFieldEB>(a, lep, pho, run_photons, s);
    else if (fm == kFieldE) reduced = launch_persistent<true, kFieldE>(a, lep, pho, run_photons, s);
    else reduced = launch_persistent<true, kFieldLocal>(a, lep, pho, run_photons, s);
  } else {
    if (fm == kFieldEB) reduced = launch_persistent<false, kFieldEB>(a, lep, pho, run_photons, s);
    else if (fm == kFieldE) reduced = launch_persistent<false, kFieldE>(a, lep, pho, run_photons, s);
    else reduced = launch_persistent<false, kFieldLocal>(a, lep, pho, run_photons, s);
  }
  if (!reduced) {
    hipLaunchKernelGGL(reduce_kernel, dim3(kReduceBlocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// Resident workgroups per CU of a step kernel: kind 0 the photon kernel, 1 the lepton
// kernel, 2 its extended form, 3 its reverse-mode form.
template <bool MIXED, int FMODE>
static int occupancy(int kind, int block) {
  int nb = 0;
  hipError_t e;
  if (kind == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, photon_kernel<MIXED, FMODE>, block, 0);
  else if (kind == 3)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lepton_runs_kernel<MIXED, FMODE>,
                                                     block, 0);
  else if (kind == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lepton_kernel<MIXED, FMODE, true>,
                                                     block, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lepton_kernel<MIXED, FMODE, false>,
                                                     block, 0);
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

template <bool MIXED>
static int occupancy_of(int fmode, int kind, int block) {
  if (fmode == kFieldEB) return occupancy<MIXED, kFieldEB>(kind, block);
  if (fmode == kFieldE) return occupancy<MIXED, kFieldE>(kind, block);
  return occupancy<MIXED, kFieldLocal>(kind, block);
}

int step_blocks_per_cu(int precision, int fmode, int kind, int block) {
  return precision == QED_MIXED ? occupancy_of<true>(fmode, kind, block)
                                : occupancy_of<false>(fmode, kind, block);
}

}  // namespace qedk
