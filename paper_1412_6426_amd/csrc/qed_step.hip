// qed_step.hip -- the per-step kernels of the QED step (Sec. IV.H adaptive event generator
// of Gonoskov et al., arXiv:1412.6426, with the Sec. V.A pair generator).
//
// One step is four launches on the caller's stream:
//   prep     (1 workgroup)  snapshot live counts, tile prefix sums, space-independent
//                           fields at t_n, zero the stats record;
//   leptons  (persistent)   electrons and positrons: push, chi, emission, photon append;
//   photons  (persistent)   photons: push, chi_gamma, pair creation, e-/e+ append;
//   finalize (1 workgroup)  clamp counts, status bits, step index + 1.
// Children land after the step-start counts, so they are first processed at step n+1.
//
// Work distribution: each wavefront pulls tiles of `tile` consecutive slots from a global
// queue and keeps its 64 lanes busy by refilling any lane whose particle has finished all
// of its sub-steps from the current tile ("per-wavefront work queue"): a wavefront
// iteration advances every active lane by exactly one sub-step, so lanes with n_sub = 1 and
// n_sub = 20 share a wavefront without idling.  Rate tables are staged once per workgroup
// into LDS.  New particles are appended with one wavefront ballot, a prefix popcount and a
// single atomic reservation per (wavefront, instance).
#include "qed_internal.h"

namespace qedk {

// ------------------------------------------------------------------------------------
// prep / finalize
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) prep_kernel(StepArgs a, int run_photons) {
  __shared__ int s_ok;
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
  // zero the stats record
  unsigned long long* sw = reinterpret_cast<unsigned long long*>(a.stats);
  for (int w = threadIdx.x; w < (int)(sizeof(qed_stats) / 8); w += blockDim.x) sw[w] = 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long lt = 0, pt = 0, ns[3] = {0, 0, 0};
    a.lep_pref[0] = 0;
    a.pho_pref[0] = 0;
    for (int i = 0; i < a.n_inst; ++i) {
      for (int s = 0; s < 2; ++s) {
        const long long c = a.n0[i * 3 + s];
        lt += (c + a.tile - 1) / a.tile;
        a.lep_pref[2 * i + s + 1] = lt;
        ns[s] += c;
      }
      const long long c = a.n0[i * 3 + 2];
      if (run_photons) pt += (c + a.tile - 1) / a.tile;
      a.pho_pref[i + 1] = pt;
      ns[2] += c;
    }
    hdr->lep_queue = 0ull;
    hdr->pho_queue = 0ull;
    hdr->lep_tiles = lt;
    hdr->pho_tiles = pt;
    hdr->step = n;
    hdr->tn = tn;
    hdr->tables_ok = (uint32_t)ok;
    a.stats->step = n;
    for (int s = 0; s < 3; ++s) a.stats->n_start[s] = ns[s];
    if (!ok) a.stats->status = QED_STATUS_NO_TABLES;
  }
}

__global__ void __launch_bounds__(256) finalize_kernel(StepArgs a) {
  for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) {
    qed_instance& I = a.inst[i];
    for (int s = 0; s < 3; ++s)
      if (I.count[s] > I.capacity[s]) I.count[s] = I.capacity[s];
  }
  if (threadIdx.x == 0) {
    qed_stats* st = a.stats;
    uint32_t status = st->status;
    if (st->dropped > 0) status |= QED_STATUS_DROPPED;
    if (st->nonfinite > 0) status |= QED_STATUS_NONFINITE;
    if (st->saturated > 0) status |= QED_STATUS_SATURATED;
    if (st->nsub_clamped > 0) status |= QED_STATUS_NSUB_CLAMPED;
    st->status = status;
    *a.d_step = a.hdr->step + 1;
  }
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

struct LaneCounters {
  int substeps = 0, events = 0, saturated = 0, near = 0, nonfinite = 0, near_int = 0,
      clamped = 0, dropped = 0, early = 0, adv0 = 0, adv1 = 0;
  double energy = 0.0, maxp = 0.0;

  __device__ __forceinline__ void note(double P, double r2) {
    if (!isfinite(P)) {
      ++nonfinite;
      return;
    }
    maxp = fmax(maxp, P);
    saturated += (P >= 1.0);
    near += (fabs(r2 - P) < kNearThreshold);
  }
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

__device__ void flush_counters(const StepArgs& a, const LaneCounters& c, bool photon_kernel,
                               long long wave_iters, long long low_occ) {
  const long long sub = wave_sum((long long)c.substeps), ev = wave_sum((long long)c.events);
  const long long sat = wave_sum((long long)c.saturated), nr = wave_sum((long long)c.near);
  const long long nf = wave_sum((long long)c.nonfinite), ni = wave_sum((long long)c.near_int);
  const long long cl = wave_sum((long long)c.clamped), dr = wave_sum((long long)c.dropped);
  const long long eo = wave_sum((long long)c.early);
  const long long a0 = wave_sum((long long)c.adv0), a1 = wave_sum((long long)c.adv1);
  const double en = wave_sum(c.energy), mp = wave_max(c.maxp);
  if (lane_id() == 0) {
    qed_stats* st = a.stats;
    auto add = [](int64_t* p, long long v) {
      if (v) atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
    };
    add(&st->substeps, sub);
    add(photon_kernel ? &st->pairs : &st->emitted, ev);
    add(&st->saturated, sat);
    add(&st->near_threshold, nr);
    add(&st->nonfinite, nf);
    add(&st->nsub_near_int, ni);
    add(&st->nsub_clamped, cl);
    add(&st->dropped, dr);
    add(&st->early_out, eo);
    if (photon_kernel) {
      add(&st->advanced[QED_PHOTON], a0);
    } else {
      add(&st->advanced[QED_ELECTRON], a0);
      add(&st->advanced[QED_POSITRON], a1);
    }
    if (!photon_kernel) {
      add(&st->wave_iters, wave_iters);
      add(&st->low_occupancy_iters, low_occ);
      if (en != 0.0) atomicAdd(&st->photon_energy, en);
    }
    atomic_max_nonneg(photon_kernel ? &st->max_p_pair : &st->max_p_emit, mp);
  }
}

// Append one child per flagged lane to species SP of the lane's own instance: one ballot,
// a prefix popcount and one atomic reservation per instance present in the wavefront.
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
    if (mine) {
      const long long pos = base + __popcll(same & below);
      const qed_instance& I = a.inst[li];
      if (pos < I.capacity[SP]) {
        write(a.sp[SP], I.base[SP] + pos);
      } else {
        atomicAdd(reinterpret_cast<unsigned long long*>(&a.inst[li].dropped), 1ull);
        ++cnt.dropped;
      }
    }
    m &= ~same;
  }
}

// Hand out the next tile of a queue to the whole wavefront; returns false once drained.
// pref holds nseg+1 tile prefix sums over segments: (instance, e-/e+) for leptons,
// instances for photons.
struct TileCursor {
  long long cur = 0, end = 0;
  int inst = 0, species = 0;
};

__device__ __forceinline__ bool next_tile(const StepArgs& a, unsigned long long* queue,
                                          long long ntiles, const long long* pref, int nseg,
                                          bool lepton, TileCursor& tc) {
  long long t = 0;
  if (lane_id() == 0) t = (long long)atomicAdd(queue, 1ull);
  t = wave_bcast(t, 0);
  if (t >= ntiles) return false;
  int lo = 0, hi = nseg;  // pref[lo] <= t < pref[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pref[mid] <= t) lo = mid;
    else hi = mid;
  }
  const int inst = lepton ? (lo >> 1) : lo;
  const int sp = lepton ? (lo & 1) : QED_PHOTON;
  const long long lt = t - pref[lo];
  const long long n0 = a.n0[inst * 3 + sp];
  const long long base = a.inst[inst].base[sp];
  tc.cur = base + lt * a.tile;
  tc.end = base + min((lt + 1) * a.tile, n0);
  tc.inst = inst;
  tc.species = sp;
  return true;
}

template <bool MIXED>
struct TabType {
  using T = double2;
};
template <>
struct TabType<true> {
  using T = float2;
};

// Column pointer of electrons or positrons without indexing the kernel-argument array.
#define LEPTON_COL(col, sp) ((sp) == QED_ELECTRON ? a.sp[QED_ELECTRON].col : a.sp[QED_POSITRON].col)

// ------------------------------------------------------------------------------------
// leptons
// ------------------------------------------------------------------------------------
template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) lepton_kernel(StepArgs a) {
  using Tab = typename TabType<MIXED>::T;
  __shared__ Tab tab[kTableN];
  __shared__ unsigned int s_nsub[QED_NSUB_HIST];
  __shared__ unsigned int s_hist[QED_SPECTRUM_BINS];
  __shared__ int s_go;
  WorkHdr* hdr = a.hdr;
  if (threadIdx.x == 0)
    s_go = (__hip_atomic_load(&hdr->lep_queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
            (unsigned long long)hdr->lep_tiles);
  __syncthreads();
  if (!s_go) return;
  {
    const Tab* src = MIXED ? reinterpret_cast<const Tab*>(a.tables->ab32)
                           : reinterpret_cast<const Tab*>(a.tables->ab64);
    for (int i = threadIdx.x; i < kTableN; i += blockDim.x) tab[i] = src[i];
    for (int i = threadIdx.x; i < QED_NSUB_HIST; i += blockDim.x) s_nsub[i] = 0u;
    for (int i = threadIdx.x; i < QED_SPECTRUM_BINS; i += blockDim.x) s_hist[i] = 0u;
  }
  __syncthreads();

  const Series64 ser64 = {a.tables->series[0], a.tables->series[1], a.tables->series[2],
                          a.tables->series[3], a.tables->series[4]};
  const Series32 ser32 = {(float)ser64.b0, (float)ser64.b1, (float)ser64.c0, (float)ser64.c1,
                          (float)ser64.c2};
  const uint32_t step = (uint32_t)hdr->step;
  const long long ntiles = hdr->lep_tiles;
  const int nseg = 2 * a.n_inst;
  FieldArgs fld = a.field;
  fld.tn = hdr->tn;
  const uint64_t below = lanes_below();

  LaneCounters cnt;
  long long wave_iters = 0, low_occ = 0;
  TileCursor tc;
  bool open = true;

  // lane state
  long long slot = -1;
  int inst = 0, sp = 0, k = 0, nsub = 0;
  V3 x{}, p{}, E{}, B{};
  uint64_t id = 0, seed = 0;
  uint32_t nev = 0;
  double qh2 = 0.0, h = 0.0, dtfac = 0.0;

  while (true) {
    // ---- refill idle lanes from the wavefront's queue ----
    uint64_t freem = wave_ballot(slot < 0);
    while (freem != 0 && open) {
      if (tc.cur >= tc.end) {
        open = next_tile(a, &hdr->lep_queue, ntiles, a.lep_pref, nseg, true, tc);
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
        nsub = 1;
        if (a.forced > 0) {
          nsub = a.forced;
        } else if (a.adaptive && chi > 0.0) {
          NsubInfo ni;
          if (MIXED) {
            const float r = (float)(chi / g);
            const float ratio = (float)a.dt * cbrtf(r * r) * (float)a.inv_lep_scale;
            ni = nsub_from_ratio((double)ratio);
          } else {
            ni = nsub_from_ratio(substep_ratio_lepton(a.dt, chi, g, a.inv_lep_scale));
          }
          nsub = ni.n;
          cnt.near_int += ni.near_int;
          cnt.clamped += ni.clamped;
        }
        if (!isfinite(chi)) ++cnt.nonfinite;
        atomicAdd(&s_nsub[nsub < QED_NSUB_HIST ? nsub : QED_NSUB_HIST - 1], 1u);
        cnt.adv0 += (sp == QED_ELECTRON);
        cnt.adv1 += (sp != QED_ELECTRON);
        h = a.dt / (double)nsub;
        dtfac = h * a.dtfac_per_h;
        qh2 = (sp == QED_ELECTRON ? -0.5 : 0.5) * h;
        k = 0;
      }
      tc.cur += take;
      freem = wave_ballot(slot < 0);
    }
    const uint64_t act = wave_ballot(slot >= 0);
    if (act == 0) break;
    ++wave_iters;
    low_occ += (__popcll(act) < 32);

    // ---- one sub-step: push, chi, emission decision (Sec. IV.G) ----
    bool emit = false;
    double f = 0.0, g = 1.0;
    if (slot >= 0) {
      if (FMODE == kFieldE) {
        // B = 0: the Boris rotation is the identity and the push is p += q h E
        p = {p.x + 2.0 * qh2 * E.x, p.y + 2.0 * qh2 * E.y, p.z + 2.0 * qh2 * E.z};
      } else {
        boris(p, qh2, E, B);
      }
      g = sqrt(1.0 + dot(p, p));
      const double hg = h / g;
      x = {x.x + hg * p.x, x.y + hg * p.y, x.z + hg * p.z};
      const double chi = chi_of(p, g, E, FMODE == kFieldE ? V3{0.0, 0.0, 0.0} : B, a.eps_r);
      ++cnt.substeps;
      if (a.emission) {
        const uint4 o = draw_words(id, seed, step, (uint32_t)k, kDraw);
        double delta;
        if (MIXED) {
          const float r1 = uniform32(o.y), r2 = uniform32(o.w);
          const float d = r1 * r1 * r1, omd = 1.0f - d;
          const float z = (2.0f / 3.0f) * d / (omd * (float)chi);
          const float P = 3.0f * r1 * r1 * ((float)(dtfac * kInvSqrt3Pi) / (float)g) *
                          emission_bracket32(reinterpret_cast<const float2*>(tab), ser32, z,
                                             d * d / omd);
          cnt.note((double)P, (double)r2);
          emit = r2 < P;
          delta = (double)d;
        } else {
          const double r1 = uniform64(o.x, o.y), r2 = uniform64(o.z, o.w);
          const double d = r1 * r1 * r1, omd = 1.0 - d;
          const double z = (2.0 / 3.0) * d / (omd * chi);
          const double P = 3.0 * r1 * r1 * (dtfac * kInvSqrt3Pi / g) *
                           emission_bracket64(reinterpret_cast<const double2*>(tab), ser64, z,
                                              d * d / omd);
          cnt.note(P, r2);
          emit = r2 < P;
          delta = d;
        }
        if (emit) {
          // photon of energy delta gamma m c^2 along p (Sec. IV.F)
          const double pabs = sqrt(dot(p, p));
          if (pabs > 0.0) {
            const double eps = delta * g;
            f = eps / pabs;
            ++nev;
            ++cnt.events;
            const double w = LEPTON_COL(w, sp)[slot];
            cnt.energy += w * eps;
            const float lb = (__log10f((float)eps) + 8.0f) * 10.0f;
            if (lb >= 0.0f && lb < (float)QED_SPECTRUM_BINS) atomicAdd(&s_hist[(int)lb], 1u);
          } else {
            emit = false;
            ++cnt.nonfinite;
          }
        }
      }
    }
    wave_append<QED_PHOTON>(a, emit, inst, cnt, [&](const qed_soa& o, long long s) {
      o.x[s] = x.x;
      o.y[s] = x.y;
      o.z[s] = x.z;
      o.px[s] = f * p.x;
      o.py[s] = f * p.y;
      o.pz[s] = f * p.z;
      o.w[s] = LEPTON_COL(w, sp)[slot];
      o.id[s] = child_id(id, seed, step, (uint32_t)k, kPhotonChild);
      o.parent[s] = id;
      o.birth[s] = birth_code(step, (uint32_t)k);
      if (o.n_events) o.n_events[s] = 0u;
    });
    if (emit) {
      // recoil: the lepton keeps p - k (momentum conservation, Sec. IV.F)
      const V3 kq = {f * p.x, f * p.y, f * p.z};
      p = {p.x - kq.x, p.y - kq.y, p.z - kq.z};
    }

    // ---- lanes whose particle has done all its sub-steps write back and go idle ----
    if (slot >= 0 && ++k == nsub) {
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

  flush_counters(a, cnt, false, wave_iters, low_occ);
  __syncthreads();
  for (int i = threadIdx.x; i < QED_NSUB_HIST; i += blockDim.x)
    if (s_nsub[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats->nsub_hist[i]),
                             (unsigned long long)s_nsub[i]);
  for (int i = threadIdx.x; i < QED_SPECTRUM_BINS; i += blockDim.x)
    if (s_hist[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats->photon_hist[i]),
                             (unsigned long long)s_hist[i]);
}

// ------------------------------------------------------------------------------------
// photons
// ------------------------------------------------------------------------------------
// Photons keep chi_gamma fixed over the step (fields frozen, k unchanged), and most of them
// are far from pair threshold: a per-octave bound of the pair probability settles those
// decisions from r2 alone, so the rate tables are read straight from the (L2-resident)
// table buffer rather than staged in LDS, leaving LDS free for occupancy.
template <bool MIXED, int FMODE>
__global__ void __launch_bounds__(256) photon_kernel(StepArgs a) {
  __shared__ int s_go;
  WorkHdr* hdr = a.hdr;
  if (threadIdx.x == 0)
    s_go = (__hip_atomic_load(&hdr->pho_queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
            (unsigned long long)hdr->pho_tiles);
  __syncthreads();
  if (!s_go) return;

  const Series64 ser64 = {a.tables->series[0], a.tables->series[1], a.tables->series[2],
                          a.tables->series[3], a.tables->series[4]};
  const Series32 ser32 = {(float)ser64.b0, (float)ser64.b1, (float)ser64.c0, (float)ser64.c1,
                          (float)ser64.c2};
  const uint32_t step = (uint32_t)hdr->step;
  const long long ntiles = hdr->pho_tiles;
  FieldArgs fld = a.field;
  fld.tn = hdr->tn;
  const uint64_t below = lanes_below();
  const qed_soa& S = a.sp[QED_PHOTON];

  LaneCounters cnt;
  TileCursor tc;
  bool open = true;

  long long slot = -1;
  int inst = 0, k = 0, nsub = 0;
  V3 x{}, kv{};
  uint64_t id = 0, seed = 0;
  double hk = 0.0, chi = 0.0, pref = 0.0, pbound = 0.0;

  while (true) {
    uint64_t freem = wave_ballot(slot < 0);
    while (freem != 0 && open) {
      if (tc.cur >= tc.end) {
        open = next_tile(a, &hdr->pho_queue, ntiles, a.pho_pref, a.n_inst, false, tc);
        continue;
      }
      const int nfree = __popcll(freem);
      const long long avail = tc.end - tc.cur;
      const int take = (int)(avail < nfree ? avail : nfree);
      const int rank = __popcll(freem & below);
      if (slot < 0 && rank < take) {
        const long long s = tc.cur + rank;
        const uint64_t pid = S.id[s];
        if (pid != QED_ID_DEAD) {
          x = {S.x[s], S.y[s], S.z[s]};
          kv = {S.px[s], S.py[s], S.pz[s]};
          const double kabs = sqrt(dot(kv, kv));
          if (!(kabs > 0.0) || !isfinite(kabs)) {
            ++cnt.nonfinite;
          } else {
            slot = s;
            inst = tc.inst;
            id = pid;
            ++cnt.adv0;
            seed = a.inst[inst].seed;
            V3 E, B{0.0, 0.0, 0.0};
            if (FMODE == kFieldLocal) {
              field_at_position(fld, a.inst[inst].amp, x, E, B);
            } else {
              const double* eb = a.eb + 6 * inst;
              E = {eb[0], eb[1], eb[2]};
              if (FMODE == kFieldEB) B = {eb[3], eb[4], eb[5]};
            }
            // chi_gamma (Eqs. (31), (32))
            chi = chi_of(kv, kabs, E, B, a.eps_r);
            nsub = 1;
            if (a.forced > 0) {
              nsub = a.forced;
            } else if (a.adaptive && chi > 0.0) {
              const NsubInfo ni =
                  nsub_from_ratio(substep_ratio_photon(a.dt, chi, kabs, a.inv_pho_scale));
              nsub = ni.n;
              cnt.near_int += ni.near_int;
              cnt.clamped += ni.clamped;
            }
            if (!isfinite(chi)) ++cnt.nonfinite;
            const double h = a.dt / (double)nsub;
            hk = h / kabs;
            pref = h * a.dtfac_per_h * kInvSqrt3Pi / kabs;
            pbound = 0.0;
            if (chi > 0.0) {
              int e2;
              frexp(chi, &e2);  // chi < 2^e2
              const int oi = e2 + kBoundOffset;
              if (oi >= kBoundOctaves) pbound = __builtin_inf();
              else if (oi >= 0)
                pbound = pref * (MIXED ? (double)a.tables->pair_bound32[oi]
                                       : a.tables->pair_bound64[oi]);
            }
            k = 0;
          }
        }
      }
      tc.cur += take;
      freem = wave_ballot(slot < 0);
    }
    if (wave_ballot(slot >= 0) == 0) break;

    bool pair = false;
    double r1d = 0.0;
    if (slot >= 0) {
      if (a.push_photons) x = {x.x + hk * kv.x, x.y + hk * kv.y, x.z + hk * kv.z};
      ++cnt.substeps;
      if (a.pairs) {
        const uint4 o = draw_words(id, seed, step, (uint32_t)k, kDraw);
        if (MIXED) {
          const float r1 = uniform32(o.y), r2 = uniform32(o.w);
          r1d = (double)r1;
          if (r2 >= (float)pbound) {
            ++cnt.early;
          } else {
            const float omd = 1.0f - r1;
            const float z = (2.0f / 3.0f) / ((float)chi * r1 * omd);
            const float P = (float)pref * pair_bracket32(a.tables->bc32, ser32, z,
                                                         r1 / omd + omd / r1);
            cnt.note((double)P, (double)r2);
            pair = r2 < P;
          }
        } else {
          const double r1 = uniform64(o.x, o.y), r2 = uniform64(o.z, o.w);
          r1d = r1;
          if (r2 >= pbound) {
            ++cnt.early;
          } else {
            const double omd = 1.0 - r1;
            const double z = (2.0 / 3.0) / (chi * r1 * omd);
            const double P = pref * pair_bracket64(a.tables->bc64, ser64, z, r1 / omd + omd / r1);
            cnt.note(P, r2);
            pair = r2 < P;
          }
        }
        cnt.events += pair;
      }
    }
    // electron takes r1 of the photon momentum, positron the rest (Sec. V.A)
    wave_append<QED_ELECTRON>(a, pair, inst, cnt, [&](const qed_soa& o, long long s) {
      o.x[s] = x.x;
      o.y[s] = x.y;
      o.z[s] = x.z;
      o.px[s] = r1d * kv.x;
      o.py[s] = r1d * kv.y;
      o.pz[s] = r1d * kv.z;
      o.w[s] = S.w[slot];
      o.id[s] = child_id(id, seed, step, (uint32_t)k, kElectronChild);
      o.parent[s] = id;
      o.birth[s] = birth_code(step, (uint32_t)k);
      if (o.n_events) o.n_events[s] = 0u;
    });
    wave_append<QED_POSITRON>(a, pair, inst, cnt, [&](const qed_soa& o, long long s) {
      const double r1c = 1.0 - r1d;
      o.x[s] = x.x;
      o.y[s] = x.y;
      o.z[s] = x.z;
      o.px[s] = r1c * kv.x;
      o.py[s] = r1c * kv.y;
      o.pz[s] = r1c * kv.z;
      o.w[s] = S.w[slot];
      o.id[s] = child_id(id, seed, step, (uint32_t)k, kPositronChild);
      o.parent[s] = id;
      o.birth[s] = birth_code(step, (uint32_t)k);
      if (o.n_events) o.n_events[s] = 0u;
    });

    if (slot >= 0 && (pair || ++k == nsub)) {
      if (a.push_photons) {
        S.x[slot] = x.x;
        S.y[slot] = x.y;
        S.z[slot] = x.z;
      }
      if (pair) S.id[slot] = QED_ID_DEAD;
      slot = -1;
    }
  }
  flush_counters(a, cnt, true, 0, 0);
}

#undef LEPTON_COL

// ------------------------------------------------------------------------------------
template <bool MIXED, int FMODE>
static void launch_persistent(const StepArgs& a, LaunchShape lep, LaunchShape pho,
                              bool run_photons, hipStream_t s) {
  if (a.events[0]) (void)hipEventRecord(a.events[0], s);
  hipLaunchKernelGGL((lepton_kernel<MIXED, FMODE>), dim3(lep.grid), dim3(lep.block), 0, s, a);
  if (a.events[1]) (void)hipEventRecord(a.events[1], s);
  if (run_photons) {
    if (a.events[2]) (void)hipEventRecord(a.events[2], s);
    hipLaunchKernelGGL((photon_kernel<MIXED, FMODE>), dim3(pho.grid), dim3(pho.block), 0, s, a);
    if (a.events[3]) (void)hipEventRecord(a.events[3], s);
  }
}

static int field_mode(int kind) {
  if (kind == QED_FIELD_UNIFORM) return kFieldEB;
  if (kind == QED_FIELD_ROTATING_E) return kFieldE;
  return kFieldLocal;
}

hipError_t launch_step(const StepArgs& a, int precision, LaunchShape lep, LaunchShape pho,
                       bool run_photons, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(256), 0, s, a, run_photons ? 1 : 0);
  const int fm = field_mode(a.field.kind);
  if (precision == QED_MIXED) {
    if (fm == kFieldEB) launch_persistent<true, kFieldEB>(a, lep, pho, run_photons, s);
    else if (fm == kFieldE) launch_persistent<true, kFieldE>(a, lep, pho, run_photons, s);
    else launch_persistent<true, kFieldLocal>(a, lep, pho, run_photons, s);
  } else {
    if (fm == kFieldEB) launch_persistent<false, kFieldEB>(a, lep, pho, run_photons, s);
    else if (fm == kFieldE) launch_persistent<false, kFieldE>(a, lep, pho, run_photons, s);
    else launch_persistent<false, kFieldLocal>(a, lep, pho, run_photons, s);
  }
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <bool MIXED, int FMODE>
static int occupancy(bool photon, int block) {
  int nb = 0;
  const hipError_t e =
      photon ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, photon_kernel<MIXED, FMODE>, block, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lepton_kernel<MIXED, FMODE>, block, 0);
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

int step_blocks_per_cu(int precision, bool photon, int block) {
  // the rotating-field specialisation is the common one; the others use the same LDS
  return precision == QED_MIXED ? occupancy<true, kFieldE>(photon, block)
                                : occupancy<false, kFieldE>(photon, block);
}

}  // namespace qedk
