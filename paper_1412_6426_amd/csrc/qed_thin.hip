// qed_thin.hip -- thinning by global even redistribution (Sec. VI of Gonoskov et al.,
// arXiv:1412.6426): in every instance whose store of one species holds more than `trigger`
// slots, each live particle survives with probability q = target / live (a Philox draw keyed
// by its id), and the survivors' weights are multiplied by sum f / (sum f - f_r), the total
// live weight over the surviving weight, so charge (total weight) is conserved.
//
// Seven launches on the caller's stream, each a grid of (nb, n_instances) or one workgroup
// per instance (nb ranges per instance, about 8192 slots each of the mean segment, at most
// kThinBlocks); workgroup b of an instance owns a contiguous range of its segment:
//   count  live particles and their weight per range;
//   plan   sums (in a fixed order), q, whether to thin;
//   keep   survivors and their weight per range;
//   plan2  K survivors in total, the factor, and per range the holes below K (removed or
//          dead slots) and the survivors at or above K, as prefix offsets;
//   holes  list the positions of the holes below K; survivors below K get the factor;
//   move   the i-th survivor at or above K moves into the i-th hole, scaled;
//   count  the instance's count becomes K.
// Sources lie at or above K and destinations below it, one survivor per hole, so the moves
// never overlap, and nothing below K is read while the moves write there.  The store order
// after thinning is deterministic (it differs from a stable compaction; the set of
// survivors does not).
#include "qed_internal.h"

namespace qedk {

namespace {

constexpr int kThinThreads = 256;
static_assert(kThinBlocks % kThinThreads == 0, "plan kernels give each thread whole ranges");

struct ThinPlan {
  long long n;      // slots of the segment when thinning started
  long long live;   // live particles
  long long kept;   // survivors (K)
  double q;         // survival probability
  double w_live, w_kept, factor;
  int thin;         // 1: thin this instance
  int pad;
};
static_assert(sizeof(ThinPlan) == 64, "plan records are 64 bytes in the workspace");

struct ThinArgs {
  qed_soa s;
  int species;
  qed_instance* inst;
  int n_inst;
  long long trigger, target;
  int nb;                      // ranges per instance, 1..kThinBlocks
  const long long* d_step;
  ThinPlan* plan;              // [n_inst]
  long long* part_n;           // [n_inst][nb] live, then kept
  double* part_w;              // [n_inst][nb] live weight, then kept weight
  long long* hole_off;         // [n_inst][nb]
  long long* surv_off;         // [n_inst][nb]
  unsigned int* holes;         // [slots]: hole positions, relative to the segment base
  qed_thin_record* rec;        // [n_inst]
};

__device__ __forceinline__ void range_of(long long n, int nb, int b, long long& lo,
                                         long long& hi) {
  const long long len = (n + nb - 1) / nb;
  lo = (long long)b * len;
  hi = lo + len < n ? lo + len : n;
  if (lo > n) lo = n;
}

__device__ __forceinline__ bool is_live(const ThinArgs& a, long long s) {
  return a.species != QED_PHOTON || a.s.id[s] != QED_ID_DEAD;
}

__device__ __forceinline__ bool keeps(const ThinArgs& a, long long s, uint64_t seed,
                                      uint32_t step, double q) {
  const uint64_t id = a.s.id[s];
  if (a.species == QED_PHOTON && id == QED_ID_DEAD) return false;
  const uint4 o = draw_words(id, seed, step, 0u, kThin);
  return uniform64(o.x, o.y) < q;
}

// Workgroup sums: a fixed tree order (waves, then the workgroup's wave totals in order).
__device__ __forceinline__ void block_sum(long long& n, double& w, long long* sn, double* sw) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    n += __shfl_xor(n, o, 64);
    w += __shfl_xor(w, o, 64);
  }
  const int wv = (int)(threadIdx.x >> 6);
  if (lane_id() == 0) {
    sn[wv] = n;
    sw[wv] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tn = 0;
    double tw = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      tn += sn[i];
      tw += sw[i];
    }
    n = tn;
    w = tw;
  }
}

__global__ void __launch_bounds__(kThinThreads) thin_count_kernel(ThinArgs a) {
  __shared__ long long sn[kThinThreads / 64];
  __shared__ double sw[kThinThreads / 64];
  const int i = blockIdx.y, b = blockIdx.x;
  const qed_instance& I = a.inst[i];
  // a count beyond the segment (left by an append that dropped) covers only its capacity
  long long n = I.count[a.species];
  n = n < 0 ? 0 : (n > I.capacity[a.species] ? I.capacity[a.species] : n);
  long long live = 0;
  double w = 0.0;
  if (n > a.trigger) {
    long long lo, hi;
    range_of(n, a.nb, b, lo, hi);
    const long long base = I.base[a.species];
    for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x)
      if (is_live(a, base + j)) {
        ++live;
        w += a.s.w[base + j];
      }
  }
  block_sum(live, w, sn, sw);
  if (threadIdx.x == 0) {
    a.part_n[(size_t)i * a.nb + b] = live;
    a.part_w[(size_t)i * a.nb + b] = w;
    if (b == 0) a.plan[i].n = n;
  }
}

// Sum of an instance's per-range partials in a fixed order: thread t takes ranges t, t + 256,
// ... in turn, then the workgroup tree.  Result in thread 0.
__device__ __forceinline__ void sum_partials(const ThinArgs& a, int i, long long& n, double& w,
                                             long long* sn, double* sw) {
  n = 0;
  w = 0.0;
  for (int b = threadIdx.x; b < a.nb; b += blockDim.x) {
    n += a.part_n[(size_t)i * a.nb + b];
    w += a.part_w[(size_t)i * a.nb + b];
  }
  block_sum(n, w, sn, sw);
}

__global__ void __launch_bounds__(kThinThreads) thin_plan_kernel(ThinArgs a) {
  __shared__ long long sn[kThinThreads / 64];
  __shared__ double sw[kThinThreads / 64];
  const int i = blockIdx.x;
  long long live;
  double w;
  sum_partials(a, i, live, w, sn, sw);
  if (threadIdx.x != 0) return;
  ThinPlan& P = a.plan[i];
  P.live = live;
  P.w_live = w;
  P.thin = (P.n > a.trigger && a.target < live) ? 1 : 0;
  P.q = P.thin ? (double)a.target / (double)live : 1.0;
  P.kept = live;
  P.w_kept = w;
  P.factor = 1.0;
}

__global__ void __launch_bounds__(kThinThreads) thin_keep_kernel(ThinArgs a) {
  __shared__ long long sn[kThinThreads / 64];
  __shared__ double sw[kThinThreads / 64];
  const int i = blockIdx.y, b = blockIdx.x;
  const ThinPlan& P = a.plan[i];
  if (!P.thin) return;
  const qed_instance& I = a.inst[i];
  const long long base = I.base[a.species];
  const uint64_t seed = I.seed;
  const uint32_t step = (uint32_t)*a.d_step;
  long long lo, hi;
  range_of(P.n, a.nb, b, lo, hi);
  long long kept = 0;
  double w = 0.0;
  for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x)
    if (keeps(a, base + j, seed, step, P.q)) {
      ++kept;
      w += a.s.w[base + j];
    }
  block_sum(kept, w, sn, sw);
  if (threadIdx.x == 0) {
    a.part_n[(size_t)i * a.nb + b] = kept;
    a.part_w[(size_t)i * a.nb + b] = w;
  }
}

// Exclusive prefix over the workgroup's threads of v (thread order), and the total.
__device__ __forceinline__ long long block_excl_scan(long long v, long long* sn,
                                                     long long& total) {
  long long x = v;
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  const int wv = (int)(threadIdx.x >> 6);
  if (lane == 63) sn[wv] = x;
  __syncthreads();
  long long before = 0;
  total = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    if (k < wv) before += sn[k];
    total += sn[k];
  }
  __syncthreads();
  return before + x - v;
}

// One workgroup per instance.  Survivors in [lo, K) of the range that straddles K are
// counted again here (the keep pass counted whole ranges).
__global__ void __launch_bounds__(kThinThreads) thin_plan2_kernel(ThinArgs a) {
  __shared__ long long sn[kThinThreads / 64];
  __shared__ double sw[kThinThreads / 64];
  __shared__ long long s_k, s_below;
  const int i = blockIdx.x;
  ThinPlan& P = a.plan[i];
  if (!P.thin) return;
  long long k;
  double w;
  sum_partials(a, i, k, w, sn, sw);
  if (threadIdx.x == 0) {
    P.kept = k;
    P.w_kept = w;
    P.factor = k > 0 ? P.w_live / w : 0.0;
    s_k = k;
  }
  __syncthreads();
  const long long K = s_k;
  const qed_instance& I = a.inst[i];
  const long long base = I.base[a.species];
  const uint64_t seed = I.seed;
  const uint32_t step = (uint32_t)*a.d_step;
  // the range containing K strictly inside it: survivors below K
  const long long len = (P.n + a.nb - 1) / a.nb;
  const int bk = len > 0 ? (int)(K / len) : 0;
  long long lo_k, hi_k;
  range_of(P.n, a.nb, bk, lo_k, hi_k);
  const bool straddle = len > 0 && bk < a.nb && lo_k < K && K < hi_k;
  long long below = 0;
  double unused = 0.0;
  if (straddle)
    for (long long j = lo_k + threadIdx.x; j < K; j += blockDim.x)
      below += keeps(a, base + j, seed, step, P.q) ? 1 : 0;
  block_sum(below, unused, sn, sw);
  if (threadIdx.x == 0) s_below = below;
  __syncthreads();
  below = s_below;
  // holes below K and survivors at or above K per range; thread t owns a contiguous group
  // of ranges, so a thread-order scan of the group sums gives range-order prefixes
  constexpr int kMaxPer = kThinBlocks / kThinThreads;
  const int per = (a.nb + kThinThreads - 1) / kThinThreads;
  long long hb[kMaxPer], sb[kMaxPer], hsum = 0, ssum = 0;
#pragma unroll
  for (int m = 0; m < kMaxPer; ++m) {
    const int b = (int)threadIdx.x * per + m;
    hb[m] = sb[m] = 0;
    if (m >= per || b >= a.nb) continue;
    long long lo, hi;
    range_of(P.n, a.nb, b, lo, hi);
    const long long kb = a.part_n[(size_t)i * a.nb + b];
    if (hi <= K) {
      hb[m] = (hi - lo) - kb;
      sb[m] = 0;
    } else if (lo >= K) {
      hb[m] = 0;
      sb[m] = kb;
    } else {
      hb[m] = (K - lo) - below;
      sb[m] = kb - below;
    }
    hsum += hb[m];
    ssum += sb[m];
  }
  long long tot;
  long long h = block_excl_scan(hsum, sn, tot);
  long long sv = block_excl_scan(ssum, sn, tot);
#pragma unroll
  for (int m = 0; m < kMaxPer; ++m) {
    const int b = (int)threadIdx.x * per + m;
    if (m >= per || b >= a.nb) continue;
    a.hole_off[(size_t)i * a.nb + b] = h;
    a.surv_off[(size_t)i * a.nb + b] = sv;
    h += hb[m];
    sv += sb[m];
  }
}

// Rank of each flagged thread among the workgroup's flagged threads, and their number.
__device__ __forceinline__ int block_rank(bool flag, int* swc, int& total) {
  const uint64_t m = wave_ballot(flag);
  const int wv = (int)(threadIdx.x >> 6);
  if (lane_id() == 0) swc[wv] = __popcll(m);
  __syncthreads();
  int before = 0;
  total = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    if (k < wv) before += swc[k];
    total += swc[k];
  }
  __syncthreads();
  return before + __popcll(m & lanes_below());
}

__global__ void __launch_bounds__(kThinThreads) thin_holes_kernel(ThinArgs a) {
  __shared__ int swc[kThinThreads / 64];
  const int i = blockIdx.y, b = blockIdx.x;
  const ThinPlan& P = a.plan[i];
  if (!P.thin) return;
  const qed_instance& I = a.inst[i];
  const long long base = I.base[a.species];
  const uint64_t seed = I.seed;
  const uint32_t step = (uint32_t)*a.d_step;
  long long lo, hi;
  range_of(P.n, a.nb, b, lo, hi);
  if (hi > P.kept) hi = P.kept;
  long long off = a.hole_off[(size_t)i * a.nb + b];
  const double f = P.factor;
  for (long long j0 = lo; j0 < hi; j0 += blockDim.x) {
    const long long j = j0 + threadIdx.x;
    const bool in = j < hi;
    const bool keep = in && keeps(a, base + j, seed, step, P.q);
    const bool hole = in && !keep;
    int total;
    const int r = block_rank(hole, swc, total);
    if (hole) a.holes[base + off + r] = (unsigned int)j;
    if (keep) a.s.w[base + j] *= f;
    off += total;
  }
}

__global__ void __launch_bounds__(kThinThreads) thin_move_kernel(ThinArgs a) {
  __shared__ int swc[kThinThreads / 64];
  const int i = blockIdx.y, b = blockIdx.x;
  const ThinPlan& P = a.plan[i];
  qed_instance& I = a.inst[i];
  if (b == 0 && threadIdx.x == 0) {
    qed_thin_record r{};
    r.live_before = P.live;
    r.kept = P.kept;
    r.weight_before = P.w_live;
    r.factor = P.factor;
    r.thinned = P.thin;
    a.rec[i] = r;
  }
  if (!P.thin) return;
  const long long base = I.base[a.species];
  const uint64_t seed = I.seed;
  const uint32_t step = (uint32_t)*a.d_step;
  const long long K = P.kept;
  const double f = P.factor;
  const qed_soa& S = a.s;
  long long lo, hi;
  range_of(P.n, a.nb, b, lo, hi);
  if (lo < K) lo = K;  // only the range at or above K is read here
  long long off = a.surv_off[(size_t)i * a.nb + b];
  for (long long j0 = lo; j0 < hi; j0 += blockDim.x) {
    const long long j = j0 + threadIdx.x;
    const bool mover = j < hi && keeps(a, base + j, seed, step, P.q);
    int total;
    const int r = block_rank(mover, swc, total);
    if (mover) {
      const long long src = base + j;
      const long long dst = base + (long long)a.holes[base + off + r];
      S.x[dst] = S.x[src];
      S.y[dst] = S.y[src];
      S.z[dst] = S.z[src];
      S.px[dst] = S.px[src];
      S.py[dst] = S.py[src];
      S.pz[dst] = S.pz[src];
      S.w[dst] = S.w[src] * f;
      S.id[dst] = S.id[src];
      S.parent[dst] = S.parent[src];
      S.birth[dst] = S.birth[src];
      if (S.n_events) S.n_events[dst] = S.n_events[src];
    }
    off += total;
  }
}

__global__ void thin_count_set_kernel(ThinArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_inst) return;
  if (a.plan[i].thin) a.inst[i].count[a.species] = a.plan[i].kept;
}

}  // namespace

hipError_t launch_thin(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                       long long slots, long long trigger, long long target,
                       const long long* d_step, qed_thin_record* rec, void* work,
                       hipStream_t st) {
  const ThinLayout L = ThinLayout::make(n_inst, slots);
  uint8_t* w = static_cast<uint8_t*>(work);
  ThinArgs a;
  a.s = s;
  a.species = species;
  a.inst = inst;
  a.n_inst = n_inst;
  a.trigger = trigger;
  a.target = target;
  a.nb = L.nb;
  a.d_step = d_step;
  a.plan = reinterpret_cast<ThinPlan*>(w + L.plan);
  a.part_n = reinterpret_cast<long long*>(w + L.part_n);
  a.part_w = reinterpret_cast<double*>(w + L.part_w);
  a.hole_off = reinterpret_cast<long long*>(w + L.hole_off);
  a.surv_off = reinterpret_cast<long long*>(w + L.surv_off);
  a.holes = reinterpret_cast<unsigned int*>(w + L.holes);
  a.rec = rec;
  const dim3 grid(a.nb, n_inst);
  hipLaunchKernelGGL(thin_count_kernel, grid, dim3(kThinThreads), 0, st, a);
  hipLaunchKernelGGL(thin_plan_kernel, dim3(n_inst), dim3(kThinThreads), 0, st, a);
  hipLaunchKernelGGL(thin_keep_kernel, grid, dim3(kThinThreads), 0, st, a);
  hipLaunchKernelGGL(thin_plan2_kernel, dim3(n_inst), dim3(kThinThreads), 0, st, a);
  hipLaunchKernelGGL(thin_holes_kernel, grid, dim3(kThinThreads), 0, st, a);
  hipLaunchKernelGGL(thin_move_kernel, grid, dim3(kThinThreads), 0, st, a);
  hipLaunchKernelGGL(thin_count_set_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace qedk
