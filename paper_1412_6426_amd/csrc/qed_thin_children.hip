// qed_thin_children.hip -- the cap on the children one particle generates in one iteration
// (Sec. VII of Gonoskov et al., arXiv:1412.6426: their thinning also restricts how many
// super-particles a single particle or photon generates during one iteration).
//
// The children of the last step are the live particles of a species store whose birth code
// names that step and that have a parent; they are grouped by parent id, per instance.  A
// group of n > cap children keeps each with probability cap / n (a Philox draw keyed by the
// child's id), at least the one with the smallest draw, and its survivors take n / K of their
// weight (K survivors).  Everything else keeps its place; the store is compacted stably.
//
// Groups are found with an open-addressing hash table per instance (twice its children,
// linear probing, keys claimed by compare-and-swap), whose counts are sums of integers and
// so do not depend on the order of the threads.  Weight totals for the records are summed
// per range in a fixed tree order and then range by range.
//
// Only the tail of a segment from its first child on is touched after the first pass: the
// children of a step are appended to the stores, so the tail is about the last step's
// children, and the rest of the store keeps its place without being read or written.
//
// Launches on the caller's stream (grids fixed by the slot count, so the sequence can be
// captured):
//   prep     one workgroup: counts, counters cleared;
//   count    the children of each instance and its first one (birth codes first, the parent
//            and id only where the birth code names the step);
//   bases    one thread per instance: table bases and sizes, the tail;
//   clear    the tables;
//   insert   each child of the tail into its instance's table: entry per slot, group sizes,
//            groups, groups above the cap;
//   draw     in groups above the cap: survivors counted, smallest draw per group;
//   tie      in groups without survivors: the children with the smallest draw;
//   keep     keep flags, and per range of the tail the kept slots, children, their weight
//            before and after;
//   plan     one thread per instance: offsets of the ranges, the new count, the records;
//   scatter  kept rows of the tail, in order, into a column copy (survivors scaled);
//   back     the copy into the tail;
//   finish   the counts.
#include "qed_internal.h"

namespace qedk {

namespace {

constexpr int kTcThreads = 256;
constexpr unsigned kNoEntry = 0xFFFFFFFFu;

struct ChildHdr {
  long long tab;        // first entry of the instance's table
  long long size;       // its entries (2 x its children; 0 when frozen)
  unsigned long long groups, thinned;
  long long before;     // slots before (the count, at most the capacity)
  long long count;      // slots after
  unsigned long long children;  // children of the last step
  unsigned long long first;     // the slot of the first one (the tail starts there)
};
static_assert(sizeof(ChildHdr) == 64, "instance headers are 64 bytes");

struct ChildPart {
  long long kept;       // slots kept in the range
  long long children;   // children of the last step in the range
  long long kept_children;
  long long pad;
  double w_before, w_after;
  double pad2[2];
};
static_assert(sizeof(ChildPart) == 64, "range partials are 64 bytes");

struct TcArgs {
  qed_soa s;
  int species;
  qed_instance* inst;
  int n_inst, nb;
  long long slots;
  long long cap;        // children allowed per parent
  const long long* d_step;
  ChildHdr* hdr;        // [n_inst]
  ChildPart* part;      // [n_inst][nb]
  long long* off;       // [n_inst][nb]
  unsigned long long* tkey;
  unsigned* tn;         // children per entry
  unsigned* tk;         // survivors per entry
  unsigned* tk2;        // children with the smallest draw, where none survived
  unsigned long long* tmin;
  unsigned* ent;        // [slots] entry of each slot's group, kNoEntry for none
  unsigned char* keep;  // [slots]
  double* cd;           // [7][slots] x, y, z, px, py, pz, w
  unsigned long long* cu;  // [2][slots] id, parent
  unsigned* cb;         // [2][slots] birth, n_events
  qed_thin_children_record* rec;
};

__device__ __forceinline__ void range_of(long long n, int nb, int b, long long& lo,
                                         long long& hi) {
  const long long len = (n + nb - 1) / nb;
  lo = (long long)b * len;
  hi = lo + len < n ? lo + len : n;
  if (lo > n) lo = n;
}

// A child of the last step: born in it (birth >> 14 == the step counter), live, with a
// parent (the birth code first: most slots stop there).
__device__ __forceinline__ bool is_child(const TcArgs& a, long long s, uint32_t step) {
  if ((a.s.birth[s] >> 14) != step) return false;
  if (a.species == QED_PHOTON && a.s.id[s] == QED_ID_DEAD) return false;
  return a.s.parent[s] != QED_NO_PARENT;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The child's draw: the top 52 bits of its first two words (ordered as the uniform is).
__device__ __forceinline__ unsigned long long draw_bits(uint64_t id, uint64_t seed,
                                                        uint32_t step) {
  const uint4 o = draw_words(id, seed, step, 0u, kThinParent);
  return ((((unsigned long long)o.y) << 32) | o.x) >> 12;
}

__device__ __forceinline__ double bits_uniform(unsigned long long m) {
  return uniform64((uint32_t)(m << 12), (uint32_t)((m << 12) >> 32));
}

__global__ void __launch_bounds__(kTcThreads) tc_prep_kernel(TcArgs a) {
  for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) {
    const qed_instance& I = a.inst[i];
    ChildHdr h{};
    // a count beyond the segment (left by an append that dropped) covers only its capacity
    const long long n = I.count[a.species];
    h.before = n < 0 ? 0 : (n > I.capacity[a.species] ? I.capacity[a.species] : n);
    h.count = h.before;
    h.first = (unsigned long long)h.before;
    a.hdr[i] = h;
  }
}

__global__ void __launch_bounds__(kTcThreads) tc_count_kernel(TcArgs a) {
  const int i = blockIdx.y;
  const qed_instance& I = a.inst[i];
  if (I.frozen) return;
  long long lo, hi;
  range_of(a.hdr[i].before, a.nb, blockIdx.x, lo, hi);
  const uint32_t step = (uint32_t)*a.d_step;
  const long long base = I.base[a.species];
  unsigned long long n = 0, first = ~0ull;
  for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    if (!is_child(a, base + j, step)) continue;
    ++n;
    if ((unsigned long long)j < first) first = (unsigned long long)j;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    n += __shfl_xor(n, o, 64);
    const unsigned long long f = __shfl_xor(first, o, 64);
    first = f < first ? f : first;
  }
  if (lane_id() == 0 && n) {
    atomicAdd(&a.hdr[i].children, n);
    atomicMin(&a.hdr[i].first, first);
  }
}

// Table bases: twice each instance's children (so an empty entry is always found), in
// instance order; one thread does the prefix.
__global__ void __launch_bounds__(kTcThreads) tc_bases_kernel(TcArgs a) {
  if (threadIdx.x != 0) return;
  long long t = 0;
  for (int i = 0; i < a.n_inst; ++i) {
    ChildHdr& h = a.hdr[i];
    h.tab = t;
    h.size = 2 * (long long)h.children;
    t += h.size;
  }
}

// The tail of instance i: from its first child to its count.
__device__ __forceinline__ void tail_range(const ChildHdr& h, int nb, int b, long long& lo,
                                           long long& hi) {
  const long long t0 = (long long)h.first;
  range_of(h.before - t0, nb, b, lo, hi);
  lo += t0;
  hi += t0;
}

__global__ void __launch_bounds__(kTcThreads) tc_clear_kernel(TcArgs a) {
  const ChildHdr& h = a.hdr[blockIdx.y];
  long long lo, hi;
  range_of(h.size, a.nb, blockIdx.x, lo, hi);
  for (long long e = h.tab + lo + threadIdx.x; e < h.tab + hi; e += blockDim.x) {
    a.tkey[e] = QED_NO_PARENT;
    a.tn[e] = 0u;
    a.tk[e] = 0u;
    a.tk2[e] = 0u;
    a.tmin[e] = ~0ull;
  }
}

__global__ void __launch_bounds__(kTcThreads) tc_insert_kernel(TcArgs a) {
  const int i = blockIdx.y;
  const qed_instance& I = a.inst[i];
  const ChildHdr& h = a.hdr[i];
  long long lo, hi;
  tail_range(h, a.nb, blockIdx.x, lo, hi);
  const uint32_t step = (uint32_t)*a.d_step;
  const long long base = I.base[a.species];
  unsigned long long groups = 0, thinned = 0;
  for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    const long long s = base + j;
    if (h.size == 0 || !is_child(a, s, step)) {
      a.ent[s] = kNoEntry;
      continue;
    }
    const unsigned long long parent = a.s.parent[s];
    // the table holds twice the children: an empty entry is always found
    unsigned long long e = mix64(parent) % (unsigned long long)h.size;
    unsigned long long old;
    for (;;) {
      old = atomicCAS(&a.tkey[h.tab + e], QED_NO_PARENT, parent);
      if (old == QED_NO_PARENT || old == parent) break;
      e = e + 1 == (unsigned long long)h.size ? 0ull : e + 1;
    }
    a.ent[s] = (unsigned)e;
    const unsigned before = atomicAdd(&a.tn[h.tab + e], 1u);
    groups += old == QED_NO_PARENT;
    thinned += (long long)before == a.cap;
  }
  // one add per wavefront to the instance's counters
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    groups += __shfl_xor(groups, o, 64);
    thinned += __shfl_xor(thinned, o, 64);
  }
  if (lane_id() == 0) {
    if (groups) atomicAdd(&a.hdr[i].groups, groups);
    if (thinned) atomicAdd(&a.hdr[i].thinned, thinned);
  }
}

// Survival in a group of n > cap: u < cap / n.
__device__ __forceinline__ double survival(long long cap, unsigned n) {
  return (double)cap / (double)n;
}

__global__ void __launch_bounds__(kTcThreads) tc_draw_kernel(TcArgs a, int tie) {
  const int i = blockIdx.y;
  const qed_instance& I = a.inst[i];
  const ChildHdr& h = a.hdr[i];
  long long lo, hi;
  tail_range(h, a.nb, blockIdx.x, lo, hi);
  const uint32_t step = (uint32_t)*a.d_step;
  const long long base = I.base[a.species];
  for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    const long long s = base + j;
    const unsigned e = a.ent[s];
    if (e == kNoEntry) continue;
    const long long t = h.tab + e;
    const unsigned n = a.tn[t];
    if ((long long)n <= a.cap) continue;
    const unsigned long long m = draw_bits(a.s.id[s], I.seed, step);
    if (!tie) {
      if (bits_uniform(m) < survival(a.cap, n)) atomicAdd(&a.tk[t], 1u);
      atomicMin(&a.tmin[t], m);
    } else if (a.tk[t] == 0u && m == a.tmin[t]) {
      atomicAdd(&a.tk2[t], 1u);
    }
  }
}

// Is slot s kept, and by what factor is its weight scaled?
__device__ __forceinline__ bool kept_slot(const TcArgs& a, const qed_instance& I,
                                          const ChildHdr& h, long long s, uint32_t step,
                                          double& f) {
  f = 1.0;
  const unsigned e = a.ent[s];
  if (e == kNoEntry) return true;
  const long long t = h.tab + e;
  const unsigned n = a.tn[t];
  if ((long long)n <= a.cap) return true;
  const unsigned long long m = draw_bits(a.s.id[s], I.seed, step);
  const unsigned k = a.tk[t];
  const bool keep = bits_uniform(m) < survival(a.cap, n) || (k == 0u && m == a.tmin[t]);
  if (keep) f = (double)n / (double)(k ? k : a.tk2[t]);
  return keep;
}

// Workgroup sums in a fixed tree order (the wavefronts, then their totals in order).
template <typename T>
__device__ __forceinline__ T block_total(T v, T* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

__global__ void __launch_bounds__(kTcThreads) tc_keep_kernel(TcArgs a) {
  __shared__ long long sn[kTcThreads / 64];
  __shared__ double sw[kTcThreads / 64];
  const int i = blockIdx.y;
  const qed_instance& I = a.inst[i];
  const ChildHdr& h = a.hdr[i];
  long long lo, hi;
  tail_range(h, a.nb, blockIdx.x, lo, hi);
  const uint32_t step = (uint32_t)*a.d_step;
  const long long base = I.base[a.species];
  long long kept = 0, children = 0, kept_children = 0;
  double wb = 0.0, wa = 0.0;
  for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    const long long s = base + j;
    double f;
    const bool k = kept_slot(a, I, h, s, step, f);
    a.keep[s] = k ? 1 : 0;
    kept += k;
    if (a.ent[s] != kNoEntry) {
      const double w = a.s.w[s];
      ++children;
      wb += w;
      if (k) {
        ++kept_children;
        wa += w * f;
      }
    }
  }
  kept = block_total(kept, sn);
  children = block_total(children, sn);
  kept_children = block_total(kept_children, sn);
  wb = block_total(wb, sw);
  wa = block_total(wa, sw);
  if (threadIdx.x == 0) {
    ChildPart p{};
    p.kept = kept;
    p.children = children;
    p.kept_children = kept_children;
    p.w_before = wb;
    p.w_after = wa;
    a.part[(size_t)i * a.nb + blockIdx.x] = p;
  }
}

// One workgroup per instance: thread t takes ranges [t k, t k + k) (k = nb / threads, rounded
// up), sums them in order, the workgroup scans the thread totals, and the ranges' offsets
// follow; the record's sums go thread by thread in order.
__global__ void __launch_bounds__(kTcThreads) tc_plan_kernel(TcArgs a) {
  __shared__ long long skept[kTcThreads];
  __shared__ long long sch[kTcThreads], skc[kTcThreads];
  __shared__ double swb[kTcThreads], swa[kTcThreads];
  const int i = blockIdx.x;
  const ChildHdr& h = a.hdr[i];
  const int per = (a.nb + (int)blockDim.x - 1) / (int)blockDim.x;
  const int b0 = (int)threadIdx.x * per;
  const int b1 = b0 + per < a.nb ? b0 + per : a.nb;
  long long kept = 0, ch = 0, kc = 0;
  double wb = 0.0, wa = 0.0;
  for (int b = b0; b < b1; ++b) {
    const ChildPart& p = a.part[(size_t)i * a.nb + b];
    kept += p.kept;
    ch += p.children;
    kc += p.kept_children;
    wb += p.w_before;
    wa += p.w_after;
  }
  skept[threadIdx.x] = kept;
  sch[threadIdx.x] = ch;
  skc[threadIdx.x] = kc;
  swb[threadIdx.x] = wb;
  swa[threadIdx.x] = wa;
  __syncthreads();
  // exclusive prefix of the kept slots over the threads before this one
  long long o = 0;
  for (int u = 0; u < (int)threadIdx.x; ++u) o += skept[u];
  for (int b = b0; b < b1; ++b) {
    a.off[(size_t)i * a.nb + b] = o;
    o += a.part[(size_t)i * a.nb + b].kept;
  }
  if (threadIdx.x != 0) return;
  qed_thin_children_record r{};
  long long total = 0;
  for (int u = 0; u < (int)blockDim.x; ++u) {
    total += skept[u];
    r.children += sch[u];
    r.kept += skc[u];
    r.weight_before += swb[u];
    r.weight_after += swa[u];
  }
  total += (long long)h.first;
  if (a.inst[i].frozen) {
    r = qed_thin_children_record{};
    total = h.count;
  }
  r.groups = (long long)h.groups;
  r.groups_thinned = (long long)h.thinned;
  a.hdr[i].count = total;  // read by back and finish only, after this kernel
  a.rec[i] = r;
}

__global__ void __launch_bounds__(kTcThreads) tc_scatter_kernel(TcArgs a) {
  __shared__ unsigned wsum[kTcThreads / 64];
  const int i = blockIdx.y;
  const qed_instance& I = a.inst[i];
  if (I.frozen) return;
  const ChildHdr& h = a.hdr[i];
  long long lo, hi;
  // the tail before thinning (the plan kernel has set the count after it)
  tail_range(h, a.nb, blockIdx.x, lo, hi);
  const uint32_t step = (uint32_t)*a.d_step;
  const long long base = I.base[a.species];
  long long run = (long long)h.first + a.off[(size_t)i * a.nb + blockIdx.x];
  const uint64_t below = lanes_below();
  const int wv = (int)(threadIdx.x >> 6);
  const long long cap = a.slots;
  for (long long j0 = lo; j0 < hi; j0 += blockDim.x) {
    const long long j = j0 + threadIdx.x;
    const long long s = base + j;
    const bool has = j < hi;
    const bool k = has && a.keep[s];
    // exclusive rank within the chunk: within the wavefront, then the wavefronts before
    const uint64_t m = wave_ballot(k);
    __syncthreads();
    if (lane_id() == 0) wsum[wv] = (unsigned)__popcll(m);
    __syncthreads();
    unsigned before = 0, total = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      if (w < wv) before += wsum[w];
      total += wsum[w];
    }
    if (k) {
      double f = 1.0;
      if (a.ent[s] != kNoEntry) (void)kept_slot(a, I, h, s, step, f);
      const long long d = base + run + before + (unsigned)__popcll(m & below);
      a.cd[d] = a.s.x[s];
      a.cd[cap + d] = a.s.y[s];
      a.cd[2 * cap + d] = a.s.z[s];
      a.cd[3 * cap + d] = a.s.px[s];
      a.cd[4 * cap + d] = a.s.py[s];
      a.cd[5 * cap + d] = a.s.pz[s];
      a.cd[6 * cap + d] = a.s.w[s] * f;
      a.cu[d] = a.s.id[s];
      a.cu[cap + d] = a.s.parent[s];
      a.cb[d] = a.s.birth[s];
      a.cb[cap + d] = a.s.n_events ? a.s.n_events[s] : 0u;
    }
    run += total;
  }
}

__global__ void __launch_bounds__(kTcThreads) tc_back_kernel(TcArgs a) {
  const int i = blockIdx.y;
  const qed_instance& I = a.inst[i];
  if (I.frozen) return;
  const ChildHdr& h = a.hdr[i];
  const long long t0 = (long long)h.first;
  long long lo, hi;
  range_of(h.count - t0, a.nb, blockIdx.x, lo, hi);
  lo += t0;
  hi += t0;
  const long long base = I.base[a.species];
  const long long cap = a.slots;
  for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    const long long d = base + j;
    a.s.x[d] = a.cd[d];
    a.s.y[d] = a.cd[cap + d];
    a.s.z[d] = a.cd[2 * cap + d];
    a.s.px[d] = a.cd[3 * cap + d];
    a.s.py[d] = a.cd[4 * cap + d];
    a.s.pz[d] = a.cd[5 * cap + d];
    a.s.w[d] = a.cd[6 * cap + d];
    a.s.id[d] = a.cu[d];
    a.s.parent[d] = a.cu[cap + d];
    a.s.birth[d] = a.cb[d];
    if (a.s.n_events) a.s.n_events[d] = a.cb[cap + d];
  }
}

__global__ void __launch_bounds__(kTcThreads) tc_finish_kernel(TcArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_inst || a.inst[i].frozen) return;
  a.inst[i].count[a.species] = a.hdr[i].count;
}

}  // namespace

ThinChildrenLayout ThinChildrenLayout::make(int n_inst, long long slots) {
  ThinChildrenLayout L{};
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t n = (size_t)(slots > 0 ? slots : 1);
  L.nb = ThinLayout::ranges(n_inst, slots);
  const size_t nb = (size_t)n_inst * L.nb;
  L.hdr = take(64 * (size_t)n_inst);
  L.part = take(64 * nb);
  L.off = take(8 * nb);
  L.tkey = take(8 * 2 * n);
  L.tn = take(4 * 2 * n);
  L.tk = take(4 * 2 * n);
  L.tk2 = take(4 * 2 * n);
  L.tmin = take(8 * 2 * n);
  L.ent = take(4 * n);
  L.keep = take(n);
  L.cd = take(8 * 7 * n);
  L.cu = take(8 * 2 * n);
  L.cb = take(4 * 2 * n);
  L.total = off;
  return L;
}

hipError_t launch_thin_children(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                                long long slots, long long max_per_parent,
                                const long long* d_step, qed_thin_children_record* rec,
                                void* work, hipStream_t st) {
  const ThinChildrenLayout L = ThinChildrenLayout::make(n_inst, slots);
  uint8_t* w = static_cast<uint8_t*>(work);
  TcArgs a{};
  a.s = s;
  a.species = species;
  a.inst = inst;
  a.n_inst = n_inst;
  a.nb = L.nb;
  a.slots = slots > 0 ? slots : 1;
  a.cap = max_per_parent;
  a.d_step = d_step;
  a.hdr = reinterpret_cast<ChildHdr*>(w + L.hdr);
  a.part = reinterpret_cast<ChildPart*>(w + L.part);
  a.off = reinterpret_cast<long long*>(w + L.off);
  a.tkey = reinterpret_cast<unsigned long long*>(w + L.tkey);
  a.tn = reinterpret_cast<unsigned*>(w + L.tn);
  a.tk = reinterpret_cast<unsigned*>(w + L.tk);
  a.tk2 = reinterpret_cast<unsigned*>(w + L.tk2);
  a.tmin = reinterpret_cast<unsigned long long*>(w + L.tmin);
  a.ent = reinterpret_cast<unsigned*>(w + L.ent);
  a.keep = reinterpret_cast<unsigned char*>(w + L.keep);
  a.cd = reinterpret_cast<double*>(w + L.cd);
  a.cu = reinterpret_cast<unsigned long long*>(w + L.cu);
  a.cb = reinterpret_cast<unsigned*>(w + L.cb);
  a.rec = rec;
  const dim3 ranges(L.nb, n_inst);
  const int per_inst = (n_inst + kTcThreads - 1) / kTcThreads;
  hipLaunchKernelGGL(tc_prep_kernel, dim3(1), dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_count_kernel, ranges, dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_bases_kernel, dim3(1), dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_clear_kernel, ranges, dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_insert_kernel, ranges, dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_draw_kernel, ranges, dim3(kTcThreads), 0, st, a, 0);
  hipLaunchKernelGGL(tc_draw_kernel, ranges, dim3(kTcThreads), 0, st, a, 1);
  hipLaunchKernelGGL(tc_keep_kernel, ranges, dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_plan_kernel, dim3(n_inst), dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_scatter_kernel, ranges, dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_back_kernel, ranges, dim3(kTcThreads), 0, st, a);
  hipLaunchKernelGGL(tc_finish_kernel, dim3(per_inst), dim3(kTcThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace qedk
