// qed_sort.hip -- reorders a species store by the grid cell of each particle.
//
// The field of a position-dependent workload is gathered from the eight nodes around each
// particle (Appendix A's CIC interpolation; Sec. IV.H notes that this interpolation is
// usually the costliest part of the particle update, and a PIC code keeps its particles cell
// by cell for it).  The stores here grow by appends in work order, so neighbouring slots
// soon hold particles far apart, and every lane of a wavefront gathers from its own lines.
// Sorting a store by cell puts the particles of one cell in neighbouring slots, so a
// wavefront's gathers share cache lines; children appended by a sorted parent store come out
// in runs from the same cells, so the order decays slowly and a sort every few steps keeps
// most of the gain.
//
// The key of a particle is the block of 2^shift x 2^shift x 2^shift cells that holds it
// (periodic wrap), numbered x fastest; shift is the smallest that leaves at most 65535
// blocks, so that the keys have 16 bits and the sort two 8-bit passes.  Removed photons get
// key 65535 and go to the end of their segment.  The sort is a stable LSD radix sort over
// each instance's live slots (ties keep their order), so the result is deterministic.
//
// Launches (all on the caller's stream, sizes fixed by the store's slot count so that a
// sequence can be captured):
//   sort_prep     one workgroup: live counts, slot prefix and tile prefix per instance;
//   sort_key      keys and the identity permutation;
//   per pass:  sort_hist (one workgroup per tile of kSortTile slots: digit counts),
//              scan_chunks, scan_sums, scan_apply (exclusive scan of the counts, ordered
//              instance, digit, tile), sort_scatter (stable ranks within the tile);
//   sort_gather   the columns, in sorted order, into the workspace;
//   sort_store    the workspace back into the segments.
#include "qed_internal.h"

namespace qedk {

namespace {

struct SortArgs {
  qed_soa s;
  qed_instance* inst;
  int n_inst, species;
  int n[3], shift;
  int nb[3];  // blocks per axis
  double inv_dx[3], origin[3];
  SortHdr* hdr;
  long long* gpref;  // [n_inst + 1] live-slot prefix
  long long* tpref;  // [n_inst + 1] tile prefix
  unsigned* key[2];
  unsigned* val[2];
  unsigned* cnt;     // [256 tiles]
  unsigned* sums;    // [chunks]
  unsigned char* cols;
  long long cap;     // slots (row length of the column copy)
};

__device__ __forceinline__ int find_instance(const long long* pref, int n, long long g) {
  int lo = 0, hi = n;  // pref[lo] <= g < pref[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pref[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) sort_prep_kernel(SortArgs a) {
  if (threadIdx.x != 0) return;
  long long g = 0, t = 0;
  a.gpref[0] = 0;
  a.tpref[0] = 0;
  for (int i = 0; i < a.n_inst; ++i) {
    long long c = a.inst[i].count[a.species];
    const long long cap = a.inst[i].capacity[a.species];
    c = c < 0 ? 0 : (c > cap ? cap : c);
    g += c;
    t += (c + kSortTile - 1) / kSortTile;
    a.gpref[i + 1] = g;
    a.tpref[i + 1] = t;
  }
  a.hdr->n = g;
  a.hdr->tiles = t;
}

__device__ __forceinline__ long long slot_of(const SortArgs& a, long long g) {
  const int i = find_instance(a.gpref, a.n_inst, g);
  return a.inst[i].base[a.species] + (g - a.gpref[i]);
}

__device__ __forceinline__ int axis_cell(double x, double org, double inv, int n) {
  if (!isfinite(x)) return -1;
  const CicAxis c = cic_axis((x - org) * inv, n);
  return c.i0;
}

__global__ void __launch_bounds__(256) sort_key_kernel(SortArgs a) {
  const long long N = a.hdr->n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
    const long long s = slot_of(a, g);
    unsigned key = kSortDeadKey;
    if (a.species != QED_PHOTON || a.s.id[s] != QED_ID_DEAD) {
      const int ix = axis_cell(a.s.x[s], a.origin[0], a.inv_dx[0], a.n[0]);
      const int iy = axis_cell(a.s.y[s], a.origin[1], a.inv_dx[1], a.n[1]);
      const int iz = axis_cell(a.s.z[s], a.origin[2], a.inv_dx[2], a.n[2]);
      if (ix < 0 || iy < 0 || iz < 0) {
        key = kSortDeadKey - 1;  // non-finite position: last of the live particles
      } else {
        key = (unsigned)((((long long)(iz >> a.shift) * a.nb[1]) + (iy >> a.shift)) * a.nb[0] +
                         (ix >> a.shift));
      }
    }
    a.key[0][g] = key;
    a.val[0][g] = (unsigned)g;
  }
}

// Tile t of the instance-ordered tile list: its instance and slots [g0, g1).
__device__ __forceinline__ bool tile_range(const SortArgs& a, long long t, int& inst,
                                           long long& g0, long long& g1, long long& nt) {
  if (t >= a.hdr->tiles) return false;
  inst = find_instance(a.tpref, a.n_inst, t);
  g0 = a.gpref[inst] + (t - a.tpref[inst]) * kSortTile;
  g1 = g0 + kSortTile < a.gpref[inst + 1] ? g0 + kSortTile : a.gpref[inst + 1];
  nt = a.tpref[inst + 1] - a.tpref[inst];
  return true;
}

// Position of (instance, digit, tile) in the scanned count array: instance-major, then
// digit, then the instance's tiles, so that the exclusive scan gives each element's slot.
__device__ __forceinline__ long long cnt_index(const SortArgs& a, int inst, int d, long long t,
                                               long long nt) {
  return a.tpref[inst] * 256 + (long long)d * nt + (t - a.tpref[inst]);
}

__global__ void __launch_bounds__(256) sort_hist_kernel(SortArgs a, int pass) {
  __shared__ unsigned h[256];
  int inst;
  long long g0, g1, nt;
  const long long t = blockIdx.x;
  if (!tile_range(a, t, inst, g0, g1, nt)) return;
  h[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned* key = a.key[pass & 1];
  const int sh = 8 * pass;
  for (long long g = g0 + threadIdx.x; g < g1; g += blockDim.x)
    atomicAdd(&h[(key[g] >> sh) & 255u], 1u);
  __syncthreads();
  a.cnt[cnt_index(a, inst, (int)threadIdx.x, t, nt)] = h[threadIdx.x];
}

// Exclusive scan of the count array in chunks of kScanChunk: per-chunk totals, a scan of the
// totals by one workgroup, then each chunk scanned with its base.
constexpr int kScanChunk = 4096;

__device__ unsigned block_exclusive_scan(unsigned v, unsigned* sw, unsigned& total) {
  // 256 threads: wavefront inclusive scans, then the four wavefront totals
  const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
  unsigned x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sw[w] = x;
  __syncthreads();
  unsigned base = 0;
  for (int i = 0; i < w; ++i) base += sw[i];
  total = sw[0] + sw[1] + sw[2] + sw[3];
  __syncthreads();
  return base + x - v;
}

__global__ void __launch_bounds__(256) scan_chunks_kernel(SortArgs a) {
  __shared__ unsigned sw[4];
  const long long M = a.hdr->tiles * 256;
  const long long c0 = (long long)blockIdx.x * kScanChunk;
  if (c0 >= M) return;
  unsigned s = 0;
  for (long long i = c0 + threadIdx.x; i < c0 + kScanChunk && i < M; i += blockDim.x)
    s += a.cnt[i];
  unsigned total;
  block_exclusive_scan(s, sw, total);
  if (threadIdx.x == 0) a.sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) scan_sums_kernel(SortArgs a) {
  __shared__ unsigned sw[4];
  const long long M = a.hdr->tiles * 256;
  const long long chunks = (M + kScanChunk - 1) / kScanChunk;
  unsigned carry = 0;
  for (long long b = 0; b < chunks; b += blockDim.x) {
    const long long i = b + threadIdx.x;
    const unsigned v = i < chunks ? a.sums[i] : 0u;
    unsigned total;
    const unsigned ex = block_exclusive_scan(v, sw, total);
    if (i < chunks) a.sums[i] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(256) scan_apply_kernel(SortArgs a) {
  __shared__ unsigned sw[4];
  const long long M = a.hdr->tiles * 256;
  const long long c0 = (long long)blockIdx.x * kScanChunk;
  if (c0 >= M) return;
  // each thread scans 16 consecutive entries; the threads' totals are scanned together
  constexpr int per = kScanChunk / 256;
  const long long i0 = c0 + (long long)threadIdx.x * per;
  unsigned v[per];
  unsigned s = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    v[k] = i0 + k < M ? a.cnt[i0 + k] : 0u;
    s += v[k];
  }
  unsigned total;
  unsigned run = a.sums[blockIdx.x] + block_exclusive_scan(s, sw, total);
#pragma unroll
  for (int k = 0; k < per; ++k) {
    if (i0 + k < M) a.cnt[i0 + k] = run;
    run += v[k];
  }
}

// Stable scatter of one tile: items are taken in 16 rounds of 256 (round r holds tile items
// r*256 .. r*256+255, in thread order), so the order of (round, thread) is the tile's order.
// An item's rank among the tile's items of its digit is the count so far of that digit, plus
// the items of that digit in the round's earlier wavefronts, plus those on lower lanes of its
// own wavefront (found with eight ballots, one per digit bit).
__global__ void __launch_bounds__(256) sort_scatter_kernel(SortArgs a, int pass) {
  __shared__ unsigned base[256];   // where the tile's next item of each digit goes
  __shared__ unsigned wcnt[4][256];
  int inst;
  long long g0, g1, nt;
  const long long t = blockIdx.x;
  if (!tile_range(a, t, inst, g0, g1, nt)) return;
  const int tid = (int)threadIdx.x, w = tid >> 6, lane = lane_id();
  base[tid] = a.cnt[cnt_index(a, inst, tid, t, nt)];
  for (int q = 0; q < 4; ++q) wcnt[q][tid] = 0u;
  __syncthreads();
  const unsigned* kin = a.key[pass & 1];
  const unsigned* vin = a.val[pass & 1];
  unsigned* kout = a.key[(pass + 1) & 1];
  unsigned* vout = a.val[(pass + 1) & 1];
  const int sh = 8 * pass;
  const uint64_t below = lanes_below();
  for (long long r0 = g0; r0 < g1; r0 += blockDim.x) {
    const long long g = r0 + tid;
    const bool has = g < g1;
    const unsigned k = has ? kin[g] : 0u;
    const unsigned v = has ? vin[g] : 0u;
    const unsigned d = (k >> sh) & 255u;
    uint64_t same = wave_ballot(has);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = wave_ballot(((d >> b) & 1u) != 0u);
      same &= ((d >> b) & 1u) ? m : ~m;
    }
    if (!has) same = 0;
    const unsigned in_wave = (unsigned)__popcll(same & below);
    // the lowest lane of each digit group records the group's size
    if (has && in_wave == 0u) wcnt[w][d] = (unsigned)__popcll(same);
    __syncthreads();
    if (has) {
      unsigned before = 0;
      for (int q = 0; q < w; ++q) before += wcnt[q][d];
      const unsigned pos = base[d] + before + in_wave;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    // advance the digit bases by the round's counts and clear them for the next round
    unsigned add = 0;
    for (int q = 0; q < 4; ++q) {
      add += wcnt[q][tid];
      wcnt[q][tid] = 0u;
    }
    base[tid] += add;
    __syncthreads();
  }
}

// Column copy in the workspace: 7 doubles, id and parent, birth and n_events per slot.
struct ColView {
  double* d[7];
  unsigned long long *id, *parent;
  unsigned *birth, *nev;
};
__device__ __forceinline__ ColView col_view(const SortArgs& a) {
  ColView c;
  const size_t col8 = ((size_t)a.cap * 8 + 255) & ~(size_t)255;
  const size_t col4 = ((size_t)a.cap * 4 + 255) & ~(size_t)255;
  unsigned char* p = a.cols;
  for (int k = 0; k < 7; ++k) {
    c.d[k] = reinterpret_cast<double*>(p);
    p += col8;
  }
  c.id = reinterpret_cast<unsigned long long*>(p);
  p += col8;
  c.parent = reinterpret_cast<unsigned long long*>(p);
  p += col8;
  c.birth = reinterpret_cast<unsigned*>(p);
  p += col4;
  c.nev = reinterpret_cast<unsigned*>(p);
  return c;
}

__global__ void __launch_bounds__(256) sort_gather_kernel(SortArgs a, int last) {
  const long long N = a.hdr->n;
  const ColView c = col_view(a);
  const unsigned* perm = a.val[last];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
    const long long s = slot_of(a, (long long)perm[g]);
    c.d[0][g] = a.s.x[s];
    c.d[1][g] = a.s.y[s];
    c.d[2][g] = a.s.z[s];
    c.d[3][g] = a.s.px[s];
    c.d[4][g] = a.s.py[s];
    c.d[5][g] = a.s.pz[s];
    c.d[6][g] = a.s.w[s];
    c.id[g] = a.s.id[s];
    c.parent[g] = a.s.parent[s];
    c.birth[g] = a.s.birth[s];
    if (a.s.n_events) c.nev[g] = a.s.n_events[s];
  }
}

__global__ void __launch_bounds__(256) sort_store_kernel(SortArgs a) {
  const long long N = a.hdr->n;
  const ColView c = col_view(a);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
    const long long s = slot_of(a, g);
    a.s.x[s] = c.d[0][g];
    a.s.y[s] = c.d[1][g];
    a.s.z[s] = c.d[2][g];
    a.s.px[s] = c.d[3][g];
    a.s.py[s] = c.d[4][g];
    a.s.pz[s] = c.d[5][g];
    a.s.w[s] = c.d[6][g];
    a.s.id[s] = c.id[g];
    a.s.parent[s] = c.parent[g];
    a.s.birth[s] = c.birth[g];
    if (a.s.n_events) a.s.n_events[s] = c.nev[g];
  }
}

}  // namespace

int sort_block_shift(const int n[3]) {
  for (int s = 0; s < 31; ++s) {
    long long b = 1;
    for (int d = 0; d < 3; ++d) b *= ((long long)n[d] + (1ll << s) - 1) >> s;
    if (b <= (long long)kSortDeadKey - 1) return s;
  }
  return 31;
}

hipError_t launch_sort_cells(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                             long long slots, const int n[3], const double dx[3],
                             const double origin[3], void* work, hipStream_t st) {
  const SortLayout L = SortLayout::make(n_inst, slots);
  unsigned char* w = static_cast<unsigned char*>(work);
  SortArgs a{};
  a.s = s;
  a.inst = inst;
  a.n_inst = n_inst;
  a.species = species;
  a.shift = sort_block_shift(n);
  for (int d = 0; d < 3; ++d) {
    a.n[d] = n[d];
    a.nb[d] = (int)(((long long)n[d] + (1ll << a.shift) - 1) >> a.shift);
    a.inv_dx[d] = 1.0 / dx[d];
    a.origin[d] = origin[d];
  }
  a.hdr = reinterpret_cast<SortHdr*>(w + L.hdr);
  a.gpref = reinterpret_cast<long long*>(w + L.gpref);
  a.tpref = reinterpret_cast<long long*>(w + L.tpref);
  for (int k = 0; k < 2; ++k) {
    a.key[k] = reinterpret_cast<unsigned*>(w + L.key[k]);
    a.val[k] = reinterpret_cast<unsigned*>(w + L.val[k]);
  }
  a.cnt = reinterpret_cast<unsigned*>(w + L.cnt);
  a.sums = reinterpret_cast<unsigned*>(w + L.sums);
  a.cols = w + L.cols;
  a.cap = L.cap;
  const long long grid = L.tiles_max;  // one workgroup per possible tile
  const long long chunks = (L.tiles_max * 256 + kScanChunk - 1) / kScanChunk;
  const long long stream_blocks = (slots + 255) / 256 < 8192 ? (slots + 255) / 256 : 8192;
  const unsigned sb = (unsigned)(stream_blocks > 0 ? stream_blocks : 1);
  hipLaunchKernelGGL(sort_prep_kernel, dim3(1), dim3(64), 0, st, a);
  hipLaunchKernelGGL(sort_key_kernel, dim3(sb), dim3(256), 0, st, a);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(sort_hist_kernel, dim3((unsigned)grid), dim3(256), 0, st, a, pass);
    hipLaunchKernelGGL(scan_chunks_kernel, dim3((unsigned)chunks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, st, a);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)chunks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)grid), dim3(256), 0, st, a, pass);
  }
  hipLaunchKernelGGL(sort_gather_kernel, dim3(sb), dim3(256), 0, st, a, 0);
  hipLaunchKernelGGL(sort_store_kernel, dim3(sb), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace qedk
