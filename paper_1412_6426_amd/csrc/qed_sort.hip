// qed_sort.hip -- reorders a species store by the grid cell of each particle.
//
// The field of a position-dependent workload is gathered from the eight nodes around each
// particle (Appendix A's CIC interpolation; Sec. IV.H notes that this interpolation is
// usually the costliest part of the particle update, and a PIC code keeps its particles cell
// by cell for it).  The stores here grow by appends in work order, so neighbouring slots
// soon hold particles far apart, and every lane of a wavefront gathers from its own lines.
// Sorting a store by cell puts the particles of one cell in neighbouring slots, so a
// wavefront's gathers share cache lines.  Children are appended in the order of their
// parents, so a sorted lepton store also hands its photons out in runs from the same cells.
//
// The key of a particle is the block of 2^shift x 2^shift x 2^shift cells that holds it
// (periodic wrap), numbered x fastest; shift is the smallest that leaves at most 2^24 - 2
// blocks (0 up to 16 million cells, 1 for 256^3), and the keys take the fewest 8-bit digits
// that hold every block plus two reserved keys: removed photons get the largest (they go to
// the end of their segment), particles with a non-finite position the one below it.  The
// sort is a stable LSD radix sort over each instance's live slots (ties keep their order),
// so the result is deterministic.
//
// Every kernel but the scans works tile by tile (kSortTile slots of one instance, one
// workgroup each), so a tile's instance and slot base are found once; each thread loads
// all of its items of a round before it stores any, which keeps many loads in flight.
//
// Launches (all on the caller's stream, sizes fixed by the store's slot count so that a
// sequence can be captured):
//   sort_prep     one workgroup: live counts (none for a frozen instance), slot prefix and
//                 tile prefix per instance;
//   sort_key      keys and the identity permutation;
//   per pass:  sort_hist (digit counts per tile), scan_chunks, scan_sums, scan_apply
//              (exclusive scan of the counts, ordered instance, digit, tile), sort_scatter
//              (stable ranks within the tile);
//   sort_gather   the columns, in sorted order, into the workspace;
//   sort_store    the workspace back into the segments.
#include "qed_internal.h"

namespace qedk {

namespace {

struct SortArgs {
  qed_soa s;
  qed_instance* inst;
  int n_inst, species;
  int n[3], shift, passes;
  unsigned dead;
  long long nb[3];  // blocks per axis
  double dx[3], origin[3];
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

constexpr int kSortThreads = 256;
constexpr int kPerThread = kSortTile / kSortThreads;  // items of one thread in a tile
constexpr int kBatch = 4;                             // items a thread loads before storing

__device__ __forceinline__ int find_instance(const long long* pref, int n, long long g) {
  int lo = 0, hi = n;  // pref[lo] <= g < pref[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pref[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(64) sort_prep_kernel(SortArgs a) {
  if (threadIdx.x != 0) return;
  long long g = 0, t = 0;
  a.gpref[0] = 0;
  a.tpref[0] = 0;
  for (int i = 0; i < a.n_inst; ++i) {
    long long c = a.inst[i].count[a.species];
    const long long cap = a.inst[i].capacity[a.species];
    c = c < 0 ? 0 : (c > cap ? cap : c);
    if (a.inst[i].frozen) c = 0;  // a frozen instance no longer steps: left as it is
    g += c;
    t += (c + kSortTile - 1) / kSortTile;
    a.gpref[i + 1] = g;
    a.tpref[i + 1] = t;
  }
  a.hdr->n = g;
  a.hdr->tiles = t;
}

// Tile t of the instance-ordered tile list: its instance, items [g0, g1) of the live-slot
// index space, the instance's tile count, and sbase such that item g sits in slot sbase + g.
struct Tile {
  int inst;
  long long g0, g1, nt, sbase;
};
__device__ __forceinline__ bool tile_of(const SortArgs& a, long long t, Tile& T) {
  if (t >= a.hdr->tiles) return false;
  T.inst = find_instance(a.tpref, a.n_inst, t);
  T.g0 = a.gpref[T.inst] + (t - a.tpref[T.inst]) * kSortTile;
  T.g1 = T.g0 + kSortTile < a.gpref[T.inst + 1] ? T.g0 + kSortTile : a.gpref[T.inst + 1];
  T.nt = a.tpref[T.inst + 1] - a.tpref[T.inst];
  T.sbase = a.inst[T.inst].base[a.species] - a.gpref[T.inst];
  return true;
}

// The block of one coordinate: cell floor((x - origin) / dx), wrapped into [0, n), >> shift
// (a division, not a product with 1/dx, so that a particle on a cell face falls in the cell
// the definition gives).
__device__ __forceinline__ long long axis_block(double x, double org, double dx, int n,
                                                int shift) {
  if (!isfinite(x)) return -1;
  const CicAxis c = cic_axis((x - org) / dx, n);
  return (long long)(c.i0 >> shift);
}

__global__ void __launch_bounds__(kSortThreads) sort_key_kernel(SortArgs a) {
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  const bool photons = a.species == QED_PHOTON;
  for (long long r0 = T.g0 + threadIdx.x; r0 < T.g1; r0 += kBatch * kSortThreads) {
    double x[kBatch], y[kBatch], z[kBatch];
    uint64_t id[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const long long g = r0 + (long long)u * kSortThreads;
      if (g < T.g1) {
        const long long s = T.sbase + g;
        id[u] = photons ? a.s.id[s] : 0ull;
        x[u] = a.s.x[s];
        y[u] = a.s.y[s];
        z[u] = a.s.z[s];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const long long g = r0 + (long long)u * kSortThreads;
      if (g >= T.g1) break;
      unsigned key = a.dead;
      if (!photons || id[u] != QED_ID_DEAD) {
        const long long bx = axis_block(x[u], a.origin[0], a.dx[0], a.n[0], a.shift);
        const long long by = axis_block(y[u], a.origin[1], a.dx[1], a.n[1], a.shift);
        const long long bz = axis_block(z[u], a.origin[2], a.dx[2], a.n[2], a.shift);
        if (bx < 0 || by < 0 || bz < 0) key = a.dead - 1u;  // last of the live particles
        else key = (unsigned)((bz * a.nb[1] + by) * a.nb[0] + bx);
      }
      a.key[0][g] = key;
      a.val[0][g] = (unsigned)g;
    }
  }
}

// Position of (instance, digit, tile) in the scanned count array: instance-major, then
// digit, then the instance's tiles, so that the exclusive scan gives each element's slot.
__device__ __forceinline__ long long cnt_index(const SortArgs& a, const Tile& T, int d,
                                               long long t) {
  return a.tpref[T.inst] * 256 + (long long)d * T.nt + (t - a.tpref[T.inst]);
}

// Lanes of this wavefront holding the same digit as this lane (eight ballots, one per bit).
__device__ __forceinline__ uint64_t same_digit(unsigned d, bool has) {
  uint64_t same = wave_ballot(has);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t m = wave_ballot(((d >> b) & 1u) != 0u);
    same &= ((d >> b) & 1u) ? m : ~m;
  }
  return has ? same : 0ull;
}

// A thread's items of its tile: item i is tile item i * 256 + thread (so that the order of
// (i, thread) is the tile's order).
__device__ __forceinline__ void load_tile_words(const unsigned* src, const Tile& T,
                                                unsigned (&k)[kPerThread]) {
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long long g = T.g0 + (long long)i * kSortThreads + threadIdx.x;
    k[i] = g < T.g1 ? src[g] : 0u;
  }
}

__global__ void __launch_bounds__(kSortThreads) sort_hist_kernel(SortArgs a, int pass) {
  __shared__ unsigned h[256];
  Tile T;
  const long long t = blockIdx.x;
  if (!tile_of(a, t, T)) return;
  h[threadIdx.x] = 0u;
  unsigned k[kPerThread];
  load_tile_words(a.key[pass & 1], T, k);
  __syncthreads();
  const int sh = 8 * pass;
  const uint64_t below = lanes_below();
  // one LDS add per digit group of a wavefront (sorted keys give few groups)
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const bool has = T.g0 + (long long)i * kSortThreads + threadIdx.x < T.g1;
    const unsigned d = (k[i] >> sh) & 255u;
    const uint64_t same = same_digit(d, has);
    if (has && (same & below) == 0ull) atomicAdd(&h[d], (unsigned)__popcll(same));
  }
  __syncthreads();
  a.cnt[cnt_index(a, T, (int)threadIdx.x, t)] = h[threadIdx.x];
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

__global__ void __launch_bounds__(kSortThreads) scan_chunks_kernel(SortArgs a) {
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

__global__ void __launch_bounds__(kSortThreads) scan_sums_kernel(SortArgs a) {
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

__global__ void __launch_bounds__(kSortThreads) scan_apply_kernel(SortArgs a) {
  __shared__ unsigned sw[4];
  const long long M = a.hdr->tiles * 256;
  const long long c0 = (long long)blockIdx.x * kScanChunk;
  if (c0 >= M) return;
  // each thread scans 16 consecutive entries; the threads' totals are scanned together
  constexpr int per = kScanChunk / kSortThreads;
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

// Stable scatter of one tile: the thread's 16 items (keys and indices) are loaded first;
// round i holds tile items i*256 .. i*256+255 in thread order.  An item's rank among the
// tile's items of its digit is the count so far of that digit, plus the items of that digit
// in the round's earlier wavefronts, plus those on lower lanes of its own wavefront.
__global__ void __launch_bounds__(kSortThreads) sort_scatter_kernel(SortArgs a, int pass) {
  __shared__ unsigned base[256];   // where the tile's next item of each digit goes
  __shared__ unsigned wcnt[4][256];
  Tile T;
  const long long t = blockIdx.x;
  if (!tile_of(a, t, T)) return;
  const int tid = (int)threadIdx.x, w = tid >> 6;
  unsigned k[kPerThread], v[kPerThread];
  load_tile_words(a.key[pass & 1], T, k);
  load_tile_words(a.val[pass & 1], T, v);
  base[tid] = a.cnt[cnt_index(a, T, tid, t)];
  for (int q = 0; q < 4; ++q) wcnt[q][tid] = 0u;
  __syncthreads();
  unsigned* kout = a.key[(pass + 1) & 1];
  unsigned* vout = a.val[(pass + 1) & 1];
  const int sh = 8 * pass;
  const uint64_t below = lanes_below();
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const bool has = T.g0 + (long long)i * kSortThreads + tid < T.g1;
    const unsigned d = (k[i] >> sh) & 255u;
    const uint64_t same = same_digit(d, has);
    const unsigned in_wave = (unsigned)__popcll(same & below);
    // the lowest lane of each digit group records the group's size
    if (has && in_wave == 0u) wcnt[w][d] = (unsigned)__popcll(same);
    __syncthreads();
    if (has) {
      unsigned before = 0;
      for (int q = 0; q < w; ++q) before += wcnt[q][d];
      const unsigned pos = base[d] + before + in_wave;
      kout[pos] = k[i];
      vout[pos] = v[i];
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

// One particle's columns.
struct Item {
  double d[7];
  unsigned long long id, parent;
  unsigned birth, nev;
};

// Items of the tile in sorted order (through the permutation, which stays inside the
// instance) into the workspace rows of the same index.
__global__ void __launch_bounds__(kSortThreads) sort_gather_kernel(SortArgs a, int last) {
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  const ColView c = col_view(a);
  const unsigned* perm = a.val[last];
  const qed_soa& s = a.s;
  const bool nev = s.n_events != nullptr;
  for (long long r0 = T.g0 + threadIdx.x; r0 < T.g1; r0 += kBatch * kSortThreads) {
    Item it[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const long long g = r0 + (long long)u * kSortThreads;
      if (g < T.g1) {
        const long long i = T.sbase + (long long)perm[g];
        it[u].d[0] = s.x[i];
        it[u].d[1] = s.y[i];
        it[u].d[2] = s.z[i];
        it[u].d[3] = s.px[i];
        it[u].d[4] = s.py[i];
        it[u].d[5] = s.pz[i];
        it[u].d[6] = s.w[i];
        it[u].id = s.id[i];
        it[u].parent = s.parent[i];
        it[u].birth = s.birth[i];
        it[u].nev = nev ? s.n_events[i] : 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const long long g = r0 + (long long)u * kSortThreads;
      if (g >= T.g1) break;
      for (int k = 0; k < 7; ++k) c.d[k][g] = it[u].d[k];
      c.id[g] = it[u].id;
      c.parent[g] = it[u].parent;
      c.birth[g] = it[u].birth;
      c.nev[g] = it[u].nev;
    }
  }
}

__global__ void __launch_bounds__(kSortThreads) sort_store_kernel(SortArgs a) {
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  const ColView c = col_view(a);
  const qed_soa& s = a.s;
  const bool nev = s.n_events != nullptr;
  for (long long r0 = T.g0 + threadIdx.x; r0 < T.g1; r0 += kBatch * kSortThreads) {
    Item it[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const long long g = r0 + (long long)u * kSortThreads;
      if (g < T.g1) {
        for (int k = 0; k < 7; ++k) it[u].d[k] = c.d[k][g];
        it[u].id = c.id[g];
        it[u].parent = c.parent[g];
        it[u].birth = c.birth[g];
        it[u].nev = c.nev[g];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const long long g = r0 + (long long)u * kSortThreads;
      if (g >= T.g1) break;
      const long long i = T.sbase + g;
      s.x[i] = it[u].d[0];
      s.y[i] = it[u].d[1];
      s.z[i] = it[u].d[2];
      s.px[i] = it[u].d[3];
      s.py[i] = it[u].d[4];
      s.pz[i] = it[u].d[5];
      s.w[i] = it[u].d[6];
      s.id[i] = it[u].id;
      s.parent[i] = it[u].parent;
      s.birth[i] = it[u].birth;
      if (nev) s.n_events[i] = it[u].nev;
    }
  }
}

// ------------------------------------------------------------------------------------
// Thinning per cell (qed_thin_cells), on the store the sort above has just ordered: a
// group is a run of one key within an instance.  Heads (first items of groups) are counted
// per tile and scanned, which numbers the groups; one thread per group then sums its weight,
// draws its survivors and fixes its factor, in store order, as a sequential loop does; the
// survivors are ranked per tile, scanned, gathered with their new weights into the column
// copy and written back to the segments, whose counts and records the last launch sets.
// ------------------------------------------------------------------------------------
struct ThinArgs {
  const unsigned* key;  // sorted keys
  unsigned* gid;        // group of each item
  unsigned* keep;       // survival flag of each item
  unsigned* kpre;       // survivor rank of each item within its tile
  unsigned* hcnt;       // per tile: heads, then (scanned) heads before the tile
  unsigned* kcnt;       // per tile: survivors, then (scanned) survivors before the tile
  unsigned* gstart;     // [groups + 1] first item of each group
  double *gfac, *gw, *gwa;
  unsigned* gkept;
  unsigned* big;        // groups of more than kBigGroup particles, for thin_big_kernel
  long long* gpfx;      // [n_inst + 1] groups before each instance
  long long* kpref;     // [n_inst + 1] survivors before each instance
  long long max_per_cell;
  const long long* d_step;
  qed_thin_cells_record* rec;
};

__device__ __forceinline__ bool is_head(const SortArgs& a, const ThinArgs& t, const Tile& T,
                                        long long g) {
  return g == a.gpref[T.inst] || t.key[g] != t.key[g - 1];
}

// Exclusive scan, in tile order, of the thread's kPerThread flags (item i*256 + thread);
// every thread of the workgroup calls it.  Returns the tile's total.
__device__ unsigned tile_exclusive_scan(const unsigned (&f)[kPerThread],
                                        unsigned (&pre)[kPerThread], unsigned* sw) {
  unsigned carry = 0;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    unsigned total;
    const unsigned ex = block_exclusive_scan(f[i], sw, total);
    pre[i] = carry + ex;
    carry += total;
  }
  return carry;
}

__global__ void __launch_bounds__(kSortThreads) thin_heads_kernel(SortArgs a, ThinArgs t) {
  __shared__ unsigned sw[4];
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  unsigned f[kPerThread], pre[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long long g = T.g0 + (long long)i * kSortThreads + threadIdx.x;
    f[i] = (g < T.g1 && is_head(a, t, T, g)) ? 1u : 0u;
  }
  const unsigned total = tile_exclusive_scan(f, pre, sw);
  if (threadIdx.x == 0) t.hcnt[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the per-tile counts (which = 0: heads, 1: survivors),
// their total, and the per-instance prefix at each instance's first tile.
__global__ void __launch_bounds__(kSortThreads) thin_scan_kernel(SortArgs a, ThinArgs t,
                                                                 int which) {
  __shared__ unsigned sw[4];
  unsigned* cnt = which == 0 ? t.hcnt : t.kcnt;
  long long* pfx = which == 0 ? t.gpfx : t.kpref;
  const long long tiles = a.hdr->tiles;
  unsigned long long carry = 0;
  for (long long b = 0; b < tiles; b += blockDim.x) {
    const long long i = b + threadIdx.x;
    const unsigned v = i < tiles ? cnt[i] : 0u;
    unsigned total;
    const unsigned ex = block_exclusive_scan(v, sw, total);
    if (i < tiles) cnt[i] = (unsigned)(carry + ex);
    carry += total;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= a.n_inst; i += blockDim.x) {
    const long long tp = a.tpref[i];
    pfx[i] = tp < tiles ? (long long)cnt[tp] : (long long)carry;
  }
  if (threadIdx.x == 0) {
    if (which == 0) {
      a.hdr->groups = (long long)carry;
      a.hdr->nbig = 0;
      t.gstart[carry] = (unsigned)a.hdr->n;
    } else {
      a.hdr->kept = (long long)carry;
    }
  }
}

__global__ void __launch_bounds__(kSortThreads) thin_groups_kernel(SortArgs a, ThinArgs t) {
  __shared__ unsigned sw[4];
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  unsigned f[kPerThread], pre[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long long g = T.g0 + (long long)i * kSortThreads + threadIdx.x;
    f[i] = (g < T.g1 && is_head(a, t, T, g)) ? 1u : 0u;
  }
  tile_exclusive_scan(f, pre, sw);
  const long long base = (long long)t.hcnt[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long long g = T.g0 + (long long)i * kSortThreads + threadIdx.x;
    if (g >= T.g1) continue;
    const long long gid = base + (long long)pre[i] + (long long)f[i] - 1;  // heads so far - 1
    t.gid[g] = (unsigned)gid;
    if (f[i]) t.gstart[gid] = (unsigned)g;
  }
}

// Groups of more particles than this go to thin_big_kernel (a workgroup each); smaller ones
// are walked by one thread, in store order.
constexpr long long kBigGroup = 1024;

// The survival draw of one particle.
__device__ __forceinline__ double thin_draw(uint64_t id, uint64_t seed, uint32_t step) {
  const uint4 o = draw_words(id, seed, step, 0u, kThinCell);
  return uniform64(o.x, o.y);
}

// One thread per group, in store order within the group: its weight, its survivors and its
// factor (a group of removed photons: none, factor 0).  Groups of more than kBigGroup
// particles are listed for thin_big_kernel.
__global__ void __launch_bounds__(kSortThreads) thin_decide_kernel(SortArgs a, ThinArgs t) {
  const long long groups = a.hdr->groups;
  const long long M = t.max_per_cell;
  const uint32_t step = (uint32_t)*t.d_step;
  const qed_soa& S = a.s;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < groups; q += stride) {
    const long long g0 = t.gstart[q], g1 = t.gstart[q + 1];
    const int inst = find_instance(a.gpref, a.n_inst, g0);
    const long long sb = a.inst[inst].base[a.species] - a.gpref[inst];
    const long long m = g1 - g0;
    if (m > kBigGroup) {  // removed photons too: all their flags are cleared there
      const unsigned long long at = atomicAdd(reinterpret_cast<unsigned long long*>(&a.hdr->nbig), 1ull);
      t.big[at] = (unsigned)q;
      continue;
    }
    if (t.key[g0] == a.dead) {  // removed photons
      for (long long g = g0; g < g1; ++g) t.keep[g] = 0u;
      t.gfac[q] = 0.0;
      t.gw[q] = 0.0;
      t.gwa[q] = 0.0;
      t.gkept[q] = 0u;
      continue;
    }
    double W = 0.0;
    for (long long g = g0; g < g1; ++g) W += S.w[sb + g];
    t.gw[q] = W;
    if (m <= M) {
      for (long long g = g0; g < g1; ++g) t.keep[g] = 1u;
      t.gfac[q] = 1.0;
      t.gwa[q] = W;
      t.gkept[q] = (unsigned)m;
      continue;
    }
    const double qs = (double)M / (double)m;
    const uint64_t seed = a.inst[inst].seed;
    double K = 0.0, umin = 2.0;
    long long kept = 0, gmin = g0;
    for (long long g = g0; g < g1; ++g) {
      const double u = thin_draw(S.id[sb + g], seed, step);
      const bool k = u < qs;
      t.keep[g] = k ? 1u : 0u;
      if (k) {
        ++kept;
        K += S.w[sb + g];
      }
      if (u < umin) {
        umin = u;
        gmin = g;
      }
    }
    if (kept == 0) {  // the group keeps its weight in its smallest draw
      t.keep[gmin] = 1u;
      K = S.w[sb + gmin];
      kept = 1;
    }
    const double fac = W / K;
    double Wa = 0.0;
    for (long long g = g0; g < g1; ++g)
      if (t.keep[g]) Wa += S.w[sb + g] * fac;
    t.gfac[q] = fac;
    t.gwa[q] = Wa;
    t.gkept[q] = (unsigned)kept;
  }
}

// Sums over a workgroup in a fixed order: each thread's partial, then a fixed tree.
__device__ double block_sum(double v, double* sd) {
  sd[threadIdx.x] = v;
  __syncthreads();
  for (int h = kSortThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sd[threadIdx.x] += sd[threadIdx.x + h];
    __syncthreads();
  }
  const double r = sd[0];
  __syncthreads();
  return r;
}

// One workgroup per listed group (more than kBigGroup particles, removed photons' too): the
// same decisions as thin_decide_kernel, with the sums taken per thread over a strided share
// and then over the workgroup in a fixed order (the weights agree with a sequential walk to
// rounding).
__global__ void __launch_bounds__(kSortThreads) thin_big_kernel(SortArgs a, ThinArgs t) {
  __shared__ double sd[kSortThreads];
  __shared__ unsigned long long sk[kSortThreads];
  __shared__ double su[kSortThreads];
  __shared__ long long sg[kSortThreads];
  const long long nbig = a.hdr->nbig;
  const long long M = t.max_per_cell;
  const uint32_t step = (uint32_t)*t.d_step;
  const qed_soa& S = a.s;
  const int tid = (int)threadIdx.x;
  for (long long b = blockIdx.x; b < nbig; b += gridDim.x) {
    const long long q = t.big[b];
    const long long g0 = t.gstart[q], g1 = t.gstart[q + 1];
    const int inst = find_instance(a.gpref, a.n_inst, g0);
    const long long sb = a.inst[inst].base[a.species] - a.gpref[inst];
    const long long m = g1 - g0;
    if (t.key[g0] == a.dead) {  // removed photons
      for (long long g = g0 + tid; g < g1; g += kSortThreads) t.keep[g] = 0u;
      if (tid == 0) {
        t.gfac[q] = 0.0;
        t.gw[q] = 0.0;
        t.gwa[q] = 0.0;
        t.gkept[q] = 0u;
      }
      continue;
    }
    double w_part = 0.0;
    for (long long g = g0 + tid; g < g1; g += kSortThreads) w_part += S.w[sb + g];
    const double W = block_sum(w_part, sd);
    if (m <= M) {  // not reached while kBigGroup >= the cap, kept for any cap
      for (long long g = g0 + tid; g < g1; g += kSortThreads) t.keep[g] = 1u;
      if (tid == 0) {
        t.gw[q] = W;
        t.gfac[q] = 1.0;
        t.gwa[q] = W;
        t.gkept[q] = (unsigned)m;
      }
      continue;
    }
    const double qs = (double)M / (double)m;
    const uint64_t seed = a.inst[inst].seed;
    double k_part = 0.0, umin = 2.0;
    unsigned long long kept = 0;
    long long gmin = g1;
    for (long long g = g0 + tid; g < g1; g += kSortThreads) {
      const double u = thin_draw(S.id[sb + g], seed, step);
      const bool k = u < qs;
      t.keep[g] = k ? 1u : 0u;
      if (k) {
        ++kept;
        k_part += S.w[sb + g];
      }
      if (u < umin) {  // strided order: the first smallest of this thread's share
        umin = u;
        gmin = g;
      }
    }
    double K = block_sum(k_part, sd);
    // kept count and the smallest draw (the first in store order on a tie)
    sk[tid] = kept;
    su[tid] = umin;
    sg[tid] = gmin;
    __syncthreads();
    for (int h = kSortThreads / 2; h > 0; h >>= 1) {
      if (tid < h) {
        sk[tid] += sk[tid + h];
        if (su[tid + h] < su[tid] || (su[tid + h] == su[tid] && sg[tid + h] < sg[tid])) {
          su[tid] = su[tid + h];
          sg[tid] = sg[tid + h];
        }
      }
      __syncthreads();
    }
    unsigned long long nkept = sk[0];
    const long long gm = sg[0];
    __syncthreads();
    long long gforce = -1;  // the survivor a group without one gets (its flag is set below)
    if (nkept == 0) {  // the group keeps its weight in its smallest draw
      gforce = gm;
      if (tid == 0) t.keep[gm] = 1u;
      K = S.w[sb + gm];
      nkept = 1;
    }
    const double fac = W / K;
    double wa_part = 0.0;
    for (long long g = g0 + tid; g < g1; g += kSortThreads) {
      // a thread reads only the flags it wrote itself
      const bool kept_g = gforce >= 0 ? g == gforce : t.keep[g] != 0u;
      if (kept_g) wa_part += S.w[sb + g] * fac;
    }
    const double Wa = block_sum(wa_part, sd);
    if (tid == 0) {
      t.gw[q] = W;
      t.gfac[q] = fac;
      t.gwa[q] = Wa;
      t.gkept[q] = (unsigned)nkept;
    }
  }
}

__global__ void __launch_bounds__(kSortThreads) thin_keep_kernel(SortArgs a, ThinArgs t) {
  __shared__ unsigned sw[4];
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  unsigned f[kPerThread], pre[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long long g = T.g0 + (long long)i * kSortThreads + threadIdx.x;
    f[i] = g < T.g1 ? t.keep[g] : 0u;
  }
  const unsigned total = tile_exclusive_scan(f, pre, sw);
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long long g = T.g0 + (long long)i * kSortThreads + threadIdx.x;
    if (g < T.g1) t.kpre[g] = pre[i];
  }
  if (threadIdx.x == 0) t.kcnt[blockIdx.x] = total;
}

// Survivors of the tile into the column copy at their rank among all survivors, with the
// group's factor on the weight.
__global__ void __launch_bounds__(kSortThreads) thin_gather_kernel(SortArgs a, ThinArgs t) {
  Tile T;
  if (!tile_of(a, blockIdx.x, T)) return;
  const ColView c = col_view(a);
  const qed_soa& s = a.s;
  const bool nev = s.n_events != nullptr;
  const long long base = (long long)t.kcnt[blockIdx.x];
  for (long long g = T.g0 + threadIdx.x; g < T.g1; g += kSortThreads) {
    if (!t.keep[g]) continue;
    const long long i = T.sbase + g;
    const long long d = base + (long long)t.kpre[g];
    c.d[0][d] = s.x[i];
    c.d[1][d] = s.y[i];
    c.d[2][d] = s.z[i];
    c.d[3][d] = s.px[i];
    c.d[4][d] = s.py[i];
    c.d[5][d] = s.pz[i];
    c.d[6][d] = s.w[i] * t.gfac[t.gid[g]];
    c.id[d] = s.id[i];
    c.parent[d] = s.parent[i];
    c.birth[d] = s.birth[i];
    c.nev[d] = nev ? s.n_events[i] : 0u;
  }
}

// The column copy back into the segments: survivor j of instance i goes to slot
// base_i + (j - survivors before instance i).
__global__ void __launch_bounds__(kSortThreads) thin_store_kernel(SortArgs a, ThinArgs t) {
  const long long kept = a.hdr->kept;
  const ColView c = col_view(a);
  const qed_soa& s = a.s;
  const bool nev = s.n_events != nullptr;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < kept; j += stride) {
    const int inst = find_instance(t.kpref, a.n_inst, j);
    const long long i = a.inst[inst].base[a.species] + (j - t.kpref[inst]);
    const double x = c.d[0][j], y = c.d[1][j], z = c.d[2][j];
    const double px = c.d[3][j], py = c.d[4][j], pz = c.d[5][j], w = c.d[6][j];
    const unsigned long long id = c.id[j], parent = c.parent[j];
    const unsigned birth = c.birth[j], ne = c.nev[j];
    s.x[i] = x;
    s.y[i] = y;
    s.z[i] = z;
    s.px[i] = px;
    s.py[i] = py;
    s.pz[i] = pz;
    s.w[i] = w;
    s.id[i] = id;
    s.parent[i] = parent;
    s.birth[i] = birth;
    if (nev) s.n_events[i] = ne;
  }
}

// One workgroup per instance: the new count and the record (fixed-order reductions over
// the instance's groups).
__global__ void __launch_bounds__(kSortThreads) thin_finish_kernel(SortArgs a, ThinArgs t) {
  __shared__ double sd[2][kSortThreads];
  __shared__ long long sl[3][kSortThreads];
  const int i = blockIdx.x;
  qed_instance& I = a.inst[i];
  qed_thin_cells_record* r = t.rec + i;
  if (I.frozen) {
    if (threadIdx.x == 0) *r = qed_thin_cells_record{};
    return;
  }
  double wb = 0.0, wa = 0.0;
  long long live = 0, groups = 0, thinned = 0;
  for (long long q = t.gpfx[i] + threadIdx.x; q < t.gpfx[i + 1]; q += blockDim.x) {
    const long long g0 = t.gstart[q], m = (long long)t.gstart[q + 1] - g0;
    if (t.key[g0] == a.dead) continue;
    live += m;
    groups += 1;
    thinned += m > t.max_per_cell ? 1 : 0;
    wb += t.gw[q];
    wa += t.gwa[q];
  }
  sd[0][threadIdx.x] = wb;
  sd[1][threadIdx.x] = wa;
  sl[0][threadIdx.x] = live;
  sl[1][threadIdx.x] = groups;
  sl[2][threadIdx.x] = thinned;
  __syncthreads();
  for (int h = kSortThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sd[0][threadIdx.x] += sd[0][threadIdx.x + h];
      sd[1][threadIdx.x] += sd[1][threadIdx.x + h];
      for (int k = 0; k < 3; ++k) sl[k][threadIdx.x] += sl[k][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long long kept = t.kpref[i + 1] - t.kpref[i];
    I.count[a.species] = kept;
    r->live_before = sl[0][0];
    r->kept = kept;
    r->groups = sl[1][0];
    r->groups_thinned = sl[2][0];
    r->weight_before = sd[0][0];
    r->weight_after = sd[1][0];
  }
}

}  // namespace

SortGeometry sort_geometry(const int n[3]) {
  SortGeometry g{};
  for (g.shift = 0; g.shift < 31; ++g.shift) {
    long long b = 1;
    for (int d = 0; d < 3; ++d) b *= ((long long)n[d] + (1ll << g.shift) - 1) >> g.shift;
    if (b <= (1ll << 24) - 2) break;
  }
  long long blocks = 1;
  for (int d = 0; d < 3; ++d) {
    g.nb[d] = ((long long)n[d] + (1ll << g.shift) - 1) >> g.shift;
    blocks *= g.nb[d];
  }
  g.passes = 1;
  while (g.passes < kSortMaxPasses && blocks > (1ll << (8 * g.passes)) - 2) ++g.passes;
  g.dead = (unsigned)((1ull << (8 * g.passes)) - 1);
  return g;
}

namespace {

SortArgs sort_args(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                   const SortLayout& L, const SortGeometry& geo, const int n[3],
                   const double dx[3], const double origin[3], unsigned char* w) {
  SortArgs a{};
  a.s = s;
  a.inst = inst;
  a.n_inst = n_inst;
  a.species = species;
  a.shift = geo.shift;
  a.passes = geo.passes;
  a.dead = geo.dead;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = n[d];
    a.nb[d] = geo.nb[d];
    a.dx[d] = dx[d];
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
  return a;
}

void enqueue_sort(const SortArgs& a, const SortLayout& L, const SortGeometry& geo,
                  hipStream_t st) {
  const unsigned grid = (unsigned)L.tiles_max;  // one workgroup per possible tile
  const unsigned chunks = (unsigned)((L.tiles_max * 256 + kScanChunk - 1) / kScanChunk);
  const dim3 blk(kSortThreads);
  hipLaunchKernelGGL(sort_prep_kernel, dim3(1), dim3(64), 0, st, a);
  hipLaunchKernelGGL(sort_key_kernel, dim3(grid), blk, 0, st, a);
  for (int pass = 0; pass < geo.passes; ++pass) {
    hipLaunchKernelGGL(sort_hist_kernel, dim3(grid), blk, 0, st, a, pass);
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(chunks), blk, 0, st, a);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), blk, 0, st, a);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(chunks), blk, 0, st, a);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3(grid), blk, 0, st, a, pass);
  }
  hipLaunchKernelGGL(sort_gather_kernel, dim3(grid), blk, 0, st, a, geo.passes & 1);
  hipLaunchKernelGGL(sort_store_kernel, dim3(grid), blk, 0, st, a);
}

}  // namespace

hipError_t launch_sort_cells(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                             long long slots, const int n[3], const double dx[3],
                             const double origin[3], void* work, hipStream_t st) {
  const SortLayout L = SortLayout::make(n_inst, slots);
  const SortGeometry geo = sort_geometry(n);
  const SortArgs a = sort_args(s, species, inst, n_inst, L, geo, n, dx, origin,
                               static_cast<unsigned char*>(work));
  enqueue_sort(a, L, geo, st);
  return hipGetLastError();
}

hipError_t launch_thin_cells(const qed_soa& s, int species, qed_instance* inst, int n_inst,
                             long long slots, const int n[3], const double dx[3],
                             const double origin[3], long long max_per_cell,
                             const long long* d_step, qed_thin_cells_record* rec, void* work,
                             hipStream_t st) {
  const ThinCellsLayout L = ThinCellsLayout::make(n_inst, slots);
  const SortGeometry geo = sort_geometry(n);
  unsigned char* w = static_cast<unsigned char*>(work);
  const SortArgs a = sort_args(s, species, inst, n_inst, L.sort, geo, n, dx, origin, w);
  enqueue_sort(a, L.sort, geo, st);
  ThinArgs t{};
  t.key = a.key[geo.passes & 1];
  t.gid = a.key[(geo.passes + 1) & 1];
  t.keep = a.val[geo.passes & 1];
  t.kpre = a.val[(geo.passes + 1) & 1];
  t.hcnt = a.cnt;
  t.kcnt = a.cnt + L.sort.tiles_max;
  t.gstart = reinterpret_cast<unsigned*>(w + L.gstart);
  t.gfac = reinterpret_cast<double*>(w + L.gfac);
  t.gw = reinterpret_cast<double*>(w + L.gw);
  t.gwa = reinterpret_cast<double*>(w + L.gwa);
  t.gkept = reinterpret_cast<unsigned*>(w + L.gkept);
  t.big = reinterpret_cast<unsigned*>(w + L.big);
  t.gpfx = reinterpret_cast<long long*>(w + L.gpfx);
  t.kpref = reinterpret_cast<long long*>(w + L.kpref);
  t.max_per_cell = max_per_cell;
  t.d_step = d_step;
  t.rec = rec;
  const unsigned grid = (unsigned)L.sort.tiles_max;
  const long long gb = (L.sort.cap + 255) / 256;
  const unsigned group_blocks = (unsigned)(gb < 4096 ? gb : 4096);
  const dim3 blk(kSortThreads);
  hipLaunchKernelGGL(thin_heads_kernel, dim3(grid), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_scan_kernel, dim3(1), blk, 0, st, a, t, 0);
  hipLaunchKernelGGL(thin_groups_kernel, dim3(grid), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_decide_kernel, dim3(group_blocks), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_big_kernel, dim3(1024), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_keep_kernel, dim3(grid), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_scan_kernel, dim3(1), blk, 0, st, a, t, 1);
  hipLaunchKernelGGL(thin_gather_kernel, dim3(grid), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_store_kernel, dim3(group_blocks), blk, 0, st, a, t);
  hipLaunchKernelGGL(thin_finish_kernel, dim3((unsigned)n_inst), blk, 0, st, a, t);
  return hipGetLastError();
}

}  // namespace qedk
