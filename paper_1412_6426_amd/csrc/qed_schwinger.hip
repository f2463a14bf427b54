// qed_schwinger.hip -- non-perturbative (Schwinger) pair production from a Yee-grid field
// (Sec. V.B of Gonoskov et al., arXiv:1412.6426).  Per step, cell and instance a pair
// appears with probability P = R_S V c dt, R_S = (E/E_S)^2 exp(-pi E_S / E) / (4 pi^3
// lambdabar_C^4), from the cell's field taken as constant (the mean of each E component's
// four staggered samples on the cell; the magnetic field is neglected, as in the paper's
// presentation).  The pair starts at rest at a random point of the cell.
//
// One launch: a wavefront takes 64 consecutive cells of one (j, k) row of the grid at a time
// (a grid-stride loop over those pieces), so its loads coalesce and the row indices are
// wavefront-uniform.  The field of a cell is read once and serves every instance; each
// instance draws with its own seed.  A probability at or below 2^-53, the smallest uniform
// the draw can give, decides without drawing.  Pairs are rare, so they reserve store slots
// directly (one atomic per wavefront, instance and species), and the store order of created
// pairs follows the reservations.
#include "qed_internal.h"

namespace qedk {

namespace {

constexpr int kXcds = 8;  // accelerator complex dies of the GPU, each with its own L2

struct SchwingerArgs {
  const float* g[3];  // Ex, Ey, Ez
  int n[3];
  double dx[3], origin[3];
  double pref;        // V dt / (4 pi^3 eps_r^4)
  double eps_r, weight;
  qed_soa e, p;       // electron and positron stores
  qed_instance* inst;
  int n_inst;
  long long cells;
  const long long* d_step;
  qed_schwinger_record* rec;
};

// Row (j, k) of a component, with the periodic wrap of j and k (wavefront-uniform).
__device__ __forceinline__ const float* grid_row(const float* g, const int n[3], int j, int k) {
  j = j == n[1] ? 0 : j;
  k = k == n[2] ? 0 : k;
  return g + (long long)n[0] * (j + (long long)n[1] * k);
}

// Reserve slots of species store S of instance li for the flagged lanes (all lanes call);
// returns the lane's slot or -1.  Drops are counted in the instance and added to the
// wavefront-uniform `dropped`.
__device__ __forceinline__ long long reserve(const SchwingerArgs& a, int sp, bool flag, int li,
                                             unsigned long long& dropped) {
  const uint64_t m = wave_ballot(flag);
  if (!m) return -1;
  const int leader = __ffsll((unsigned long long)m) - 1;
  long long base = 0;
  if (lane_id() == leader)
    base = (long long)atomicAdd(reinterpret_cast<unsigned long long*>(&a.inst[li].count[sp]),
                                (unsigned long long)__popcll(m));
  base = wave_bcast(base, leader);
  const long long pos = base + __popcll(m & lanes_below());
  const bool fits = pos < a.inst[li].capacity[sp];
  const uint64_t lost = wave_ballot(flag && !fits);
  if (lost && lane_id() == leader) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.inst[li].dropped),
              (unsigned long long)__popcll(lost));
  }
  dropped += (unsigned long long)__popcll(lost);
  return (flag && fits) ? a.inst[li].base[sp] + pos : -1;
}

__device__ __forceinline__ float at_offset(const float* row, uint32_t byte_offset) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(row) + byte_offset);
}

// 64 consecutive cells of one row (lane i0 + lane) and their twelve field samples: Ex at
// rows (j, k), (j+1, k), (j, k+1), (j+1, k+1) of column i; Ey at (j, k) and (j, k+1) of
// columns i, i+1; Ez at (j, k) and (j+1, k) of columns i, i+1 (periodic).
struct Piece {
  int i, j, k;
  bool has;
  long long c;  // cell index i + n0 (j + n1 k)
  float v[12];
};

__device__ __forceinline__ Piece load_piece(const SchwingerArgs& a, int piece, int ppr,
                                            int lane) {
  Piece q{};
  const int row = piece / ppr;
  q.i = ((piece - row * ppr) << 6) + lane;
  q.j = row % a.n[1];
  q.k = row / a.n[1];
  q.has = q.i < a.n[0];
  q.c = (long long)q.i + (long long)a.n[0] * row;
  const float* x00 = grid_row(a.g[0], a.n, q.j, q.k);
  const float* x10 = grid_row(a.g[0], a.n, q.j + 1, q.k);
  const float* x01 = grid_row(a.g[0], a.n, q.j, q.k + 1);
  const float* x11 = grid_row(a.g[0], a.n, q.j + 1, q.k + 1);
  const float* y00 = grid_row(a.g[1], a.n, q.j, q.k);
  const float* y01 = grid_row(a.g[1], a.n, q.j, q.k + 1);
  const float* z00 = grid_row(a.g[2], a.n, q.j, q.k);
  const float* z10 = grid_row(a.g[2], a.n, q.j + 1, q.k);
  if (q.has) {
    // 32-bit byte offsets from the wavefront-uniform row pointers (a scalar base and one
    // offset register per load)
    const uint32_t o = (uint32_t)q.i << 2;
    const uint32_t o1 = q.i + 1 == a.n[0] ? 0u : o + 4u;
    q.v[0] = at_offset(x00, o);
    q.v[1] = at_offset(x10, o);
    q.v[2] = at_offset(x01, o);
    q.v[3] = at_offset(x11, o);
    q.v[4] = at_offset(y00, o);
    q.v[5] = at_offset(y00, o1);
    q.v[6] = at_offset(y01, o);
    q.v[7] = at_offset(y01, o1);
    q.v[8] = at_offset(z00, o);
    q.v[9] = at_offset(z00, o1);
    q.v[10] = at_offset(z10, o);
    q.v[11] = at_offset(z10, o1);
  }
  return q;
}

// Orders a wavefront's LDS stores before its following LDS loads (other lanes' slots).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Draws of one lane's cell c with probability P for every non-frozen instance (all lanes
// call; lanes with has == false take part in the ballots only), and the pairs they make.
// `pairs` and `dropped` are wavefront-uniform counts.
__device__ __forceinline__ void draw_cells(const SchwingerArgs& a, long long c, double P, bool has,
                                           uint32_t step, unsigned long long& pairs,
                                           unsigned long long& dropped) {
  for (int li = 0; li < a.n_inst; ++li) {
    const qed_instance& I = a.inst[li];
    if (I.frozen) continue;  // instance-uniform
    const uint64_t seed = I.seed;
    bool make = false;
    if (has) {
      const uint4 o = draw_words((uint64_t)c, seed, step, 0u, kSchwinger);
      make = uniform64(o.x, o.y) < P;
    }
    const uint64_t made = wave_ballot(make);
    if (!made) continue;
    pairs += (unsigned long long)__popcll(made);
    uint4 w{};
    long long i = 0, j = 0, k = 0;
    if (make) {
      w = draw_words((uint64_t)c, seed, step, 0u, kSchwingerPos);
      const long long row = c / a.n[0];
      i = c - row * a.n[0];
      j = row % a.n[1];
      k = row / a.n[1];
    }
    const double x = a.origin[0] + ((double)i + ((double)w.x + 0.5) * 0x1p-32) * a.dx[0];
    const double y = a.origin[1] + ((double)j + ((double)w.y + 0.5) * 0x1p-32) * a.dx[1];
    const double z = a.origin[2] + ((double)k + ((double)w.z + 0.5) * 0x1p-32) * a.dx[2];
    for (int sp = 0; sp < 2; ++sp) {
      const long long q = reserve(a, sp, make, li, dropped);
      if (q < 0) continue;
      const qed_soa& S = sp == 0 ? a.e : a.p;
      S.x[q] = x;
      S.y[q] = y;
      S.z[q] = z;
      S.px[q] = 0.0;
      S.py[q] = 0.0;
      S.pz[q] = 0.0;
      S.w[q] = a.weight;
      S.id[q] = child_id((uint64_t)c, seed, step, 0u,
                         sp == 0 ? kSchwingerElectron : kSchwingerPositron);
      S.parent[q] = QED_NO_PARENT;
      S.birth[q] = birth_code(step, 0u);
      if (S.n_events) S.n_events[q] = 0u;
    }
  }
}

__global__ void __launch_bounds__(256) schwinger_kernel(SchwingerArgs a) {
  __shared__ long long s_qc[4][128];  // per-wavefront queue of cells to draw for
  __shared__ double s_qp[4][128];     // and their probabilities
  __shared__ double s_exp[4];
  __shared__ unsigned long long s_cnt[4][3];
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform: scalar indexing
  const uint32_t step = (uint32_t)*a.d_step;
  const int pieces_per_row = (a.n[0] + 63) >> 6;
  const int rows = a.n[1] * a.n[2];
  const int pieces = rows * pieces_per_row;
  // Workgroups go to the 8 XCDs in turn (workgroup b to XCD b % 8).  XCD x takes the x-th
  // eighth of the pieces, in row order, so that a row's neighbours in j and k, which its
  // cells also read, are read through the same L2.
  const int xcd = (int)(blockIdx.x & (kXcds - 1));
  const int per_xcd = (pieces + kXcds - 1) / kXcds;
  const int p_lo = xcd * per_xcd;
  const int p_hi = p_lo + per_xcd < pieces ? p_lo + per_xcd : pieces;
  const int V = (int)(gridDim.x / kXcds) * (int)(blockDim.x >> 6);  // wavefronts of this XCD
  double expected = 0.0;
  // per lane: the expected count; per wavefront (uniform): pairs, saturated cells, drops
  unsigned long long pairs = 0, sat = 0, dropped = 0;
  int n_active = 0;
  for (int li = 0; li < a.n_inst; ++li) n_active += a.inst[li].frozen ? 0 : 1;
  // Cells whose probability needs a draw wait in this wavefront's queue, and are drawn for 64
  // at a time, so that the Philox rounds run with full wavefronts wherever the field puts the
  // drawing cells (a row of 64 cells can mix strong and weak fields).
  long long* const qc = s_qc[wv];
  double* const qp = s_qp[wv];
  int qn = 0;  // wavefront-uniform
  // wavefront-uniform loop, so that every lane reaches the ballots
  for (int piece = p_lo + (int)(blockIdx.x / kXcds) * (int)(blockDim.x >> 6) + wv; piece < p_hi;
       piece += V) {
    const Piece cur = load_piece(a, piece, pieces_per_row, lane);
    double P = 0.0;
    if (cur.has) {
      // each component the mean of its four samples on the cell, summed in this order
      const float* v = cur.v;
      const double ex = 0.25 * ((double)v[0] + (double)v[1] + (double)v[2] + (double)v[3]);
      const double ey = 0.25 * ((double)v[4] + (double)v[5] + (double)v[6] + (double)v[7]);
      const double ez = 0.25 * ((double)v[8] + (double)v[9] + (double)v[10] + (double)v[11]);
      const double e = sqrt(ex * ex + ey * ey + ez * ez) * a.eps_r;  // E / E_S
      if (e > 0.0) P = a.pref * e * e * exp(-kPi / e);
      for (int li = 0; li < n_active; ++li) {  // once per drawing instance
        expected += P < 1.0 ? P : 1.0;
      }
    }
    sat += (unsigned long long)__popcll(wave_ballot(P >= 1.0)) * (unsigned long long)n_active;
    // below 2^-53 (the smallest uniform the draw gives) a cell decides without drawing
    const bool need = cur.has && n_active > 0 && P > 0x1p-53;
    const uint64_t m = wave_ballot(need);
    if (need) {
      const int at = qn + __popcll(m & lanes_below());
      qc[at] = cur.c;
      qp[at] = P;
    }
    qn += __popcll(m);
    if (qn >= 64) {
      qn -= 64;
      wave_lds_sync();
      draw_cells(a, qc[qn + lane], qp[qn + lane], true, step, pairs, dropped);
      wave_lds_sync();
    }
  }
  if (qn > 0) {
    wave_lds_sync();
    const bool has = lane < qn;
    draw_cells(a, has ? qc[lane] : 0, has ? qp[lane] : 0.0, has, step, pairs, dropped);
  }
  // workgroup totals (fixed order within a workgroup), then one atomic each
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) expected += __shfl_xor(expected, o, 64);
  if (lane == 0) {
    s_exp[wv] = expected;
    s_cnt[wv][0] = pairs;
    s_cnt[wv][1] = sat;
    s_cnt[wv][2] = dropped;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    unsigned long long p = 0, s = 0, d = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      e += s_exp[q];
      p += s_cnt[q][0];
      s += s_cnt[q][1];
      d += s_cnt[q][2];
    }
    // the cells visited are counted by the clearing kernel
    if (e != 0.0) atomicAdd(&a.rec->expected, e);
    if (p) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->pairs), p);
    if (s) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->saturated), s);
    if (d) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->dropped), d);
  }
}

// Clears the record and counts the cells to visit (cells times non-frozen instances), so
// that the main kernel's workgroups add only what they found (one atomic each, mostly).
__global__ void schwinger_clear_kernel(qed_schwinger_record* rec, const qed_instance* inst,
                                       int n_inst, long long cells) {
  if (threadIdx.x != 0) return;
  long long active = 0;
  for (int i = 0; i < n_inst; ++i) active += inst[i].frozen ? 0 : 1;
  qed_schwinger_record r{};
  r.cells = active * cells;
  *rec = r;
}

// Reservations raise an instance's count past its capacity when pairs are dropped; bring
// every lepton count back to the capacity so that whatever reads the counts next (thinning,
// the caller, the next step) sees only slots that hold particles.
__global__ void schwinger_clamp_kernel(qed_instance* inst, int n_inst) {
  for (int i = (int)threadIdx.x; i < n_inst; i += (int)blockDim.x)
    for (int sp = 0; sp < 2; ++sp)
      if (inst[i].count[sp] > inst[i].capacity[sp]) inst[i].count[sp] = inst[i].capacity[sp];
}

}  // namespace

hipError_t launch_schwinger(const qed_stores& st, const float* const grid[3], const int n[3],
                            const double dx[3], const double origin[3], double dt, double eps_r,
                            double weight, const long long* d_step, qed_schwinger_record* rec,
                            hipStream_t s) {
  SchwingerArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.g[d] = grid[d];
    a.n[d] = n[d];
    a.dx[d] = dx[d];
    a.origin[d] = origin[d];
  }
  a.pref = dx[0] * dx[1] * dx[2] * dt / (4.0 * kPi * kPi * kPi * pow(eps_r, 4.0));
  a.eps_r = eps_r;
  a.weight = weight;
  a.e = st.species[QED_ELECTRON];
  a.p = st.species[QED_POSITRON];
  a.inst = st.d_instances;
  a.n_inst = st.n_instances;
  a.cells = (long long)n[0] * n[1] * n[2];
  a.d_step = d_step;
  a.rec = rec;
  // 4 wavefronts per SIMD on 256 CUs (each workgroup ends with a few atomics on the record,
  // so not more), a multiple of the XCD count so that every XCD gets the same number
  long long blocks = (a.cells + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  blocks = ((blocks + kXcds - 1) / kXcds) * kXcds;
  hipLaunchKernelGGL(schwinger_clear_kernel, dim3(1), dim3(64), 0, s, rec, a.inst, a.n_inst,
                     a.cells);
  hipLaunchKernelGGL(schwinger_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(schwinger_clamp_kernel, dim3(1), dim3(256), 0, s, a.inst, a.n_inst);
  return hipGetLastError();
}

}  // namespace qedk
