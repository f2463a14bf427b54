// qed_schwinger.hip -- non-perturbative (Schwinger) pair production from a Yee-grid field
// (Sec. V.B of Gonoskov et al., arXiv:1412.6426).  Per step, cell and instance a pair
// appears with probability P = R_S V c dt, R_S = (E/E_S)^2 exp(-pi E_S / E) / (4 pi^3
// lambdabar_C^4), from the cell's field taken as constant (the mean of each E component's
// four staggered samples on the cell; the magnetic field is neglected, as in the paper's
// presentation).  The pair starts at rest at a random point of the cell.
//
// One launch: a grid-stride loop over the cells, one lane per cell.  The field of a cell is
// read once and serves every instance; each instance draws with its own seed.  Pairs are
// rare, so they reserve store slots directly (one atomic per wavefront, instance and
// species), and the store order of created pairs follows the reservations.
#include "qed_internal.h"

namespace qedk {

namespace {

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

__device__ __forceinline__ double grid_at(const float* g, const int n[3], int i, int j, int k) {
  i = i == n[0] ? 0 : i;
  j = j == n[1] ? 0 : j;
  k = k == n[2] ? 0 : k;
  return (double)g[i + (long long)n[0] * (j + (long long)n[1] * k)];
}

// Reserve slots of species store S of instance li for the flagged lanes (all lanes call);
// returns the lane's slot or -1.  Drops are counted in the instance and added to the
// leader lane's `dropped`.
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
    dropped += (unsigned long long)__popcll(lost);
  }
  return (flag && fits) ? a.inst[li].base[sp] + pos : -1;
}

__global__ void __launch_bounds__(256) schwinger_kernel(SchwingerArgs a) {
  __shared__ double s_exp[4];
  __shared__ unsigned long long s_cnt[4][4];
  const int lane = lane_id();
  const int wv = (int)(threadIdx.x >> 6);
  const uint32_t step = (uint32_t)*a.d_step;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double expected = 0.0;
  unsigned long long visited = 0, pairs = 0, sat = 0, dropped = 0;
  // the loop bound is wavefront-uniform so that every lane reaches the ballots
  for (long long c0 = (long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); c0 < a.cells;
       c0 += stride) {
    const long long c = c0 + lane;
    const bool has = c < a.cells;
    double P = 0.0;
    int i = 0, j = 0, k = 0;
    if (has) {
      i = (int)(c % a.n[0]);
      const long long r = c / a.n[0];
      j = (int)(r % a.n[1]);
      k = (int)(r / a.n[1]);
      const double ex = 0.25 * (grid_at(a.g[0], a.n, i, j, k) + grid_at(a.g[0], a.n, i, j + 1, k) +
                                grid_at(a.g[0], a.n, i, j, k + 1) +
                                grid_at(a.g[0], a.n, i, j + 1, k + 1));
      const double ey = 0.25 * (grid_at(a.g[1], a.n, i, j, k) + grid_at(a.g[1], a.n, i + 1, j, k) +
                                grid_at(a.g[1], a.n, i, j, k + 1) +
                                grid_at(a.g[1], a.n, i + 1, j, k + 1));
      const double ez = 0.25 * (grid_at(a.g[2], a.n, i, j, k) + grid_at(a.g[2], a.n, i + 1, j, k) +
                                grid_at(a.g[2], a.n, i, j + 1, k) +
                                grid_at(a.g[2], a.n, i + 1, j + 1, k));
      const double e = sqrt(ex * ex + ey * ey + ez * ez) * a.eps_r;  // E / E_S
      if (e > 0.0) P = a.pref * e * e * exp(-kPi / e);
    }
    for (int li = 0; li < a.n_inst; ++li) {
      const qed_instance& I = a.inst[li];
      if (I.frozen) continue;  // instance-uniform
      const uint64_t seed = I.seed;
      if (has) {
        ++visited;
        expected += P < 1.0 ? P : 1.0;
        sat += P >= 1.0 ? 1u : 0u;
      }
      bool make = false;
      uint4 w{};
      if (has && P > 0.0) {
        const uint4 o = draw_words((uint64_t)c, seed, step, 0u, kSchwinger);
        make = uniform64(o.x, o.y) < P;
        if (make) w = draw_words((uint64_t)c, seed, step, 0u, kSchwingerPos);
      }
      if (!wave_ballot(make)) continue;
      pairs += make ? 1u : 0u;
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
  // workgroup totals (fixed order within a workgroup), then one atomic each
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    expected += __shfl_xor(expected, o, 64);
    visited += __shfl_xor(visited, o, 64);
    pairs += __shfl_xor(pairs, o, 64);
    sat += __shfl_xor(sat, o, 64);
    dropped += __shfl_xor(dropped, o, 64);
  }
  if (lane == 0) {
    s_exp[wv] = expected;
    s_cnt[wv][0] = visited;
    s_cnt[wv][1] = pairs;
    s_cnt[wv][2] = sat;
    s_cnt[wv][3] = dropped;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    unsigned long long v = 0, p = 0, s = 0, d = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      e += s_exp[q];
      v += s_cnt[q][0];
      p += s_cnt[q][1];
      s += s_cnt[q][2];
      d += s_cnt[q][3];
    }
    if (e != 0.0) atomicAdd(&a.rec->expected, e);
    if (v) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->cells), v);
    if (p) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->pairs), p);
    if (s) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->saturated), s);
    if (d) atomicAdd(reinterpret_cast<unsigned long long*>(&a.rec->dropped), d);
  }
}

__global__ void schwinger_clear_kernel(qed_schwinger_record* rec) {
  if (threadIdx.x == 0) *rec = qed_schwinger_record{};
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
  long long blocks = (a.cells + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(schwinger_clear_kernel, dim3(1), dim3(64), 0, s, rec);
  hipLaunchKernelGGL(schwinger_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace qedk
