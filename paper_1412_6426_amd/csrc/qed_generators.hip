// qed_generators.hip -- the emission event generators of Sec. IV.G of Gonoskov et al.,
// arXiv:1412.6426, as independent trials for one lepton state (the setting of the paper's
// comparison of their spectra): the modified generator of Eq. (25) that the step uses, the
// alternative one of Eq. (24), and the standard one of Eqs. (22)-(23) with its cutoff.
//
// With q = 1.5 chi 2^u, delta(u) = q / (1 + q) maps u = log2 z (z the argument of the
// synchrotron functions) to the photon's energy fraction, and d delta / du =
// ln 2 delta (1 - delta).  The standard generator's W is integrated in u over the rate
// table's own intervals (the interpolated rate is smooth inside each one) by 8-point
// Gauss-Legendre, one interval per thread, and summed in a fixed order; a trial then finds
// the interval that holds r2 W(1) by binary search and solves inside it by Newton steps on
// the interval's quadrature, kept inside a shrinking bracket.
#include <math.h>

#include "qed_internal.h"

namespace qedk {

namespace {

constexpr int kGl = 8;         // Gauss-Legendre points per interval
constexpr int kScanThreads = 1024;
constexpr long long kMaxPanels = 1ll << 22;

struct TrialArgs {
  const DevTables* tables;
  int generator;
  double chi, gamma, dtfac;
  uint32_t key0, key1;
  long long first, n;
  double* out;
  // standard generator: W at the interval ends, the intervals
  const double* cum;
  double* part;
  long long panels;
  double u0;  // log2 z at delta_min: the first interval's start
  double k0;  // table node index of the first interval's end
  double glx[kGl / 2], glw[kGl / 2];  // positive nodes on [-1, 1] and their weights
};

// Eq. (24)'s density P(delta) from the FP64 tables (global memory; L2-resident).
__device__ __forceinline__ double density(const TrialArgs& a, const Series64& ser, double d) {
  if (!(d > 0.0 && d < 1.0)) return 0.0;
  const double omd = 1.0 - d;
  const double z = (2.0 / 3.0) * d / (omd * a.chi);
  return (a.dtfac * kInvSqrt3Pi / a.gamma) *
         emission_bracket64(a.tables->ab64, ser, z, d * d / omd);
}

// W's integrand in u.
__device__ __forceinline__ double integrand(const TrialArgs& a, const Series64& ser, double u) {
  const double q = 1.5 * a.chi * exp2(u);
  const double d = q / (1.0 + q);
  return density(a, ser, d) * 0.6931471805599453 * d / (1.0 + q);
}

__device__ __forceinline__ double gauss_legendre(const TrialArgs& a, const Series64& ser,
                                                 double lo, double hi) {
  const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < kGl / 2; ++m)
    s += a.glw[m] * (integrand(a, ser, c - h * a.glx[m]) + integrand(a, ser, c + h * a.glx[m]));
  return h * s;
}

// End of interval k (k = 0..panels): u0, then table nodes, the last one at z = 2^7.
__device__ __forceinline__ double edge(const TrialArgs& a, long long k) {
  if (k == 0) return a.u0;
  const double e = kLog2ZLo + (a.k0 + (double)(k - 1)) / kNodesPerLog2;
  return k >= a.panels || e > kLog2ZHi ? kLog2ZHi : e;
}

__device__ __forceinline__ Series64 series_of(const DevTables* t) {
  return Series64{t->series[0], t->series[1], t->series[2], t->series[3], t->series[4]};
}

__global__ void __launch_bounds__(256) w_panel_kernel(TrialArgs a) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.panels) return;
  const Series64 ser = series_of(a.tables);
  a.part[k] = gauss_legendre(a, ser, edge(a, k), edge(a, k + 1));
}

// cum[0] = 0, cum[k + 1] = cum[k] + part[k]: each thread sums one contiguous run, the run
// totals are scanned in LDS, then each run is written out (a fixed order of additions).
__global__ void __launch_bounds__(kScanThreads) w_scan_kernel(TrialArgs a) {
  __shared__ double tot[kScanThreads];
  const long long n = a.panels;
  const long long per = (n + kScanThreads - 1) / kScanThreads;
  const long long lo = per * threadIdx.x;
  const long long hi = lo + per < n ? lo + per : n;
  double s = 0.0;
  for (long long k = lo; k < hi; ++k) s += a.part[k];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int t = 0; t < kScanThreads; ++t) {
      const double v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  double* cum = const_cast<double*>(a.cum);
  double run = tot[threadIdx.x];
  if (threadIdx.x == 0) cum[0] = 0.0;
  for (long long k = lo; k < hi; ++k) {
    run += a.part[k];
    cum[k + 1] = run;
  }
}

// Eq. (22): the root of W(delta) = target, W(1) >= target >= 0 (cum: W at the interval
// ends, in LDS or global memory).
__device__ double standard_delta(const TrialArgs& a, const Series64& ser, const double* cum,
                                 double target) {
  long long lo = 0, hi = a.panels;
  while (hi - lo > 1) {
    const long long mid = (lo + hi) >> 1;
    if (cum[mid] <= target) lo = mid; else hi = mid;
  }
  const double ua = edge(a, lo), ub = edge(a, lo + 1);
  const double base = cum[lo], span = cum[lo + 1] - base;
  const double want = target - base;
  double blo = ua, bhi = ub;
  double u = span > 0.0 ? ua + (ub - ua) * (want / span) : 0.5 * (ua + ub);
  if (!(u > blo && u < bhi)) u = 0.5 * (blo + bhi);
  const double tol = 0x1p-50 * fmax(fmax(fabs(ua), fabs(ub)), 1.0);
  for (int it = 0; it < 60; ++it) {
    const double g = gauss_legendre(a, ser, ua, u) - want;
    if (g > 0.0) bhi = u; else blo = u;
    const double f = integrand(a, ser, u);
    if (f > 0.0) {
      // converged once the Newton step is below the tolerance (it may then round to u, which
      // is why this is tested before the bracket)
      const double step = g / f;
      if (fabs(step) <= tol) {
        u -= step;
        break;
      }
      u -= step;
    } else {
      u = 0.5 * (blo + bhi);
    }
    if (!(u > blo && u < bhi)) u = 0.5 * (blo + bhi);
    if (!(bhi - blo > tol)) break;
  }
  const double q = 1.5 * a.chi * exp2(u);
  return q / (1.0 + q);
}

// The modified and alternative generators (one kernel each, so that both stay lean).
template <int GEN>
__global__ void __launch_bounds__(256) trial_kernel(TrialArgs a) {
  const bool ok = a.tables->magic == kTableMagic;
  const Series64 ser = series_of(a.tables);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    if (!ok) {
      a.out[i] = __builtin_nan("");
      continue;
    }
    const uint64_t j = (uint64_t)(a.first + i);
    const uint4 o = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)(j >> 32), 0u, 0u), a.key0,
                                  a.key1);
    const double r1 = uniform64(o.x, o.y), r2 = uniform64(o.z, o.w);
    double delta = 0.0;
    if (GEN == QED_GEN_MODIFIED) {
      const double d = r1 * r1 * r1;
      if (r2 < 3.0 * r1 * r1 * density(a, ser, d)) delta = d;
    } else {
      if (r2 < density(a, ser, r1)) delta = r1;
    }
    a.out[i] = delta;
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The standard generator.  W's interval ends are staged in LDS when they fit (the binary
// search then stays on chip).  Only about W(1) of the trials emit, and their inversion is the
// costly part, so a wavefront queues its emitting trials in LDS and inverts them 64 at a
// time with every lane busy.
constexpr int kLdsCumMax = 6144;  // 48 KB
__global__ void __launch_bounds__(256) standard_kernel(TrialArgs a) {
  extern __shared__ double s_cum[];
  __shared__ long long s_qi[4][128];
  __shared__ double s_qt[4][128];
  const bool ok = a.tables->magic == kTableMagic;
  const Series64 ser = series_of(a.tables);
  const bool staged = a.panels + 1 <= kLdsCumMax;
  if (staged)
    for (long long k = threadIdx.x; k <= a.panels; k += blockDim.x) s_cum[k] = a.cum[k];
  __syncthreads();
  const double* cum = staged ? s_cum : a.cum;
  const double w1 = a.panels > 0 ? cum[a.panels] : 0.0;
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  long long* const qi = s_qi[wv];
  double* const qt = s_qt[wv];
  int qn = 0;  // wavefront-uniform
  const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long base = ((long long)blockIdx.x * (blockDim.x >> 6) + wv) * 64; base < a.n;
       base += waves * 64) {
    const long long i = base + lane;
    bool emit = false;
    double target = 0.0;
    if (i < a.n) {
      if (!ok) {
        a.out[i] = __builtin_nan("");
      } else {
        const uint64_t j = (uint64_t)(a.first + i);
        const uint4 o = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)(j >> 32), 0u, 0u),
                                      a.key0, a.key1);
        const double r1 = uniform64(o.x, o.y), r2 = uniform64(o.z, o.w);
        emit = r1 < w1;
        target = r2 * w1;
        if (!emit) a.out[i] = 0.0;
      }
    }
    const uint64_t m = wave_ballot(emit);
    if (emit) {
      const int at = qn + __popcll(m & lanes_below());
      qi[at] = i;
      qt[at] = target;
    }
    qn += __popcll(m);
    if (qn >= 64) {
      qn -= 64;
      wave_lds_sync();
      const long long qi_l = qi[qn + lane];
      const double qt_l = qt[qn + lane];
      wave_lds_sync();
      a.out[qi_l] = standard_delta(a, ser, cum, qt_l);
    }
  }
  wave_lds_sync();
  if (lane < qn) a.out[qi[lane]] = standard_delta(a, ser, cum, qt[lane]);
}

// W(1) gamma / dtfac for chi_i (one workgroup per chi): each thread integrates every 256th
// interval, then the workgroup adds the threads' sums in a fixed tree order.
struct WTableArgs {
  const DevTables* tables;
  double chi_min, log2_ratio, delta_min;
  int n;
  double* out;
  double glx[kGl / 2], glw[kGl / 2];
};

__device__ __forceinline__ long long panels_for(double chi, double delta_min, double& u0,
                                                double& k0) {
  u0 = log2((2.0 / 3.0) * delta_min / (chi * (1.0 - delta_min)));
  k0 = 0.0;
  if (!(u0 < kLog2ZHi)) return 0;
  k0 = floor((u0 - kLog2ZLo) * kNodesPerLog2) + 1.0;
  const double first_end = kLog2ZLo + k0 / kNodesPerLog2;
  if (!(first_end < kLog2ZHi)) return 1;
  return 1 + (long long)ceil((kLog2ZHi - first_end) * kNodesPerLog2);
}

__global__ void __launch_bounds__(256) w_table_kernel(WTableArgs w) {
  __shared__ double part[256];
  const int i = blockIdx.x;
  const double chi =
      w.n > 1 ? w.chi_min * exp2(w.log2_ratio * (double)i / (double)(w.n - 1)) : w.chi_min;
  TrialArgs a{};
  a.tables = w.tables;
  a.chi = chi;
  a.gamma = 1.0;
  a.dtfac = 1.0;
  a.panels = panels_for(chi, w.delta_min, a.u0, a.k0);
  for (int m = 0; m < kGl / 2; ++m) {
    a.glx[m] = w.glx[m];
    a.glw[m] = w.glw[m];
  }
  const bool ok = w.tables->magic == kTableMagic;
  const Series64 ser = series_of(w.tables);
  double s = 0.0;
  if (ok)
    for (long long k = threadIdx.x; k < a.panels; k += blockDim.x)
      s += gauss_legendre(a, ser, edge(a, k), edge(a, k + 1));
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) w.out[i] = ok ? part[0] : __builtin_nan("");
}

// Positive nodes and weights of n-point Gauss-Legendre on [-1, 1]: Newton's method on the
// Legendre polynomial P_n from the asymptotic guesses cos(pi (i + 3/4) / (n + 1/2)), the
// weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre_rule(int n, double* x, double* w) {
  for (int i = 0; i < n / 2; ++i) {
    double z = cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;  // P_n' at the final node
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

hipError_t launch_standard_w_table(const DevTables* tables, double chi_min, double chi_max,
                                   int n, double delta_min, double* out, hipStream_t s) {
  WTableArgs w{};
  w.tables = tables;
  w.chi_min = chi_min;
  w.log2_ratio = log2(chi_max / chi_min);
  w.delta_min = delta_min;
  w.n = n;
  w.out = out;
  gauss_legendre_rule(kGl, w.glx, w.glw);
  hipLaunchKernelGGL(w_table_kernel, dim3((unsigned)n), dim3(256), 0, s, w);
  return hipGetLastError();
}

// Intervals of the standard generator's W for (chi, delta_min): from u0 = log2 z(delta_min)
// to the first table node above it, then table intervals up to z = 2^7 (0: no rate).
long long standard_panels(double chi, double delta_min, double* u0, double* k0) {
  const double u = log2((2.0 / 3.0) * delta_min / (chi * (1.0 - delta_min)));
  *u0 = u;
  *k0 = 0.0;
  if (!(u < kLog2ZHi)) return 0;
  const double k = floor((u - kLog2ZLo) * kNodesPerLog2) + 1.0;
  *k0 = k;
  const double first_end = kLog2ZLo + k / kNodesPerLog2;
  if (!(first_end < kLog2ZHi)) return 1;
  return 1 + (long long)ceil((kLog2ZHi - first_end) * kNodesPerLog2);
}

size_t generator_work_bytes(long long panels) {
  const size_t part = ((size_t)panels * sizeof(double) + 255) & ~(size_t)255;
  return part + (size_t)(panels + 1) * sizeof(double);
}

long long generator_max_panels() { return kMaxPanels; }

hipError_t launch_generator_trials(const DevTables* tables, int generator, double chi,
                                   double gamma, double dtfac, double delta_min, uint64_t key,
                                   long long first, long long n, double* out, void* work,
                                   hipStream_t s) {
  TrialArgs a{};
  a.tables = tables;
  a.generator = generator;
  a.chi = chi;
  a.gamma = gamma;
  a.dtfac = dtfac;
  a.key0 = (uint32_t)key;
  a.key1 = (uint32_t)(key >> 32);
  a.first = first;
  a.n = n;
  a.out = out;
  if (generator == QED_GEN_STANDARD) {
    a.panels = standard_panels(chi, delta_min, &a.u0, &a.k0);
    char* w = static_cast<char*>(work);
    a.part = reinterpret_cast<double*>(w);
    a.cum = reinterpret_cast<const double*>(
        w + (((size_t)a.panels * sizeof(double) + 255) & ~(size_t)255));
    gauss_legendre_rule(kGl, a.glx, a.glw);
    if (a.panels > 0) {
      hipLaunchKernelGGL(w_panel_kernel, dim3((unsigned)((a.panels + 255) / 256)), dim3(256),
                         0, s, a);
      hipLaunchKernelGGL(w_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a);
    }
  }
  if (n > 0) {
    const long long blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 2048 ? blocks : 2048));
    if (generator == QED_GEN_MODIFIED) {
      hipLaunchKernelGGL(trial_kernel<QED_GEN_MODIFIED>, grid, dim3(256), 0, s, a);
    } else if (generator == QED_GEN_ALTERNATIVE) {
      hipLaunchKernelGGL(trial_kernel<QED_GEN_ALTERNATIVE>, grid, dim3(256), 0, s, a);
    } else {
      const size_t lds = a.panels + 1 <= kLdsCumMax ? (size_t)(a.panels + 1) * sizeof(double) : 0;
      hipLaunchKernelGGL(standard_kernel, grid, dim3(256), lds, s, a);
    }
  }
  return hipGetLastError();
}

}  // namespace qedk
