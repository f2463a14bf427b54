// qed_tables.hip -- FP64 construction of the rate tables on the GPU.
//
// The paper replaces per-event integration of the spectrum by tabulation and
// interpolation (Sec. IV.F).  Here the three functions
//   A(z) = int_z^inf K_{5/3},  B(z) = K_{2/3}(z),  C(z) = int_z^inf K_{1/3}
// are tabulated at z_i = 2^(-20 + 27 i/4095).  Each value comes from the integral
// representation K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt (DLMF 10.32.9) and its
// integral over z, int_z^inf K_nu = int_0^inf exp(-z cosh t) cosh(nu t) / cosh t dt,
// scaled by e^z (so the integrand is exp(-2 z sinh^2(t/2)) ...) and summed by the
// trapezoid rule with step 1/48 up to a cut-off where the integrand has underflowed.  One
// wavefront integrates one (node, function): lane j sums the terms j, j+64, ... and the
// wavefront reduces.
#include <math.h>

#include "qed_internal.h"

namespace qedk {

__device__ double scaled_bessel_integral(double nu, bool over_cosh, double z, int lane) {
  const double h = 1.0 / 48.0;
  // beyond t_max, 2 z sinh^2(t/2) > 100 + (nu + 1) t, so every further term is < e^-100 of
  // the largest one
  const double tmax = 2.0 * asinh(sqrt(50.0 / z)) + 4.0;
  const int nterms = (int)(tmax / h) + 1;
  double acc = 0.0;
  for (int j = lane; j <= nterms; j += 64) {
    const double t = (double)j * h;
    const double sh = sinh(0.5 * t);
    double f = exp(-2.0 * z * sh * sh) * cosh(nu * t);
    if (over_cosh) f /= cosh(t);
    acc += (j == 0) ? 0.5 * f : f;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  return acc * h;
}

__global__ void __launch_bounds__(256) table_nodes_kernel(DevTables* t) {
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = (int)(threadIdx.x & 63u);
  if (wave >= 3 * kTableN) return;  // whole wavefront leaves together
  const int node = wave / 3;
  const int fn = wave - 3 * node;
  const double du = (kLog2ZHi - kLog2ZLo) / (double)(kTableN - 1);
  const double z = exp2(kLog2ZLo + (double)node * du);
  double v;
  if (fn == 0) v = scaled_bessel_integral(5.0 / 3.0, true, z, lane);
  else if (fn == 1) v = scaled_bessel_integral(2.0 / 3.0, false, z, lane);
  else v = scaled_bessel_integral(1.0 / 3.0, true, z, lane);
  if (lane == 0) {
    if (fn == 0) {
      t->ab64[node].x = v;
    } else if (fn == 1) {
      t->ab64[node].y = v;
      t->bc64[node].x = v;
    } else {
      t->bc64[node].y = v;
    }
  }
}

// FP32 copies, the pair-rate bounds and the series constants.
// Bound: with z = 2/(3 chi d(1-d)) >= z_min = 8/(3 chi), the bracket of Eq. (30) is
//   (d/(1-d) + (1-d)/d) B(z) + C(z) <= 1.5 chi z B(z) + C(z) <= 1.5 chi F2sup + C(z_min),
// F2 = z K_{2/3}(z) rising to max 0.60705 at z = 0.416 then falling: F2sup = F2(z_min) when
// z_min >= 0.45, else 0.61.  Both terms grow with chi, so the bound at an interval's top
// chi holds for the whole interval.  Octave [2^(e-1), 2^e) is split into kBoundSub equal
// intervals [(1/2 + j/32) 2^e, (1/2 + (j+1)/32) 2^e); for small chi the rate grows like
// exp(-8/(3 chi)), so a whole octave's bound would overstate its lower part many times.
// A 1.001 margin covers table interpolation (~1e-6) and FP32 rounding.
__global__ void __launch_bounds__(256) table_finish_kernel(DevTables* t, Series64 s) {
  const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int nthreads = (int)(gridDim.x * blockDim.x);
  for (int i = tid; i < kTableN; i += nthreads) {
    t->ab32[i] = make_float2((float)t->ab64[i].x, (float)t->ab64[i].y);
    t->bc32[i] = make_float2((float)t->bc64[i].x, (float)t->bc64[i].y);
  }
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int nwaves = nthreads >> 6;
  for (int o = wave; o < kBoundEntries; o += nwaves) {
    const int oct = o / kBoundSub, sub = o - oct * kBoundSub;
    const double chi_hi = ldexp(0.5 + (double)(sub + 1) / (2.0 * kBoundSub), oct - kBoundOffset);
    const double zmin = 8.0 / (3.0 * chi_hi);
    double bound = 0.0;
    if (zmin < kZHi) {
      const double e = exp(-zmin);
      const double Bz = scaled_bessel_integral(2.0 / 3.0, false, zmin, lane) * e;
      const double Cz = scaled_bessel_integral(1.0 / 3.0, true, zmin, lane) * e;
      const double f2sup = zmin >= 0.45 ? zmin * Bz : 0.61;
      bound = (1.5 * chi_hi * f2sup + Cz) * 1.001;
    }
    if (lane == 0) {
      t->pair_bound64[o] = bound;
      t->pair_bound32[o] = (float)bound;
    }
  }
  if (tid == 0) {
    t->series[0] = s.b0;
    t->series[1] = s.b1;
    t->series[2] = s.c0;
    t->series[3] = s.c1;
    t->series[4] = s.c2;
    t->series[5] = t->series[6] = t->series[7] = 0.0;
  }
}

__global__ void table_seal_kernel(DevTables* t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) t->magic = kTableMagic;
}

hipError_t launch_build_tables(DevTables* t, const Series64& s, hipStream_t st) {
  const int waves = 3 * kTableN;
  hipLaunchKernelGGL(table_nodes_kernel, dim3((waves * 64 + 255) / 256), dim3(256), 0, st, t);
  hipLaunchKernelGGL(table_finish_kernel, dim3(128), dim3(256), 0, st, t, s);
  hipLaunchKernelGGL(table_seal_kernel, dim3(1), dim3(64), 0, st, t);
  return hipGetLastError();
}

}  // namespace qedk
