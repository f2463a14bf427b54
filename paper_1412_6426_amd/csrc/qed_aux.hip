// qed_aux.hip -- kernels around the step: stats log append, photon spectrum, and the
// standing-wave sampler that stands in for a field solver in the grid workload.
#include "qed_internal.h"

namespace qedk {

__global__ void __launch_bounds__(256) append_stats_kernel(const qed_stats* src, qed_stats* log,
                                                           long long cap, long long* cnt) {
  __shared__ long long s_slot;
  if (threadIdx.x == 0) s_slot = *cnt;
  __syncthreads();
  const long long slot = s_slot;
  if (slot >= 0 && slot < cap) {
    const unsigned long long* a = reinterpret_cast<const unsigned long long*>(src);
    unsigned long long* b = reinterpret_cast<unsigned long long*>(log + slot);
    for (int w = threadIdx.x; w < (int)(sizeof(qed_stats) / 8); w += blockDim.x) b[w] = a[w];
  }
  __syncthreads();
  if (threadIdx.x == 0) *cnt = slot + 1;
}

hipError_t launch_append_stats(const qed_stats* src, qed_stats* log, long long cap,
                               long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(append_stats_kernel, dim3(1), dim3(256), 0, s, src, log, cap, cnt);
  return hipGetLastError();
}

// Weighted log10 histogram of |k| over the live photons of every instance.
__global__ void __launch_bounds__(256) spectrum_kernel(qed_soa ph, const qed_instance* inst,
                                                       double llo, double inv_dl, int bins,
                                                       double* hist) {
  const qed_instance& I = inst[blockIdx.y];
  const long long n = I.count[QED_PHOTON];
  const long long base = I.base[QED_PHOTON];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long s = base + i;
    if (ph.id[s] == QED_ID_DEAD) continue;
    const double e = sqrt(ph.px[s] * ph.px[s] + ph.py[s] * ph.py[s] + ph.pz[s] * ph.pz[s]);
    if (!(e > 0.0)) continue;
    const double u = (log10(e) - llo) * inv_dl;
    if (u >= 0.0 && u < (double)bins) atomicAdd(&hist[(int)u], ph.w[s]);
  }
}

hipError_t launch_spectrum(const qed_soa& ph, qed_instance* inst, int n_inst, double lo,
                           double hi, int bins, double* hist, hipStream_t s) {
  const double llo = log10(lo);
  const double inv_dl = (double)bins / (log10(hi) - llo);
  hipLaunchKernelGGL(spectrum_kernel, dim3(256, n_inst), dim3(256), 0, s, ph, inst, llo, inv_dl,
                     bins, hist);
  return hipGetLastError();
}

struct GridPtrs {
  float* g[6];
};

// E = 2a cos(w x)(0, cos phi, sin phi), B = 2a sin(w x)(0, cos phi, sin phi) at each
// component's Yee node.
__global__ void __launch_bounds__(256) fill_standing_kernel(GridPtrs gp, int nx, int ny, int nz,
                                                            double dx, double ox, double amp,
                                                            double omega, double phase,
                                                            double t) {
  double sph, cph;
  sincos(omega * t + phase, &sph, &cph);
  const long long plane = (long long)nx * ny;
  const long long total = plane * nz;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
       c += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx);
    const double xn = ox + (double)i * dx;        // Ey, Ez, Bx nodes (x offset 0)
    const double xh = ox + ((double)i + 0.5) * dx;  // Ex, By, Bz nodes (x offset 1/2)
    const double ce = 2.0 * amp * cos(omega * xn);
    const double sb = 2.0 * amp * sin(omega * xh);
    gp.g[0][c] = 0.0f;
    gp.g[1][c] = (float)(ce * cph);
    gp.g[2][c] = (float)(ce * sph);
    gp.g[3][c] = 0.0f;
    gp.g[4][c] = (float)(sb * cph);
    gp.g[5][c] = (float)(sb * sph);
  }
}

hipError_t launch_fill_standing(float* const g[6], const int n[3], const double dx[3],
                                const double org[3], double amp, double omega, double phase,
                                double t, hipStream_t s) {
  GridPtrs gp;
  for (int c = 0; c < 6; ++c) gp.g[c] = g[c];
  const long long total = (long long)n[0] * n[1] * n[2];
  long long blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_standing_kernel, dim3((unsigned)blocks), dim3(256), 0, s, gp, n[0],
                     n[1], n[2], dx[0], org[0], amp, omega, phase, t);
  return hipGetLastError();
}

}  // namespace qedk
