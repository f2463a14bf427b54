// hbm_patterns.hip -- the HBM rate this GPU reaches for the column patterns of the step
// kernels, with no other work: the ceiling a streaming kernel with that pattern can reach.
//
// For a store of 10^8 slots (the rotating-field cascade's photon capacity) it times, with
// HIP events, the best of four launches of:
//   copy     one double column read, one written (16 bytes per slot);
//   photon   the photon kernel's columns: id, x, y, z, kx, ky, kz read, x, y, z written
//            (80 bytes per slot), x += h k for a live id;
//   lepton   the lepton kernel's columns: id, x, y, z, px, py, pz and the 4-byte event
//            count read, x..pz and the count written (112 bytes per slot);
// each with grid-stride loops of 256-thread workgroups at 4, 8, 16 and 64 workgroups per
// compute unit, and prints one line per pattern and grid with the bytes moved per second.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

struct Cols {
  unsigned long long* id;
  double *x, *y, *z, *px, *py, *pz;
  unsigned* nev;
};

__global__ void __launch_bounds__(256) fill_kernel(double* p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v + 1e-9 * (double)(i & 1023);
}

__global__ void __launch_bounds__(256) copy_kernel(const double* __restrict__ a,
                                                   double* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void __launch_bounds__(256) photon_pattern(Cols c, long long n, double h) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long id = c.id[i];
    const double kx = c.px[i], ky = c.py[i], kz = c.pz[i];
    const double x = c.x[i], y = c.y[i], z = c.z[i];
    if (id != ~0ull) {
      c.x[i] = x + h * kx;
      c.y[i] = y + h * ky;
      c.z[i] = z + h * kz;
    }
  }
}

__global__ void __launch_bounds__(256) lepton_pattern(Cols c, long long n, double h) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long id = c.id[i];
    const double px = c.px[i], py = c.py[i], pz = c.pz[i];
    const double x = c.x[i], y = c.y[i], z = c.z[i];
    const unsigned ne = c.nev[i];
    if (id != ~0ull) {
      c.x[i] = x + h * px;
      c.y[i] = y + h * py;
      c.z[i] = z + h * pz;
      c.px[i] = px * (1.0 - h);
      c.py[i] = py * (1.0 - h);
      c.pz[i] = pz * (1.0 - h);
      c.nev[i] = ne + 1u;
    }
  }
}

int main() {
  const long long n = 100000000;
  Cols c{};
  double** cols[6] = {&c.x, &c.y, &c.z, &c.px, &c.py, &c.pz};
  for (int k = 0; k < 6; ++k) CHECK(hipMalloc(cols[k], n * sizeof(double)));
  CHECK(hipMalloc(&c.id, n * sizeof(unsigned long long)));
  CHECK(hipMalloc(&c.nev, n * sizeof(unsigned)));
  double *a = nullptr, *b = nullptr;
  CHECK(hipMalloc(&a, n * sizeof(double)));
  CHECK(hipMalloc(&b, n * sizeof(double)));
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  for (int k = 0; k < 6; ++k)
    hipLaunchKernelGGL(fill_kernel, dim3(cus * 16), dim3(256), 0, 0, *cols[k], n, 1.0 + k);
  hipLaunchKernelGGL(fill_kernel, dim3(cus * 16), dim3(256), 0, 0, a, n, 3.0);
  CHECK(hipMemset(c.id, 0, n * sizeof(unsigned long long)));
  CHECK(hipMemset(c.nev, 0, n * sizeof(unsigned)));
  CHECK(hipMemset(b, 0, n * sizeof(double)));
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int per_cu[4] = {4, 8, 16, 64};
  const char* name[3] = {"copy", "photon", "lepton"};
  const double bytes[3] = {16.0, 80.0, 112.0};
  for (int kind = 0; kind < 3; ++kind) {
    for (int gi = 0; gi < 4; ++gi) {
      const dim3 grid(cus * per_cu[gi]);
      float best = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {
        CHECK(hipEventRecord(e0));
        if (kind == 0) hipLaunchKernelGGL(copy_kernel, grid, dim3(256), 0, 0, a, b, n);
        if (kind == 1) hipLaunchKernelGGL(photon_pattern, grid, dim3(256), 0, 0, c, n, 1e-3);
        if (kind == 2) hipLaunchKernelGGL(lepton_pattern, grid, dim3(256), 0, 0, c, n, 1e-3);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
      }
      std::printf("pattern=%s bytes_per_slot=%.0f slots=%lld workgroups_per_cu=%d ms=%.4f "
                  "GB/s=%.1f\n",
                  name[kind], bytes[kind], n, per_cu[gi], best, bytes[kind] * n / best / 1e6);
    }
  }
  for (int k = 0; k < 6; ++k) CHECK(hipFree(*cols[k]));
  CHECK(hipFree(c.id));
  CHECK(hipFree(c.nev));
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  return 0;
}
