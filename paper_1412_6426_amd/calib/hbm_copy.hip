// hbm_copy.hip -- reference copy kernel for calibrating HBM byte counters.
//
// Copies N doubles (N = 10^8: 800 MB read, 800 MB written per launch) with a grid-stride
// loop, five launches, and prints the event-timed bandwidth of each.  Run under
// `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE), the counters' reading for this kernel
// against its known bytes gives the factor that turns the same counters of another kernel
// into HBM bytes.
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

__global__ void __launch_bounds__(256) hbm_fill(double* p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v + 1e-9 * (double)(i & 1023);
}

__global__ void __launch_bounds__(256) hbm_copy(const double* __restrict__ a,
                                                double* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

int main() {
  const long long n = 100000000;
  double *a = nullptr, *b = nullptr;
  CHECK(hipMalloc(&a, n * sizeof(double)));
  CHECK(hipMalloc(&b, n * sizeof(double)));
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  const int grid = cus * 16;
  hipLaunchKernelGGL(hbm_fill, dim3(grid), dim3(256), 0, 0, a, n, 3.0);
  hipLaunchKernelGGL(hbm_fill, dim3(grid), dim3(256), 0, 0, b, n, 0.0);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  for (int rep = 0; rep < 5; ++rep) {
    CHECK(hipEventRecord(e0));
    hipLaunchKernelGGL(hbm_copy, dim3(grid), dim3(256), 0, 0, a, b, n);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::printf("hbm_copy bytes_read=%lld bytes_written=%lld ms=%.4f GB/s=%.1f\n",
                n * 8, n * 8, ms, 16.0 * (double)n / ms / 1e6);
  }
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  return 0;
}
