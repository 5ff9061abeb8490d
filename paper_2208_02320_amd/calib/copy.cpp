// Plain device-to-device copy of a known size, used to calibrate the HBM
// byte counters of rocprofv3 (FETCH_SIZE / WRITE_SIZE) and as the practical
// bandwidth reference for the solver passes.  One 16-byte load and one store
// per thread; prints the achieved read+write rate.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ void __launch_bounds__(256) copy16(const float4* __restrict__ a, float4* __restrict__ b, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

#define CK(x)                                                                    \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));        \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

int main(int argc, char** argv) {
  const long long mib = argc > 1 ? std::atoll(argv[1]) : 1024;
  const long long bytes = mib << 20, n = bytes / 16;
  float4 *a = nullptr, *b = nullptr;
  CK(hipMalloc(&a, bytes));
  CK(hipMalloc(&b, bytes));
  CK(hipMemset(a, 0, bytes));
  CK(hipMemset(b, 0, bytes));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const long long blocks = (n + 255) / 256;
  for (int w = 0; w < 2; ++w) copy16<<<blocks, 256>>>(a, b, n);
  CK(hipGetLastError());
  const int reps = 10;
  CK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) copy16<<<blocks, 256>>>(a, b, n);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  ms /= reps;
  std::printf("copy %lld MiB: %.4f ms per launch, %.1f GB/s read+write, %lld bytes read and written per launch\n",
              mib, ms, 2.0 * bytes / ms / 1e6, bytes);
  CK(hipFree(a));
  CK(hipFree(b));
  return 0;
}
