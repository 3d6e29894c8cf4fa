// Plain device-to-device copy of a known size, used to calibrate the HBM
// byte counters (FETCH_SIZE / WRITE_SIZE) and to measure copy bandwidth on
// the device: every 16-byte element is read once and written once.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void copy_probe(const f4* __restrict__ src, f4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) __builtin_nontemporal_store(src[i], dst + i);
}

#define CHECK(x)                                                             \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
      return 1;                                                              \
    }                                                                        \
  } while (0)

int main(int argc, char** argv) {
  const size_t bytes = (argc > 1) ? std::strtoull(argv[1], nullptr, 10) : ((size_t)1 << 30);
  const int reps = (argc > 2) ? std::atoi(argv[2]) : 10;
  const size_t n = bytes / sizeof(f4);
  f4 *a = nullptr, *b = nullptr;
  CHECK(hipMalloc(&a, n * sizeof(f4)));
  CHECK(hipMalloc(&b, n * sizeof(f4)));
  CHECK(hipMemset(a, 0, n * sizeof(f4)));
  CHECK(hipMemset(b, 0, n * sizeof(f4)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const unsigned grid = 4096;
  hipLaunchKernelGGL(copy_probe, dim3(grid), dim3(256), 0, 0, a, b, n);
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(copy_probe, dim3(grid), dim3(256), 0, 0, a, b, n);
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  std::printf("copy_probe bytes_per_launch_read=%zu bytes_per_launch_written=%zu ms_per_launch=%.4f GBps=%.1f\n",
              n * sizeof(f4), n * sizeof(f4), ms / reps, 2.0 * n * sizeof(f4) * reps / (ms * 1e-3) / 1e9);
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  return 0;
}
