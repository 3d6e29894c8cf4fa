// Streaming probes of a known size, used to calibrate the HBM byte counters
// (FETCH_SIZE / WRITE_SIZE) and to measure what plain streaming reaches on
// the device:
//   copy   every 16-byte element read once and written once (1R1W);
//   mix31  three sources read, one destination written, dst = a + b * c:
//          the access mix of semantic mutation and crossover (3R1W);
//   mix31nt the same with non-temporal loads;
//   read   one source read, one float per thread written at the end.
// Usage: copy_probe [bytes per array] [reps] [copy|mix31|mix31nt|read] [grid]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int kUnroll = 4;

// Each thread moves kUnroll elements kBlock apart per step; every access is
// bounds-checked against n.
__global__ __launch_bounds__(kBlock) void copy_probe(const f4* __restrict__ src, f4* __restrict__ dst, size_t n) {
  const size_t step = (size_t)gridDim.x * kBlock * kUnroll;
  for (size_t base = (size_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < n; base += step) {
    f4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

__global__ __launch_bounds__(kBlock) void mix31_probe(const f4* __restrict__ a, const f4* __restrict__ b,
                                                      const f4* __restrict__ c, f4* __restrict__ dst, size_t n) {
  const size_t step = (size_t)gridDim.x * kBlock * kUnroll;
  for (size_t base = (size_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < n; base += step) {
    f4 x[kUnroll], y[kUnroll], z[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) {
        x[u] = a[i];
        y[u] = b[i];
        z[u] = c[i];
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) __builtin_nontemporal_store(x[u] + y[u] * z[u], dst + i);
    }
  }
}

__global__ __launch_bounds__(kBlock) void mix31nt_probe(const f4* __restrict__ a, const f4* __restrict__ b,
                                                      const f4* __restrict__ c, f4* __restrict__ dst, size_t n) {
  const size_t step = (size_t)gridDim.x * kBlock * kUnroll;
  for (size_t base = (size_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < n; base += step) {
    f4 x[kUnroll], y[kUnroll], z[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) {
        x[u] = __builtin_nontemporal_load(a + i);
        y[u] = __builtin_nontemporal_load(b + i);
        z[u] = __builtin_nontemporal_load(c + i);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) __builtin_nontemporal_store(x[u] + y[u] * z[u], dst + i);
    }
  }
}

__global__ __launch_bounds__(kBlock) void read_probe(const f4* __restrict__ src, float* __restrict__ out, size_t n) {
  const size_t step = (size_t)gridDim.x * kBlock * kUnroll;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (size_t base = (size_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < n; base += step) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t i = base + (size_t)u * kBlock;
      if (i < n) acc += src[i];
    }
  }
  out[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
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
  const char* mode = (argc > 3) ? argv[3] : "copy";
  const unsigned grid = (argc > 4) ? (unsigned)std::strtoul(argv[4], nullptr, 10) : 32768u;
  const int kind = !std::strcmp(mode, "copy") ? 0 : !std::strcmp(mode, "mix31") ? 1 : !std::strcmp(mode, "read") ? 2 : !std::strcmp(mode, "mix31nt") ? 3 : -1;
  if (kind < 0 || reps < 1 || grid < 1 || grid > 65536 || bytes < sizeof(f4)) {
    std::fprintf(stderr, "usage: copy_probe [bytes] [reps>=1] [copy|mix31|mix31nt|read] [grid 1..65536]\n");
    return 2;
  }
  const size_t n = bytes / sizeof(f4);
  const int nsrc = (kind == 1 || kind == 3) ? 3 : 1;
  f4* src[3] = {nullptr, nullptr, nullptr};
  f4* dst = nullptr;
  float* out = nullptr;
  for (int s = 0; s < nsrc; ++s) {
    CHECK(hipMalloc(&src[s], n * sizeof(f4)));
    CHECK(hipMemset(src[s], 0, n * sizeof(f4)));
  }
  if (kind == 2) {
    CHECK(hipMalloc(&out, (size_t)grid * kBlock * sizeof(float)));
  } else {
    CHECK(hipMalloc(&dst, n * sizeof(f4)));
    CHECK(hipMemset(dst, 0, n * sizeof(f4)));
  }
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(copy_probe, dim3(grid), dim3(kBlock), 0, 0, src[0], dst, n);
    else if (kind == 1)
      hipLaunchKernelGGL(mix31_probe, dim3(grid), dim3(kBlock), 0, 0, src[0], src[1], src[2], dst, n);
    else if (kind == 3)
      hipLaunchKernelGGL(mix31nt_probe, dim3(grid), dim3(kBlock), 0, 0, src[0], src[1], src[2], dst, n);
    else
      hipLaunchKernelGGL(read_probe, dim3(grid), dim3(kBlock), 0, 0, src[0], out, n);
  };
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  launch();
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < reps; ++r) launch();
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const size_t rd = (size_t)nsrc * n * sizeof(f4), wr = kind == 2 ? 0 : n * sizeof(f4);
  std::printf("%s_probe grid=%u bytes_per_launch_read=%zu bytes_per_launch_written=%zu ms_per_launch=%.4f GBps=%.1f\n",
              mode, grid, rd, wr, ms / reps, (double)(rd + wr) * reps / (ms * 1e-3) / 1e9);
  for (int s = 0; s < nsrc; ++s) CHECK(hipFree(src[s]));
  if (dst) CHECK(hipFree(dst));
  if (out) CHECK(hipFree(out));
  return 0;
}
