// Device helpers shared by the HIP translation units of libgsgp.so
// (kernels.hip: genomes, variation, fitness, survival, reconstruction;
// interp.hip: genome compiler and interpreter).  Internal, not part of the
// ABI.
#pragma once

#include <float.h>
#include <math.h>

#include <type_traits>

#include "common.hpp"

namespace gsgp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

template <typename T>
struct VecOf;
template <>
struct VecOf<float> {
  typedef f4 type;
  static constexpr int N = 4;
};
template <>
struct VecOf<double> {
  typedef d2 type;
  static constexpr int N = 2;
};

constexpr double kFltMax = 3.4028234663852886e38;  // largest finite binary32 value

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Buffers reach the kernels through RunDev as generic pointers; casting to
// the global address space lets the compiler emit global (not flat) memory
// instructions, the constant address space gives scalar loads for data no
// kernel in flight writes (records, compiled programs, generation counter),
// and the local address space gives LDS instructions for shared memory.
#define GSGP_GLOBAL __attribute__((address_space(1)))
#define GSGP_CONST __attribute__((address_space(4)))
#define GSGP_LDS __attribute__((address_space(3)))

template <typename VT>
__device__ __forceinline__ VT gload(const void* p) {
  return *(const GSGP_GLOBAL VT*)p;
}

template <typename VT>
__device__ __forceinline__ void gstore_nt(const VT& v, void* p) {
  __builtin_nontemporal_store(v, (GSGP_GLOBAL VT*)p);
}

template <typename X>
__device__ __forceinline__ X cload(const X* p) {
  return *(const GSGP_CONST X*)p;
}


// ---------------------------------------------------------------------------
// Run lookup: runs are laid out in launch order; find the last run whose
// first task is <= t.  Single-run launches skip the search.
template <typename F>
__device__ __forceinline__ int find_run(int n_runs, int64_t t, F first_of) {
  if (n_runs == 1) return 0;
  int lo = 0, hi = n_runs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first_of(mid) <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace
}  // namespace gsgp
