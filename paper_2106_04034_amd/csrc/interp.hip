// The genome compiler and the stack-machine interpreter of libgsgp.so
// (ComputeSemantics of Algorithm 1; Section 2.2 "Interpreter" of the
// GSGP-CUDA paper, arXiv 2106.04034), for gfx950:
//   k_compile         one thread per genome: drops the functions the
//                     interpreter would skip and the pushes after the last
//                     function, fuses each push with a function that
//                     directly consumes it, and records every op's stack
//                     depth; k_order files the programs into lists by stack
//                     need, longest first;
//   k_interpret_wide  one wavefront per (program, 256 or 128 cases), four
//                     or two cases per lane: the compiled program is
//                     wave-uniform (no divergence), the top two stack values
//                     live in registers and the rest in a lane-strided LDS
//                     column sized for the list;
//   k_interpret       the same evaluator with LDS columns up to 63 values
//                     (deeper programs); k_interpret_spill beyond;
//   k_interpret_list  given programs on new cases (lineage reconstruction).
// This translation unit is built with
// -structurizecfg-skip-uniform-regions: the interpreter dispatches every op
// on wave-uniform bits, and those branches stay plain scalar branches.  The
// other kernels are built without it (it made the variation kernel about
// 0.5 % slower).
#include "device.hpp"

namespace gsgp {
namespace {

// End of a compiled program for eval_program_wide: a push-class word with
// bit 1 set (a push uses only bit 0).
constexpr int32_t kOpEnd = 2;

// Division (the protected division of Section 2.2: a / b where |b| >= 1e-6).
// The FP64 division the compiler emits is a reciprocal estimate refined by
// two Newton-Raphson steps, a quotient, and one correction by its residual,
// all with FMA, inside an operand range scaling and a special-case fix-up.
// When |b| lies in [1e-6, 2^128], |a| >= 2^-700 and the quotient is at most
// 2^127 in magnitude, no operand, reciprocal or quotient comes near either
// end of the exponent range, so the scaling and the fix-up leave every value
// as it is and the core steps alone (div_recip, div_short) give the same
// bits.  The reciprocal depends on b alone: for a constant divisor the
// compile step refines it once.
constexpr double kDivShortMinDivisor = 1e-6;
constexpr double kDivShortMaxDivisor = 0x1p128;
constexpr double kDivShortMinDividend = 0x1p-700;
constexpr double kDivShortMaxQuotient = 0x1p127;

__device__ __forceinline__ double div_recip(double b) {
  double y = __builtin_amdgcn_rcp(b);
  double e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  e = fma(-b, y, 1.0);
  return fma(y, e, y);
}

__device__ __forceinline__ double div_short(double a, double b, double y) {
  const double q = a * y;
  const double r = fma(-b, q, a);
  return fma(r, y, q);
}

// Compile a genome: drop the functions the stack machine would skip (fewer
// than two operands) and everything after the last function that runs, and
// store each op's stack depth so the interpreter needs no depth counter.
// One thread per genome, one wave per block of 64 genomes of one run; also
// records the deepest stack per run.  The wave stages its genomes' codes
// and constants in LDS kCompileChunk genes at a time with coalesced loads
// (a genome row per load instruction), so each thread walks its genome
// from LDS instead of with one scattered load per gene.
constexpr int kCompileChunk = 64;

__global__ __launch_bounds__(kWave) void k_compile(const RunDev* __restrict__ runs, Params p, int32_t groups) {
  __shared__ int32_t s_code[kWave][kCompileChunk + 1];
  __shared__ double s_cval[kWave][kCompileChunk + 1];
  const int lane = threadIdx.x;
  const int rows = p.m + p.r;
  const int run = blockIdx.x / groups;
  const int prog0 = (blockIdx.x - run * groups) * kWave;
  const int prog = prog0 + lane;
  const bool mine = prog < rows;
  const RunDev& R = runs[run];
  int32_t* ops = R.ops + (int64_t)prog * p.k;
  double* opv = R.opv + (int64_t)prog * p.k;
  double* opy = R.opy + (int64_t)prog * p.k;
  // deepest: the deepest stack up to the last valid function; pushes after
  // it are dropped and never run, so they do not count
  int depth = 0, n = 0, last = 0, deepest = 0, peak = 0;
  int32_t prev = 0;   // the last op word written, ops[n - 1]
  double prevv = 0;   // and its constant slot, opv[n - 1]
  for (int q0 = 0; q0 < p.k; q0 += kCompileChunk) {
    const int len = p.k - q0 < kCompileChunk ? p.k - q0 : kCompileChunk;
    __syncthreads();  // the previous chunk is consumed
    for (int i = 0; i < kWave && prog0 + i < rows; ++i) {
      if (lane < len) {
        const int64_t at = (int64_t)(prog0 + i) * p.k + q0 + lane;
        s_code[i][lane] = R.code[at];
        s_cval[i][lane] = R.cval[at];
      }
    }
    __syncthreads();
    if (!mine) continue;
    for (int u = 0; u < len; ++u) {
      const int32_t c = s_code[lane][u];
      // depths before the last function are at most k - 1 <= kOpDepthMax, and
      // ops after the last function never run; the cap only keeps the field
      // inside its bits
      const int dfield = (depth < kOpDepthMax ? depth : kOpDepthMax) << 4;
      if (c >= 0) {
        prev = (kClsPush << 2) | kPushFeature | dfield | (c << 16);
        // the byte offset of the feature's row in a tile of this run's X,
        // bit for bit (see eval_program)
        prevv = __longlong_as_double((long long)((int64_t)c * kXTile * (int64_t)sizeof(double)));
        ops[n] = prev;
        opv[n] = prevv;
        opy[n] = 0.0;
        ++n;
        ++depth;
      } else if (c == -5) {
        prev = (kClsPush << 2) | kPushConst | dfield;
        prevv = s_cval[lane][u];
        ops[n] = prev;
        opv[n] = prevv;
        opy[n] = 0.0;
        ++n;
        ++depth;
      } else {
        if (depth < 2) continue;  // skipped by the interpreter
        const int fn = -1 - c;
        if (n > 0 && ((prev >> 2) & 3) == kClsPush) {
          // push b, then op(a, b) with a the value below it: one op on the
          // top of the stack; the depth field stays the one before the push,
          // the feature index and the constant stay where the push put them
          const int cls = (prev & 3) == kPushConst ? kClsConst : kClsFeature;
          prev = (prev & ~0xF) | (cls << 2) | fn;
          ops[n - 1] = prev;
          if (cls == kClsConst && fn == kFnDiv) {
            // a constant divisor in the short division's range: its
            // reciprocal refinement, once (0 selects the full division)
            const double ab = fabs(prevv);
            opy[n - 1] = ab >= kDivShortMinDivisor && ab <= kDivShortMaxDivisor ? div_recip(prevv) : 0.0;
          }
        } else {
          prev = (kClsStack << 2) | fn | dfield;
          prevv = 0.0;
          ops[n] = prev;
          opv[n] = 0.0;
          opy[n] = 0.0;
          ++n;
        }
        --depth;
        last = n;
        deepest = peak;
      }
      peak = depth > peak ? depth : peak;
    }
  }
  // the run's deepest stack: one atomic per wave (one per genome put every
  // genome of a run on one address, serialised at one L2 channel)
  int dmax = mine ? deepest : 0;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int other = __shfl_xor(dmax, o);
    dmax = other > dmax ? other : dmax;
  }
  if (lane == 0) atomicMax(&R.state[kStMaxDepth], dmax);
  if (!mine) return;
  R.nops[prog] = last;
  // the end word of eval_program_wide: a program with a valid function
  // starts with a push fused into it, so last <= k - 1 and the word stays in
  // the program's row (a program without one gets it at 0)
  ops[last] = kOpEnd;
  const int need = deepest > 2 ? deepest - 2 : 0;  // the top two values live in registers
  R.need[prog] = need;
}

// Files each run's programs into the stack-need lists, each list in order
// of decreasing length (a counting sort on kOrderBins length bins, one block
// per run): the long programs of a case block start first and the launch
// ends on short ones (3.5 % faster at the Section 3.1 shape).  The order
// within a bin is arbitrary; semantics do not depend on it.
constexpr int kOrderBins = 256;
__global__ __launch_bounds__(1024) void k_order(const RunDev* __restrict__ runs, Params p, int shift) {
  __shared__ int32_t at[kLists * kOrderBins];
  const RunDev& R = runs[blockIdx.x];
  const int rows = p.m + p.r;
  auto key = [&](int prog, int& list) {
    list = list_of(R.need[prog]);
    return list * kOrderBins + ((p.k - R.nops[prog]) >> shift);
  };
  for (int i = threadIdx.x; i < kLists * kOrderBins; i += blockDim.x) at[i] = 0;
  __syncthreads();
  for (int prog = threadIdx.x; prog < rows; prog += blockDim.x) {
    int list;
    atomicAdd(&at[key(prog, list)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kLists) {  // bin counts to first positions, per list
    int32_t* h = at + threadIdx.x * kOrderBins;
    int32_t sum = 0;
    for (int j = 0; j < kOrderBins; ++j) {
      const int32_t c = h[j];
      h[j] = sum;
      sum += c;
    }
    R.state[kStList0 + threadIdx.x] = sum;
  }
  __syncthreads();
  for (int prog = threadIdx.x; prog < rows; prog += blockDim.x) {
    int list;
    const int slot = atomicAdd(&at[key(prog, list)], 1);
    R.lists[(int64_t)list * rows + slot] = prog;
  }
}

// Evaluate one compiled program on V cases per lane (Section 2.2
// "Interpreter").  The op stream is wave-uniform and read with scalar loads,
// eight ops per batch in one load of words and one of constants.  Stack
// element i of depth d (0 = bottom) lives in
// registers for the top two (tos = d-1, nos = d-2) and in LDS below them,
// at stk[(i * V + v) * 64 + lane]; a function of the top two values reads
// its new second operand from LDS only after it has produced its result, so
// the LDS latency falls outside the op's dependency chain.  A fused op (a
// push the next function consumes) applies the function to tos and the
// terminal and touches neither nos nor LDS.  The value of the program is the
// output of its last function (the Out register), 0.0 if none runs.
// This form serves the list interpreter (programs on a caller's cases): X is
// feature-major in global memory, row stride ld, and a feature op's index
// sits in its op word.
typedef GSGP_LDS double* LdsStack;        // stack column in LDS
typedef GSGP_GLOBAL double* GlobalStack;  // stack column in the workspace (spill pass)

template <int V, typename Stack>
__device__ __forceinline__ void eval_program(const int32_t* ops, const double* opv, int n, const double* X,
                                             int64_t ld, const int64_t (&col)[V], const bool (&ok)[V],
                                             Stack stk, int lane, double (&out)[V]) {
  constexpr int kBatch = kOpPad;
  const GSGP_CONST int32_t* cops = (const GSGP_CONST int32_t*)ops;
  const GSGP_CONST double* copv = (const GSGP_CONST double*)opv;
  double tos[V], nos[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    tos[v] = 0.0;
    nos[v] = 0.0;
  }
  // lanes past the last column read the last column instead (no exec-mask
  // branches around the loads); their values are never stored
  int64_t at[V];
#pragma unroll
  for (int v = 0; v < V; ++v) at[v] = ok[v] ? col[v] : ld - 1;
  auto feature = [&](int w, double (&x)[V]) {
    const GSGP_GLOBAL double* xg = (const GSGP_GLOBAL double*)X + (int64_t)((uint32_t)w >> 16) * ld;
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = xg[at[v]];
  };
  for (int j0 = 0; j0 < n; j0 += kBatch) {
    int wv[kBatch];
    double cv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      // one contiguous batch (two scalar loads); the last batch of a program
      // may read up to kBatch - 1 words past it, which the buffers' padding
      // after the last program keeps in bounds, and never uses them
      wv[u] = cops[j0 + u];
      cv[u] = copv[j0 + u];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (j0 + u >= n) break;
      const int w = wv[u];
      const int cls = (w >> 2) & 3;
      const int fn = w & 3;
      const int d = (w >> 4) & kOpDepthMax;  // stack depth before the op
      if (cls == kClsPush) {
        if (d >= 2) {
#pragma unroll
          for (int v = 0; v < V; ++v) stk[((d - 2) * V + v) * kWave + lane] = nos[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) nos[v] = tos[v];
        if (fn == kPushFeature) {
          feature(w, tos);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) tos[v] = cv[u];
        }
      } else {
        // op(a, b): b is the top of the stack (or the fused terminal), a the
        // value below it (or the top of the stack).  The two forms are
        // separate call sites of `apply`, so neither first copies its
        // operands into a common pair of registers.
        // Every operand is finite (finite features and constants, results
        // clamped here, protected division), so min/max clamp exactly as a
        // compare-and-select would.  The clamp sits in each branch, on the
        // arithmetic result itself, where the compiler knows the value needs
        // no NaN canonicalisation before min/max.
        auto clamp = [](double x) { return fmin(fmax(x, -kFltMax), kFltMax); };
        auto apply = [&](const double (&a)[V], const double (&b)[V]) {
          if (fn == kFnAdd) {
#pragma unroll
            for (int v = 0; v < V; ++v) tos[v] = clamp(a[v] + b[v]);
          } else if (fn == kFnSub) {
#pragma unroll
            for (int v = 0; v < V; ++v) tos[v] = clamp(a[v] - b[v]);
          } else if (fn == kFnMul) {
#pragma unroll
            for (int v = 0; v < V; ++v) tos[v] = clamp(a[v] * b[v]);
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
              // protected division without a per-lane branch: the quotient
              // of a safe denominator is kept only where |b| >= 1e-6, and
              // there it is a / b
              const bool tiny = fabs(b[v]) < 1e-6;
              const double q = a[v] / (tiny ? 1.0 : b[v]);
              tos[v] = clamp(tiny ? 1.0 : q);
            }
          }
        };
        if (cls == kClsStack) {
          double t0[V];
#pragma unroll
          for (int v = 0; v < V; ++v) t0[v] = tos[v];
          apply(nos, t0);
        } else {
          double x[V], t0[V];
#pragma unroll
          for (int v = 0; v < V; ++v) t0[v] = tos[v];
          if (cls == kClsFeature) {
            feature(w, x);
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = cv[u];
          }
          apply(t0, x);
        }
        if (cls == kClsStack && d >= 3) {
#pragma unroll
          for (int v = 0; v < V; ++v) nos[v] = stk[((d - 3) * V + v) * kWave + lane];
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) out[v] = tos[v];
}

// The interpreter passes over the handle's X: eval_program for V cases per
// lane, written to keep the work per op small.
//   - Dispatch tests single bits of the op word: bit 3 a function applied
//     to the top of the stack and a terminal (fused op), else bit 2 a
//     function of the top two values, else a push; bit 1 multiplication or
//     division, bit 0 subtraction or division (or, for a push, a constant).
//   - A feature op's constant slot holds the byte offset of its row in an X
//     tile.  Features are read through a buffer resource over the block's
//     tile: the scalar offset is the row's offset and each lane's fixed
//     32-bit byte offset (its pair of cases) is the vector offset, so a
//     feature load takes no vector address arithmetic.
//   - Both function forms share one `apply` (tos = f(tos, b)): a function of
//     the top two values first moves them into place.
//   - The program ends at its end word (kOpEnd), tested only on the push
//     path, instead of a count compared before every op.
//   - REG = 1 keeps a third stack value (n2, element d - 3) in registers as
//     well, so that a program needs one LDS value per lane fewer (the LDS
//     column is what bounds the resident waves of the deeper lists).
// The FP64 operations and their order are those of eval_program, so results
// are the same bits.
template <int V, int REG, typename Stack>
__device__ __forceinline__ void eval_program_wide(const int32_t* ops, const double* opv, const double* opy,
                                                  const double* X, bool short_feature_div,
                                                  const uint32_t (&off)[V], Stack stk, int lane, double (&out)[V]) {
  static_assert(REG == 0 || REG == 1, "two or three stack values in registers");
  constexpr int kBatch = kOpPad;
  const GSGP_CONST int32_t* cops = (const GSGP_CONST int32_t*)ops;
  const GSGP_CONST double* copv = (const GSGP_CONST double*)opv;
  const GSGP_CONST double* copy = (const GSGP_CONST double*)opy;
  double tos[V], nos[V], n2[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    tos[v] = 0.0;
    nos[v] = 0.0;
    n2[v] = 0.0;
  }
  // raw buffer over X: no stride, num_records at the largest offset, and the
  // third descriptor word of a plain dword buffer on gfx9-family parts
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, 0x7fffffff, 0x00020000);
  // cases v and v + 1 (v even) of a lane are adjacent: one 16-byte load.
  // The vector memory unit, busy nearly all the time here, costs about the
  // same per instruction for 8 or 16 bytes a lane, so pairs halve its time
  // (10 % faster at the Section 3.1 shape with 127 genes, 14 % with 2,047).
  auto feature = [&](double c, double (&x)[V]) {
    const int row = (int)__double_as_longlong(c);  // the row's byte offset in the tile
#pragma unroll
    for (int v = 0; v < V; v += 2) {
      typedef double double2v __attribute__((ext_vector_type(2)));
      const double2v t = __builtin_bit_cast(double2v, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)off[v], row, 0));
      x[v] = t.x;
      x[v + 1] = t.y;
    }
  };
  auto clamp = [](double x) { return fmin(fmax(x, -kFltMax), kFltMax); };
  // The clamp changes nothing where |x| <= FLT_MAX: one compare per case,
  // and the min/max only when some case of the wave needs them (NaN, which
  // finite operands never produce, takes them too).
  auto settle = [&]() {
    uint64_t out_of_range = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) out_of_range |= __builtin_amdgcn_ballot_w64(!(fabs(tos[v]) <= kFltMax));
    if (out_of_range) {
#pragma unroll
      for (int v = 0; v < V; ++v) tos[v] = clamp(tos[v]);
    }
  };
  auto divide_full = [&](const double (&b)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const bool tiny = fabs(b[v]) < 1e-6;  // protected division, as in eval_program
      const double q = tos[v] / (tiny ? 1.0 : b[v]);
      tos[v] = clamp(tiny ? 1.0 : q);
    }
  };
  // The short division (div_short): taken when every case of the wave has
  // |b| >= 1e-6 (with y its reciprocal refinement), |tos| >= 2^-700 and a
  // quotient of at most 2^127, where it gives the bits of the full one.
  auto divide = [&](const double (&b)[V], const double (&y)[V], uint64_t bad) {
    double q[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      q[v] = div_short(tos[v], b[v], y[v]);
      bad |= __builtin_amdgcn_ballot_w64(!(fabs(tos[v]) >= kDivShortMinDividend)) |
             __builtin_amdgcn_ballot_w64(!(fabs(q[v]) <= kDivShortMaxQuotient));
    }
    if (bad) {
      divide_full(b);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) tos[v] = q[v];
    }
  };
  // a divisor from the registers: every case refines its own reciprocal
  auto divide_by = [&](const double (&b)[V]) {
    double y[V];
    uint64_t bad = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      y[v] = div_recip(b[v]);
      bad |= __builtin_amdgcn_ballot_w64(!(fabs(b[v]) >= kDivShortMinDivisor));
    }
    divide(b, y, bad);
  };
  auto arith = [&](int w, const double (&b)[V]) {
    if (w & 2) {
#pragma unroll
      for (int v = 0; v < V; ++v) tos[v] = tos[v] * b[v];
    } else if (w & 1) {
#pragma unroll
      for (int v = 0; v < V; ++v) tos[v] = tos[v] - b[v];
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) tos[v] = tos[v] + b[v];
    }
    settle();
  };
  for (int j0 = 0;; j0 += kBatch) {
    int wv[kBatch];
    double cv[kBatch], yv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      // one batch per three scalar loads; reads past a program's end word
      // stay inside the buffers' padding and are never used
      wv[u] = cops[j0 + u];
      cv[u] = copv[j0 + u];
      yv[u] = copy[j0 + u];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int w = wv[u];
      if (w & 8) {  // fused: tos = f(tos, terminal)
        double b[V];
        if (w & 4) {
#pragma unroll
          for (int v = 0; v < V; ++v) b[v] = cv[u];
          if ((w & 3) != kFnDiv) {
            arith(w, b);
          } else if (__double_as_longlong(yv[u]) != 0) {
            // the compile step refined the constant's reciprocal (and
            // checked the constant's range)
            double y[V];
#pragma unroll
            for (int v = 0; v < V; ++v) y[v] = yv[u];
            divide(b, y, 0);
          } else {
            divide_full(b);
          }
        } else {
          feature(cv[u], b);
          if ((w & 3) != kFnDiv)
            arith(w, b);
          else if (short_feature_div)
            divide_by(b);
          else
            divide_full(b);
        }
      } else if (w & 4) {  // tos = f(nos, tos), then the new nos from LDS
        double b[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          b[v] = tos[v];
          tos[v] = nos[v];
        }
        // b is the output of a function, so |b| <= FLT_MAX
        if ((w & 3) != kFnDiv)
          arith(w, b);
        else
          divide_by(b);
        const int d = (w >> 4) & kOpDepthMax;
        if constexpr (REG == 0) {
          if (d >= 3) {
#pragma unroll
            for (int v = 0; v < V; ++v) nos[v] = stk[((d - 3) * V + v) * kWave + lane];
          }
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) nos[v] = n2[v];
          if (d >= 4) {
#pragma unroll
            for (int v = 0; v < V; ++v) n2[v] = stk[((d - 4) * V + v) * kWave + lane];
          }
        }
      } else {  // push: the lowest register value to LDS, the rest down one, the terminal to tos
        if (w & 2) goto done;  // kOpEnd
        const int d = (w >> 4) & kOpDepthMax;
        if constexpr (REG == 0) {
          if (d >= 2) {
#pragma unroll
            for (int v = 0; v < V; ++v) stk[((d - 2) * V + v) * kWave + lane] = nos[v];
          }
        } else {
          if (d >= 3) {
#pragma unroll
            for (int v = 0; v < V; ++v) stk[((d - 3) * V + v) * kWave + lane] = n2[v];
          }
#pragma unroll
          for (int v = 0; v < V; ++v) n2[v] = nos[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) nos[v] = tos[v];
        if (w & 1) {
#pragma unroll
          for (int v = 0; v < V; ++v) tos[v] = cv[u];
        } else {
          feature(cv[u], tos);
        }
      }
    }
  }
done:
#pragma unroll
  for (int v = 0; v < V; ++v) out[v] = tos[v];
}

constexpr int kInterpV = 2;              // cases per lane
constexpr int kInterpTile = kWave * kInterpV;  // cases per block
static_assert(kInterpTile == kInterpCases, "the runtime plans kInterpCases-case blocks");
// Programs each wave interprets on its case block.  One per wave keeps the
// last waves of a launch from holding up its end when programs are long
// (k = 2,047 at the Section 3.1 shape: 425 ms with one per wave, 449 with
// four, 468 with eight; k = 127: 29.8 / 30.4 / 31.1 ms) and costs about 1 %
// on 2,048 programs x 125,000 cases (4.1 against 4.0 ms).  Taking the
// count as a launch argument instead of a constant cost 3 %.
constexpr int kInterpProgsPerWave = 1;

// Hardware dispatch sends block b of a grid of n to XCD b % 8.  Interpreter
// blocks are numbered case block by case block; xcd_block gives each XCD a
// contiguous range of them, so the CUs of one XCD work on the same X tile
// and each tile is read into one XCD's L2, not into all eight.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t x = b & 7, i = b >> 3, q = n >> 3, rem = n & 7;
  return x * q + (x < rem ? x : rem) + i;
}

// The cases of a lane in a block of 64 x V cases starting at case `first`
// (a multiple of 64 x V inside one X tile): lane l owns cases 2l and 2l + 1
// (and, for V = 4, 128 + 2l and 129 + 2l), so that each pair is one 16-byte
// load; off[v] is the case's byte offset in its row of the X tile.
template <int V>
__device__ __forceinline__ void lane_cases(int64_t first, int lane, int64_t ld, int64_t (&col)[V], bool (&ok)[V],
                                           uint32_t (&off)[V]) {
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = (v >> 1) * (2 * kWave) + 2 * lane + (v & 1);
    col[v] = first + c;
    ok[v] = col[v] < ld;
    off[v] = (uint32_t)((first % kXTile + c) * sizeof(double));
  }
}

// Writes one program's values for one case block: population rows as they
// are, pool rows squashed by the logistic function (the random functions R_u
// of GSM, Section 2); padding columns as exact zeros.
template <typename T, int V>
__device__ __forceinline__ void store_program(const RunDev& R, const Params& p, int prog, const int64_t (&col)[V],
                                              const bool (&ok)[V], const double (&out)[V]) {
  const bool pool = prog >= p.m;
  T* dst = pool ? (T*)R.sigR : (T*)R.S[0];
  const int64_t nrows = pool ? p.r : p.m;
  const int64_t row = pool ? prog - p.m : prog;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    if (!ok[v]) continue;
    const int64_t c = col[v];
    const bool real = c < R.n_train || (c >= R.tr_pad && c < R.tr_pad + R.n_test);
    double val = out[v];
    if (pool) val = 1.0 / (1.0 + exp(-val));
    dst[tiled_index(R.tr_pad, R.te_pad, R.nch_tr, chunk_cases(sizeof(T)), nrows, row, c)] = real ? (T)val : (T)0;
  }
}

// ComputeSemantics(P) and ComputeSemantics(R) (Algorithm 1).  A block takes
// one block of 128 cases of one run and a group of programs of one
// stack-need list; each wave interprets kInterpProgsPerWave programs on the
// block's cases.  The LDS stack column of a wave bounds how many waves a CU
// holds, and the kernel is latency-bound, so each list runs in a pass of
// its own with a column sized for it.  Pool rows
// are squashed by the logistic function (the random functions R_u of GSM,
// Section 2) before storage.  Padding columns are written as exact zeros.
// (Staging the case block's features in LDS was slower: the tile cut the
// number of resident waves more than it saved in L2 reads.)
template <typename T>
__global__ __launch_bounds__(256) void k_interpret(const RunDev* __restrict__ runs, Params p, int32_t pgroups,
                                                   int lo, int slots, int list) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int W = blockDim.x >> 6;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t cbg = blk / pgroups;  // case block over all runs
  const int pg = (int)(blk - cbg * pgroups);
  const int run = find_run(p.n_runs, cbg, [&](int r) { return runs[r].cblk0; });
  const RunDev& R = runs[run];
  const int64_t cb = cbg - R.cblk0;
  const int rows = p.m + p.r;
  double* stk = lds + wave * slots * kInterpV * kWave;
  const int64_t first = cb * kInterpTile;
  int64_t col[kInterpV];
  bool ok[kInterpV];
  uint32_t off[kInterpV];
  lane_cases<kInterpV>(first, lane, R.ld, col, ok, off);
  for (int j = 0; j < kInterpProgsPerWave; ++j) {
    const int idx = (pg * kInterpProgsPerWave + j) * W + wave;
    if (idx >= uni(cload(&R.state[kStList0 + list]))) break;
    const int prog = uni(cload(&R.lists[(int64_t)list * rows + idx]));
    // this pass takes the programs with lo < need <= slots (the list holds
    // no other; the test keeps every stack inside the column regardless)
    const int need = uni(cload(&R.need[prog]));
    if (need <= lo || need > slots) continue;
    double out[kInterpV];
    eval_program_wide<kInterpV, 0>(R.ops + (int64_t)prog * p.k, R.opv + (int64_t)prog * p.k,
                                R.opy + (int64_t)prog * p.k, R.X + (first / kXTile) * R.l * kXTile,
                                uni(R.x_big) == 0, off, (LdsStack)stk, lane, out);
    store_program<T, kInterpV>(R, p, prog, col, ok, out);
  }
}

// ComputeSemantics with eval_program_wide: a block of one wave takes one
// block of 64 x V cases of one run (each lane owns V of them) and one
// program of a stack-need list; the wave's LDS column holds SLOTS stack
// values per lane.  The pass takes the list's programs with lo < need <=
// SLOTS.  One wave per block: a block's LDS and slot are released as soon
// as its program is done, where four waves of unequal programs held them
// until the longest ended (3 % faster at the Section 3.1 shape, 7 % on 256
// small runs).  V = 4 (256 cases) for the shallow lists, V = 2 (128 cases)
// for the deepest, whose LDS column bounds the resident waves (each stack
// value costs V x 512 bytes of LDS per wave).  A block's cases lie in one
// tile of X: the
// feature loads go through a buffer over that tile, with the row's byte
// offset as the scalar offset and the lane's column as the vector offset
// (lanes past the last case read the tile's padding and are never stored).
static_assert(kXTile == 4 * kWave && kXTile % kInterpTile == 0, "interpreter case blocks lie inside one X tile");
static_assert(65535LL * kXTile * sizeof(double) < (1LL << 31), "a tile of the most features the runtime accepts "
                                                                  "takes 32-bit buffer offsets");

template <typename T, int SLOTS, int V, int REG>
__global__ __launch_bounds__(kWave) void k_interpret_wide(const RunDev* __restrict__ runs, Params p, int32_t pgroups,
                                                          int lo, int list) {
  static_assert(V == 2 || V == 4, "two or four cases per lane");
  constexpr int kTile = kWave * V;
  __shared__ double lds[(SLOTS - REG) * V * kWave];
  const int lane = threadIdx.x & 63;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t cbg = blk / pgroups;  // case block over all runs
  const int pg = (int)(blk - cbg * pgroups);
  const int run = find_run(p.n_runs, cbg, [&](int r) { return V == 4 ? runs[r].cblk0w : runs[r].cblk0; });
  const RunDev& R = runs[run];
  const int64_t cb = cbg - (V == 4 ? R.cblk0w : R.cblk0);
  if (pg >= uni(cload(&R.state[kStList0 + list]))) return;
  const int prog = uni(cload(&R.lists[(int64_t)list * (p.m + p.r) + pg]));
  const int need = uni(cload(&R.need[prog]));
  if (need <= lo || need > SLOTS) return;
  const int64_t first = cb * kTile;  // the block's first case
  int64_t col[V];
  bool ok[V];
  uint32_t off[V];
  lane_cases<V>(first, lane, R.ld, col, ok, off);
  double out[V];
  eval_program_wide<V, REG>(R.ops + (int64_t)prog * p.k, R.opv + (int64_t)prog * p.k, R.opy + (int64_t)prog * p.k,
                       R.X + (first / kXTile) * R.l * kXTile, uni(R.x_big) == 0, off, (LdsStack)lds, lane, out);
  store_program<T, V>(R, p, prog, col, ok, out);
}

// Last pass: the programs of the last list whose stack exceeds the largest
// LDS column (need > kMaxLdsSlots).  kSpillWaves waves, one per block, each own
// a column of `slots` x kInterpV x 64 doubles in `spill` (lane-strided as in
// LDS, so every stack access is one coalesced 512-byte row) and sweep the
// (program, case block) tasks of every run in turn.
template <typename T>
__global__ __launch_bounds__(64) void k_interpret_spill(const RunDev* __restrict__ runs, Params p, double* spill,
                                                        int slots) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x;
  double* stk = spill + (int64_t)w * slots * kInterpV * kWave;
  for (int run = 0; run < p.n_runs; ++run) {
    const RunDev& R = runs[run];
    const int cnt = uni(cload(&R.state[kStList0 + kLists - 1]));
    const int32_t* list = R.lists + (int64_t)(kLists - 1) * (p.m + p.r);
    const int64_t cblocks = (R.ld + kInterpTile - 1) / kInterpTile;
    const int64_t tasks = (int64_t)cnt * cblocks;
    for (int64_t t = w; t < tasks; t += gridDim.x) {
      const int j = (int)(t / cblocks);
      const int64_t cb = t - (int64_t)j * cblocks;
      const int prog = uni(cload(&list[j]));
      const int need = uni(cload(&R.need[prog]));
      if (need <= kMaxLdsSlots || need > slots) continue;  // LDS passes took it; never beyond the column
      const int64_t first = cb * kInterpTile;
      int64_t col[kInterpV];
      bool ok[kInterpV];
      uint32_t off[kInterpV];
      lane_cases<kInterpV>(first, lane, R.ld, col, ok, off);
      double out[kInterpV];
      eval_program_wide<kInterpV, 0>(R.ops + (int64_t)prog * p.k, R.opv + (int64_t)prog * p.k,
                                  R.opy + (int64_t)prog * p.k, R.X + (first / kXTile) * R.l * kXTile,
                                  uni(R.x_big) == 0, off, (GlobalStack)stk, lane, out);
      store_program<T, kInterpV>(R, p, prog, col, ok, out);
    }
  }
}

// ---------------------------------------------------------------------------
// One (program, 128-case block) task of the list interpreter: nprog
// programs (prog[j], squashed by the logistic when squash[j]) on cases of
// the feature-major Xfm, out[j][ld].
template <typename Stack>
__device__ __forceinline__ void list_task(const int32_t* ops, const double* opv, const int32_t* nops, int32_t k,
                                          const int32_t* prog, const int32_t* squash, int32_t nprog,
                                          const double* Xfm, int64_t ld, int64_t n, double* out, int64_t task,
                                          Stack stk, int lane) {
  const int64_t cb = task / nprog;
  const int j = (int)(task - cb * nprog);
  const int pr = uni(prog[j]);
  int64_t col[kInterpV];
  bool ok[kInterpV];
#pragma unroll
  for (int v = 0; v < kInterpV; ++v) {
    col[v] = cb * (kWave * kInterpV) + v * kWave + lane;
    ok[v] = col[v] < ld;
  }
  double val[kInterpV];
  eval_program<kInterpV>(ops + (int64_t)pr * k, opv + (int64_t)pr * k, uni(nops[pr]), Xfm, ld, col, ok, stk,
                                lane, val);
  const bool sq = squash[j] != 0;
#pragma unroll
  for (int v = 0; v < kInterpV; ++v) {
    if (!ok[v]) continue;
    double x = val[v];
    if (sq) x = 1.0 / (1.0 + exp(-x));
    out[(int64_t)j * ld + col[v]] = col[v] < n ? x : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_interpret_list(const int32_t* __restrict__ ops,
                                                        const double* __restrict__ opv,
                                                        const int32_t* __restrict__ nops, int32_t k,
                                                        const int32_t* __restrict__ prog,
                                                        const int32_t* __restrict__ squash,
                                                        int32_t nprog, const double* __restrict__ Xfm,
                                                        int64_t ld, int64_t n, double* __restrict__ out,
                                                        int slots, int64_t total) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int64_t task = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (task >= total) return;
  double* stk = lds + wave * slots * kInterpV * kWave;
  list_task(ops, opv, nops, k, prog, squash, nprog, Xfm, ld, n, out, task, (LdsStack)stk, lane);
}

// The same with stacks deeper than an LDS column: kSpillWaves one-wave
// blocks, each with a column of `slots` x kInterpV x 64 doubles in `spill`,
// sweep the tasks.
__global__ __launch_bounds__(64) void k_interpret_list_spill(const int32_t* __restrict__ ops,
                                                             const double* __restrict__ opv,
                                                             const int32_t* __restrict__ nops, int32_t k,
                                                             const int32_t* __restrict__ prog,
                                                             const int32_t* __restrict__ squash,
                                                             int32_t nprog, const double* __restrict__ Xfm,
                                                             int64_t ld, int64_t n, double* __restrict__ out,
                                                             double* spill, int slots, int64_t total) {
  const int lane = threadIdx.x & 63;
  double* stk = spill + (int64_t)blockIdx.x * slots * kInterpV * kWave;
  for (int64_t task = blockIdx.x; task < total; task += gridDim.x)
    list_task(ops, opv, nops, k, prog, squash, nprog, Xfm, ld, n, out, task, (GlobalStack)stk, lane);
}

// Waves per interpreter block so that the LDS stacks of one block stay
// within 64 KiB: each wave needs slots * kInterpV * 64 doubles.
inline int interp_waves(int slots) {
  const int per_wave = slots * kInterpV * kWave * (int)sizeof(double);
  int w = 65536 / per_wave;
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

}  // namespace

hipError_t launch_compile(const RunDev* d_runs, const Params& p, hipStream_t s) {
  const int32_t groups = (p.m + p.r + kWave - 1) / kWave;  // 64-genome groups per run
  hipLaunchKernelGGL(k_compile, dim3((unsigned)p.n_runs * groups), dim3(kWave), 0, s, d_runs, p, groups);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // length bins: (k - length) >> shift < kOrderBins for lengths 0 .. k
  int shift = 0;
  while ((p.k >> shift) >= kOrderBins) ++shift;
  hipLaunchKernelGGL(k_order, dim3(p.n_runs), dim3(1024), 0, s, d_runs, p, shift);
  return hipGetLastError();
}

hipError_t launch_interpret(const RunDev* d_runs, const Params& p, int64_t case_blocks, int lo, int slots,
                            int list, int32_t progs, hipStream_t s) {
  if (slots < 1) slots = 1;
  if (slots > kMaxLdsSlots) return hipErrorInvalidValue;  // deeper stacks take the spill pass
  if (list < 0 || list >= kLists) return hipErrorInvalidValue;
  if (progs <= 0) return hipSuccess;
  // one LDS stack column block per wave, at most 64 KiB per block
  const int waves = interp_waves(slots);
  const size_t shmem = (size_t)waves * slots * kInterpV * kWave * sizeof(double);
  const int32_t pgroups = (progs + waves * kInterpProgsPerWave - 1) / (waves * kInterpProgsPerWave);
  // any workspace that fits on the device keeps this far below the limit
  if (case_blocks * pgroups > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)(case_blocks * pgroups)), block(waves * kWave);
  if (p.precision == GSGP_FP64)
    hipLaunchKernelGGL((k_interpret<double>), grid, block, shmem, s, d_runs, p, pgroups, lo, slots, list);
  else
    hipLaunchKernelGGL((k_interpret<float>), grid, block, shmem, s, d_runs, p, pgroups, lo, slots, list);
  return hipGetLastError();
}

// Cases per lane of each list's pass (see k_interpret_wide).
// Four cases per lane except for the deepest list, whose 6-value column
// would hold the LDS to 13 waves per CU (V = 2 there: 4 % faster at the
// Section 3.1 shape with 2,047 genes; two cases per lane on the other lists
// was slower).
constexpr int kListV[kLists - 1] = {4, 4, 4, 2};
// Stack values kept in registers beyond the top two (see eval_program_wide):
// one more on the 4- and 6-value lists, whose LDS columns then shrink to 3
// and 5 values (2,047 genes at the Section 3.1 shape: 222 -> 216 ms; on the
// 3-value list as well it was slower, 223 ms).
constexpr int kListReg[kLists - 1] = {0, 0, 1, 1};

template <typename T, int B>
void launch_wide_list(const RunDev* d_runs, const Params& p, int64_t case_blocks, int32_t progs, int lo, int list,
                      hipStream_t s) {
  const dim3 grid((unsigned)(case_blocks * progs));
  hipLaunchKernelGGL((k_interpret_wide<T, kListSlots[B], kListV[B], kListReg[B]>), grid, dim3(kWave), 0, s, d_runs, p,
                     progs, lo, list);
}

template <typename T>
hipError_t launch_wide_lists(const RunDev* d_runs, const Params& p, int64_t blocks256, int64_t blocks128, int lo,
                             int list, int32_t progs, hipStream_t s) {
  const int64_t case_blocks = kListV[list] == 4 ? blocks256 : blocks128;
  if (case_blocks * progs > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  switch (list) {
    case 0: launch_wide_list<T, 0>(d_runs, p, case_blocks, progs, lo, list, s); break;
    case 1: launch_wide_list<T, 1>(d_runs, p, case_blocks, progs, lo, list, s); break;
    case 2: launch_wide_list<T, 2>(d_runs, p, case_blocks, progs, lo, list, s); break;
    case 3: launch_wide_list<T, 3>(d_runs, p, case_blocks, progs, lo, list, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_interpret_wide(const RunDev* d_runs, const Params& p, int64_t blocks256, int64_t blocks128, int lo,
                                 int list, int32_t progs, hipStream_t s) {
  if (list < 0 || list >= kLists - 1) return hipErrorInvalidValue;
  if (progs <= 0) return hipSuccess;
  return p.precision == GSGP_FP64 ? launch_wide_lists<double>(d_runs, p, blocks256, blocks128, lo, list, progs, s)
                                  : launch_wide_lists<float>(d_runs, p, blocks256, blocks128, lo, list, progs, s);
}

hipError_t launch_interpret_spill(const RunDev* d_runs, const Params& p, double* spill, int slots,
                                  hipStream_t s) {
  if (slots <= kMaxLdsSlots) return hipSuccess;
  if (!spill) return hipErrorInvalidValue;
  if (p.precision == GSGP_FP64)
    hipLaunchKernelGGL((k_interpret_spill<double>), dim3(kSpillWaves), dim3(kWave), 0, s, d_runs, p, spill, slots);
  else
    hipLaunchKernelGGL((k_interpret_spill<float>), dim3(kSpillWaves), dim3(kWave), 0, s, d_runs, p, spill, slots);
  return hipGetLastError();
}

hipError_t launch_interpret_list(const int32_t* ops, const double* opv, const int32_t* nops,
                                 int32_t k, const int32_t* prog, const int32_t* squash,
                                 int32_t nprog, const double* Xfm, int64_t ld, int64_t n,
                                 double* out, int slots, double* spill, hipStream_t s) {
  if (nprog <= 0) return hipSuccess;
  if (slots < 1) slots = 1;
  const int64_t cblocks = (ld + kWave * kInterpV - 1) / (kWave * kInterpV);
  const int64_t total = cblocks * nprog;
  if (slots > kMaxLdsSlots) {
    if (!spill) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_interpret_list_spill, dim3(kSpillWaves), dim3(kWave), 0, s, ops, opv, nops, k, prog,
                       squash, nprog, Xfm, ld, n, out, spill, slots, total);
    return hipGetLastError();
  }
  const int waves = interp_waves(slots);
  const size_t shmem = (size_t)waves * slots * kInterpV * kWave * sizeof(double);
  hipLaunchKernelGGL(k_interpret_list, dim3(blocks_for(total, waves)), dim3(waves * kWave),
                     shmem, s, ops, opv, nops, k, prog, squash, nprog, Xfm, ld, n, out, slots, total);
  return hipGetLastError();
}

}  // namespace gsgp
