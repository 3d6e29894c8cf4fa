// HIP kernels of the GSGP hot path for gfx950 (MI355X, CDNA4, wave64).
//
// Method: "GSGP-CUDA - a CUDA framework for Geometric Semantic Genetic
// Programming" (Trujillo et al., arXiv 2106.04034), Algorithm 1 and the
// Section 2.2 paragraphs on initialization, the interpreter, fitness, GSM and
// survival.  The paper's own CUDA design (one thread per individual for the
// interpreter and the fitness, cuBLAS I?AMIN / I?AMAX for survival) is prior
// art; the mapping here is:
//   k_genome     one thread per gene, counter-based Philox draws;
//   k_compile, k_interpret*  (interp.hip) the genome compiler and the
//                stack-machine interpreter;
//   k_vary       the hot loop: every offspring row of one 2 KiB case chunk is
//                formed from its parent and pool rows with 16-byte loads and
//                non-temporal 16-byte stores, and the chunk's squared
//                residual sum is reduced across the wave with xor shuffles;
//                blocks on one XCD share a chunk so distinct parent and pool
//                rows are fetched from HBM about once per chunk;
//   k_fitness    lanes own individuals and waves own chunk ranges; FP64 sums;
//   k_survive    argmin / argmax with lowest-index ties, elite row copy,
//                per-generation summary and the next generation's tournaments.
// All kernels are compiled without floating-point contraction so that the
// per-element arithmetic matches the method's definitions operation by
// operation.
#include "device.hpp"

namespace gsgp {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32 -> 64-bit products with a Weyl key schedule.
struct Words4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t x0 = hi1 ^ c1 ^ k0;
    const uint32_t x2 = hi0 ^ c3 ^ k1;
    c0 = x0;
    c1 = lo1;
    c2 = x2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words4{c0, c1, c2, c3};
}

// Integer in [0, n) by multiply-shift of one 32-bit word.
__device__ __forceinline__ int32_t draw_below(uint32_t w, uint32_t n) {
  return (int32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

// Uniform in [0, 1) on the 2^-53 grid from two words (27 + 26 bits).
__device__ __forceinline__ double draw_u53(uint32_t a, uint32_t b) {
  const double hi = (double)(a >> 5);
  const double lo = (double)(b >> 6);
  return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

// ---------------------------------------------------------------------------
// Data preparation: FP64 row-major cases -> feature-major padded X, target in
// the storage type, zero pads, non-finite detection.  One thread per padded
// column of every run.
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const RunDev* __restrict__ runs, Params p,
                                              int64_t total, const double* const* __restrict__ src) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int run = find_run(p.n_runs, g, [&](int r) { return runs[r].col0; });
  const RunDev& R = runs[run];
  const int64_t col = g - R.col0;
  const double* Xs = nullptr;
  const double* ys = nullptr;
  int64_t row = -1;
  if (col < R.n_train) {
    Xs = src[4 * run + 0];
    ys = src[4 * run + 1];
    row = col;
  } else if (col >= R.tr_pad && col < R.tr_pad + R.n_test) {
    Xs = src[4 * run + 2];
    ys = src[4 * run + 3];
    row = col - R.tr_pad;
  }
  bool bad = false, big = false;
  for (int f = 0; f < R.l; ++f) {
    const double v = (row >= 0) ? Xs[row * R.l + f] : 0.0;
    bad |= !isfinite(v);
    big |= fabs(v) > 0x1p128;
    R.X[x_index(col, f, R.l)] = v;
  }
  const double yv = (row >= 0) ? ys[row] : 0.0;
  bad |= !isfinite(yv) || fabs(yv) > kFltMax;
  ((T*)R.y)[col] = (T)yv;
  if (bad) atomicOr(&R.state[kStNonFinite], 1);
  if (big) atomicOr(&R.state[kStXBig], 1);
}

// ---------------------------------------------------------------------------
// CreatePopulation (Algorithm 1; Section 2.2 "Initialization"): gene q of
// tree t draws Philox counter (q, t, 0, tag), key (seed, run), tag 1 for the
// population and 2 for the random-tree pool.  Word 0 picks the gene type
// against the cumulative thresholds, word 1 the function or feature, words 2
// and 3 the constant.
__global__ __launch_bounds__(256) void k_genome(const RunDev* __restrict__ runs, Params p,
                                                int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int64_t per_run = (int64_t)(p.m + p.r) * p.k;
  const int run = (int)(g / per_run);
  const int64_t local = g - (int64_t)run * per_run;
  const int row = (int)(local / p.k);
  const int q = (int)(local - (int64_t)row * p.k);
  const RunDev& R = runs[run];
  const uint32_t tag = row < p.m ? 1u : 2u;
  const uint32_t t = row < p.m ? (uint32_t)row : (uint32_t)(row - p.m);
  const Words4 w = philox4x32_10((uint32_t)q, t, 0u, tag, p.seed, R.run_id);
  int32_t code;
  double val = 0.0;
  if ((uint64_t)w.w0 < p.t_func) {
    code = -1 - (int32_t)(w.w1 >> 30);
  } else if ((uint64_t)w.w0 < p.t_feat) {
    code = draw_below(w.w1, (uint32_t)R.l);
  } else {
    const double u = draw_u53(w.w2, w.w3);
    const double span = p.erc_hi - p.erc_lo;
    const double scaled = span * u;
    code = -5;
    val = p.erc_lo + scaled;
  }
  R.code[local] = code;
  R.cval[local] = val;
}

// ---------------------------------------------------------------------------
// Wave reductions.  xor butterflies give every lane the same bits because
// each step adds the same two operands in both partner lanes.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Compensated combination of Kahan pairs (value = s - c) with Knuth's
// two-sum: exact error of s1 + s2 is folded into the compensation term.
__device__ __forceinline__ void wave_sum_kahan(float& s, float& c) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float s2 = __shfl_xor(s, o, kWave);
    const float c2 = __shfl_xor(c, o, kWave);
    const float sum = s + s2;
    const float bp = sum - s;
    const float err = (s - (sum - bp)) + (s2 - bp);
    c = (c + c2) - err;
    s = sum;
  }
}

// Sum over one chunk of (o - t)^2 in the canonical order: each lane adds its
// elements in address order (LaneSse, fed one 16-byte vector at a time as
// the offspring values are formed), then the wave butterfly (sse_finish).
// FP32 forms fall back to FP64 when a square overflows.  The fallback takes
// the offspring values from registers (each offspring vector occupies the
// registers its three operands free) and reads the target chunk again from
// memory (`tgt`, an L2 hit): converting the target vectors to FP64 ahead of
// the rare branch would hold 32 more registers for the whole kernel.
template <typename T, int PREC>
struct LaneSse {
  typedef typename std::conditional<PREC == GSGP_FP64, double, float>::type A;
  A s = 0, c = 0;
  template <typename VT>
  __device__ __forceinline__ void add(const VT& o, const VT& t) {
    constexpr int N = VecOf<T>::N;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const A e = (A)o[k] - (A)t[k];
      if constexpr (PREC == GSGP_FP32_KAHAN) {
        const A y = e * e - c;
        const A u = s + y;
        c = (u - s) - y;
        s = u;
      } else {
        s += e * e;
      }
    }
  }
};

template <typename T, int PREC, int NJ, typename VT>
__device__ __forceinline__ double sse_finish(LaneSse<T, PREC> acc, const bool (&ok)[NJ], const VT (&o)[NJ],
                                             const T* tgt, int lane) {
  constexpr int N = VecOf<T>::N;
  if constexpr (PREC == GSGP_FP64) {
    return wave_sum(acc.s);
  } else {
    double total;
    if constexpr (PREC == GSGP_FP32) {
      total = (double)wave_sum(acc.s);
    } else {
      wave_sum_kahan(acc.s, acc.c);
      total = (double)acc.s - (double)acc.c;
    }
    if (!isfinite(total)) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (!ok[j]) continue;
        const int e = j * kWave * N + lane * N;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const double d = (double)o[j][c] - (double)tgt[e + c];
          s += d * d;
        }
      }
      total = wave_sum(s);
    }
    return total;
  }
}

template <typename T, int PREC, int NJ, typename VT>
__device__ __forceinline__ double chunk_sse(const VT (&o)[NJ], const VT (&t)[NJ], const bool (&ok)[NJ],
                                            const T* tgt, int lane) {
  LaneSse<T, PREC> acc;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    if (ok[j]) acc.add(o[j], t[j]);
  return sse_finish<T, PREC, NJ>(acc, ok, o, tgt, lane);
}

// One offspring's operands for one chunk.  Mutation reads S[p1], sR[r1],
// sR[r2]; crossover reads S[p1], S[p2], sR[r1].  The pointer choice is
// wave-uniform, so both kinds issue the same three 16-byte loads per slot.
// FULL chunks need no lane masks (only a segment's last chunk can be short).
template <typename T, int PREC, bool FULL, int NJ>
__device__ __forceinline__ void vary_offspring(const gsgp_record* rc, const T* Sc, const T* gc, T* dst,
                                               int lane, int64_t len,
                                               const typename VecOf<T>::type (&t)[NJ], const T* tgt,
                                               double* part_out) {
  typedef typename VecOf<T>::type VT;
  constexpr int N = VecOf<T>::N;
  constexpr int64_t kChunk = chunk_cases(sizeof(T));
  // row stride inside a chunk block is the chunk length (compile-time for full chunks)
  const int64_t stride = FULL ? kChunk : len;
  const int op = uni(cload(&rc->op));
  const int p1 = uni(cload(&rc->p1));
  const int r1 = uni(cload(&rc->r1));
  const int second = uni(op == 1 ? cload(&rc->p2) : cload(&rc->r2));
  const T ms = (T)cload(&rc->ms);
  const T* A = Sc + (int64_t)p1 * stride;
  const T* B = (op == 1 ? Sc : gc) + (int64_t)(op == 1 ? second : r1) * stride;
  const T* C = gc + (int64_t)(op == 1 ? r1 : second) * stride;
  bool ok[NJ];
  VT x[NJ], y[NJ], z[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = j * kWave * N + lane * N;
    ok[j] = FULL || e < len;
    if (ok[j]) {
      x[j] = gload<VT>(A + e);
      y[j] = gload<VT>(B + e);
      z[j] = gload<VT>(C + e);
    } else {
      x[j] = VT(0);
      y[j] = VT(0);
      z[j] = VT(0);
    }
  }
  // Form, clamp, store and accumulate one 16-byte vector at a time, so the
  // operands of a vector die as soon as its offspring value is stored.
  LaneSse<T, PREC> acc;
  VT o[NJ];
  auto emit = [&](int j, VT v) {
    if constexpr (PREC != GSGP_FP64) {
      // a convex combination of two values near +-FLT_MAX can round past it;
      // operands are finite, so a median-of-three clamps exactly
#pragma unroll
      for (int c = 0; c < N; ++c) v[c] = __builtin_amdgcn_fmed3f(v[c], (T)-kFltMax, (T)kFltMax);
    }
    o[j] = v;
    if (ok[j]) {
      gstore_nt<VT>(v, dst + j * kWave * N + lane * N);
      acc.add(v, t[j]);
    }
  };
  if (op == 1) {
    // GSC: O = S[p1] * sR[r1] + S[p2] * (1 - sR[r1])
#pragma unroll
    for (int j = 0; j < NJ; ++j) emit(j, x[j] * z[j] + y[j] * ((T)1 - z[j]));
  } else {
    // GSM: O = S[p1] + ms * (sR[r1] - sR[r2])
#pragma unroll
    for (int j = 0; j < NJ; ++j) emit(j, x[j] + ms * (y[j] - z[j]));
  }
  const double sse = sse_finish<T, PREC, NJ>(acc, ok, o, tgt, lane);
  if (lane == 0) *part_out = sse;
}

// Local search form of vary_offspring.  Stored rows are the operators'
// outputs; individual p's semantics are alpha_p + beta_p * S[p] with its
// scaling from the generation's table `lsg` ([m][2]), applied here as the
// parents are read (so scaling costs no extra pass over the rows).  The
// offspring row is stored unscaled, and the chunk's sums of o, o^2 and o * t
// (FP64, lane then butterfly, over the real cases only) go to part_out[0],
// part_out[m], part_out[2 m]; the fitness kernel fits the offspring's own
// scaling from them.  Real cases of the chunk are its first `real` columns.
template <typename T, bool FULL, int NJ>
__device__ __forceinline__ void vary_offspring_ls(const gsgp_record* rc, const double* lsg, const T* Sc, const T* gc,
                                                  T* dst, int lane, int64_t len, int64_t real,
                                                  const typename VecOf<T>::type (&t)[NJ], double* part_out,
                                                  int64_t m) {
  typedef typename VecOf<T>::type VT;
  constexpr int N = VecOf<T>::N;
  constexpr int64_t kChunk = chunk_cases(sizeof(T));
  const int64_t stride = FULL ? kChunk : len;
  const int op = uni(cload(&rc->op));
  const int p1 = uni(cload(&rc->p1));
  const int r1 = uni(cload(&rc->r1));
  const int second = uni(op == 1 ? cload(&rc->p2) : cload(&rc->r2));
  const T ms = (T)cload(&rc->ms);
  const T* A = Sc + (int64_t)p1 * stride;
  const T* B = (op == 1 ? Sc : gc) + (int64_t)(op == 1 ? second : r1) * stride;
  const T* C = gc + (int64_t)(op == 1 ? r1 : second) * stride;
  // scaling of the parents (the second one only for crossover); in the FP32
  // forms the coefficients are rounded to FP32 and kept finite
  auto coef = [](double v) {
    if constexpr (std::is_same<T, float>::value) return (T)fmin(fmax(v, -kFltMax), kFltMax);
    else return (T)v;
  };
  const T a1 = coef(cload(&lsg[2 * (int64_t)p1])), b1 = coef(cload(&lsg[2 * (int64_t)p1 + 1]));
  const T a2 = op == 1 ? coef(cload(&lsg[2 * (int64_t)second])) : (T)0;
  const T b2 = op == 1 ? coef(cload(&lsg[2 * (int64_t)second + 1])) : (T)1;
  const bool padded = real < len;
  bool ok[NJ];
  VT x[NJ], y[NJ], z[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = j * kWave * N + lane * N;
    ok[j] = FULL || e < len;
    if (ok[j]) {
      x[j] = gload<VT>(A + e);
      y[j] = gload<VT>(B + e);
      z[j] = gload<VT>(C + e);
    } else {
      x[j] = VT(0);
      y[j] = VT(0);
      z[j] = VT(0);
    }
  }
  auto clamp = [](VT v) {
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
      for (int c = 0; c < N; ++c) v[c] = __builtin_amdgcn_fmed3f(v[c], (T)-kFltMax, (T)kFltMax);
    }
    return v;
  };
  double so = 0.0, soo = 0.0, sot = 0.0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = j * kWave * N + lane * N;
    const VT xe = clamp(a1 + b1 * x[j]);
    VT o;
    if (op == 1) {
      // GSC on the parents' semantics: O = T1 * sR[r1] + T2 * (1 - sR[r1])
      const VT ye = clamp(a2 + b2 * y[j]);
      o = clamp(xe * z[j] + ye * ((T)1 - z[j]));
    } else {
      // GSM: O = T + ms * (sR[r1] - sR[r2])
      o = clamp(xe + ms * (y[j] - z[j]));
    }
    if (padded) {
#pragma unroll
      for (int c = 0; c < N; ++c) o[c] = (e + c < real) ? o[c] : (T)0;  // pads stay exact zeros
    }
    if (ok[j]) {
      gstore_nt<VT>(o, dst + e);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const double ov = (double)o[c];
        so += ov;
        soo += ov * ov;
        sot += ov * (double)t[j][c];
      }
    }
  }
  so = wave_sum(so);
  soo = wave_sum(soo);
  sot = wave_sum(sot);
  if (lane == 0) {
    part_out[0] = so;
    part_out[m] = soo;
    part_out[2 * m] = sot;
  }
}

// Partial sums of an existing row (generation-0 fitness).
template <typename T, int PREC, bool FULL, int NJ>
__device__ __forceinline__ void row_partial(const T* row, int lane, int64_t len,
                                            const typename VecOf<T>::type (&t)[NJ], const T* tgt,
                                            double* part_out) {
  typedef typename VecOf<T>::type VT;
  constexpr int N = VecOf<T>::N;
  bool ok[NJ];
  VT o[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = j * kWave * N + lane * N;
    ok[j] = FULL || e < len;
    o[j] = ok[j] ? gload<VT>(row + e) : VT(0);
  }
  const double sse = chunk_sse<T, PREC, NJ, VT>(o, t, ok, tgt, lane);
  if (lane == 0) *part_out = sse;
}

template <typename T, int PREC, bool ROWS, bool FULL, bool LS>
__device__ __forceinline__ void vary_task(const RunDev& R, const Params& p, const VaryLaunch& lc, int chunk,
                                          int grp, int lane, int wave) {
  typedef typename VecOf<T>::type VT;
  constexpr int N = VecOf<T>::N;
  constexpr int kChunk = chunk_cases(sizeof(T));
  constexpr int NJ = kChunk / (kWave * N);
  // each instance derives the chunk geometry itself from the chunk index
  const ChunkGeom g = chunk_geom(R.tr_pad, R.te_pad, R.nch_tr, chunk, kChunk);
  const int64_t cs = g.cs;
  const int64_t len = FULL ? (int64_t)kChunk : g.len;
  const int gen = ROWS ? 0 : uni(cload(&R.state[kStGen]));
  const int cur = gen & 1;
  // chunk blocks of the tiled buffers (see chunk_geom): rows * cs elements in
  const T* Sc = (const T*)R.S[cur] + (int64_t)p.m * cs;
  T* Oc = (T*)R.S[cur ^ 1] + (int64_t)p.m * cs;
  const T* gc = (const T*)R.sigR + (int64_t)p.r * cs;
  const T* yv = (const T*)R.y + cs;
  const int64_t stride = FULL ? (int64_t)chunk_cases(sizeof(T)) : len;
  VT t[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = j * kWave * N + lane * N;
    t[j] = (FULL || e < len) ? gload<VT>(yv + e) : VT(0);
  }
  int i_end = (grp + 1) * lc.opb;
  i_end = i_end < p.m ? i_end : p.m;
  double* part = R.part + (int64_t)chunk * p.m;
  if constexpr (ROWS) {
    for (int i = grp * lc.opb + wave; i < i_end; i += lc.waves)
      row_partial<T, PREC, FULL, NJ>(Sc + (int64_t)i * stride, lane, len, t, yv, part + i);
  } else if constexpr (LS) {
    const gsgp_record* recs = R.rec + (int64_t)gen * p.m;
    const double* lsg = R.ls + (int64_t)gen * p.m * 2;
    // real cases of this chunk: the segment's real cases past its first column
    const bool train = chunk < R.nch_tr;
    const int64_t first = train ? cs : cs - R.tr_pad;
    int64_t real = (train ? R.n_train : R.n_test) - first;
    real = real < 0 ? 0 : (real > len ? len : real);
    double* part3 = R.part + (int64_t)chunk * 3 * p.m;
    for (int i = grp * lc.opb + wave; i < i_end; i += lc.waves)
      vary_offspring_ls<T, FULL, NJ>(recs + i, lsg, Sc, gc, Oc + (int64_t)i * stride, lane, len, real, t,
                                     part3 + i, p.m);
  } else {
    const gsgp_record* recs = R.rec + (int64_t)gen * p.m;
    for (int i = grp * lc.opb + wave; i < i_end; i += lc.waves)
      vary_offspring<T, PREC, FULL, NJ>(recs + i, Sc, gc, Oc + (int64_t)i * stride, lane, len, t, yv, part + i);
  }
}

// ---------------------------------------------------------------------------
// GSM / GSC + fitness partials (Algorithm 1 loop: GSM, ComputeFitness).
// Task = (run, 2 KiB chunk of cases, group of `opb` offspring).  Each wave
// takes offspring grp*opb + wave, + waves, ...; per offspring it reads its
// variation record, forms the chunk of the offspring row
//   mutation:  O = S[p1] + ms * (sR[r1] - sR[r2])
//   crossover: O = S[p1] * sR[r1] + S[p2] * (1 - sR[r1])
// (sR holds the squashed pool semantics), stores it with non-temporal
// 16-byte stores and writes the chunk's sum of squared residuals.  With
// ROWS the kernel only forms the partial sums of the current population
// (generation-0 fitness).
template <typename T, int PREC, bool ROWS, bool LOOP, bool LS>
__global__ __launch_bounds__(512) void k_vary(const RunDev* __restrict__ runs, Params p, VaryLaunch lc) {
  constexpr int kChunk = chunk_cases(sizeof(T));
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  // Hardware dispatch sends block b to XCD b % 8.  remap 1: each XCD takes a
  // contiguous range of tasks.  remap 2: XCD x takes the x-th group of
  // `ogroups` tasks (one chunk) of every run of 8 chunks, so the XCDs sweep
  // the rows side by side through an 8-chunk window.
  // LOOP: a persistent grid, blocks sweep the tasks; otherwise the grid
  // covers every task in one sweep and the loop body runs once (no values
  // hoisted across iterations, fewer registers).
  const int64_t xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = lc.grid >> 3;
  for (int64_t it = 0; LOOP || it == 0; ++it) {
    int64_t task;
    if (lc.remap == 2) {
      const int64_t q = slot + it * per;
      task = (q / lc.ogroups) * 8 * lc.ogroups + xcd * lc.ogroups + q % lc.ogroups;
      if ((q / lc.ogroups) * 8 * lc.ogroups >= lc.total_tasks) break;
      if (task >= lc.total_tasks) continue;
    } else {
      task = (lc.remap ? xcd * per + slot : (int64_t)blockIdx.x) + it * lc.grid;
      if (task >= lc.total_tasks) break;
    }
    const int run = find_run(p.n_runs, task, [&](int r) { return runs[r].vary_task0; });
    const RunDev& R = runs[run];
    const int64_t local = task - R.vary_task0;
    const int chunk = (int)(local / lc.ogroups);
    const int grp = (int)(local - (int64_t)chunk * lc.ogroups);
    const ChunkGeom g = chunk_geom(R.tr_pad, R.te_pad, R.nch_tr, chunk, kChunk);
    if (g.len == kChunk)
      vary_task<T, PREC, ROWS, true, LS>(R, p, lc, chunk, grp, lane, wave);
    else
      vary_task<T, PREC, ROWS, false, LS>(R, p, lc, chunk, grp, lane, wave);
  }
}

// (the generation-0 partial sums never scale: every individual starts with
// alpha = 0, beta = 1)

// ComputeFitness (Section 2.2 "Fitness computation"): a block takes 64
// individuals of one run (lane = individual, so the chunk-major partial sums
// are read with coalesced loads); its kFitWaves waves split each segment's
// chunks into contiguous ranges, sum them in chunk order, and the ranges are
// added in wave order in FP64.  Then the root mean.
constexpr int kFitWaves = 16;

__device__ __forceinline__ double sum_range(const double* __restrict__ part, int64_t m, int i, int c0, int c1) {
  double s = 0.0;
  int c = c0;
  for (; c + 4 <= c1; c += 4) {
    const double a = part[(int64_t)c * m + i];
    const double b = part[(int64_t)(c + 1) * m + i];
    const double d = part[(int64_t)(c + 2) * m + i];
    const double e = part[(int64_t)(c + 3) * m + i];
    s += a;
    s += b;
    s += d;
    s += e;
  }
  for (; c < c1; ++c) s += part[(int64_t)c * m + i];
  return s;
}

__global__ __launch_bounds__(kFitWaves * 64) void k_fitness(const RunDev* __restrict__ runs, Params p,
                                                             int32_t blocks_per_run, int init) {
  __shared__ double sh_tr[kFitWaves][kWave];
  __shared__ double sh_te[kFitWaves][kWave];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int run = blockIdx.x / blocks_per_run;
  const int i = (blockIdx.x - run * blocks_per_run) * kWave + lane;
  const RunDev& R = runs[run];
  const bool live = i < p.m;
  const int ii = live ? i : 0;
  const int nt = R.nch_tr, ne = R.nch - R.nch_tr;
  const int a0 = (int)((int64_t)nt * wave / kFitWaves), a1 = (int)((int64_t)nt * (wave + 1) / kFitWaves);
  const int b0 = nt + (int)((int64_t)ne * wave / kFitWaves), b1 = nt + (int)((int64_t)ne * (wave + 1) / kFitWaves);
  sh_tr[wave][lane] = sum_range(R.part, p.m, ii, a0, a1);
  sh_te[wave][lane] = sum_range(R.part, p.m, ii, b0, b1);
  __syncthreads();
  if (wave == 0 && live) {
    double s = sh_tr[0][lane], st = sh_te[0][lane];
    for (int w = 1; w < kFitWaves; ++w) {
      s += sh_tr[w][lane];
      st += sh_te[w][lane];
    }
    const int dst = init ? 0 : ((R.state[kStGen] + 1) & 1);
    R.F[dst][i] = sqrt(s / (double)R.n_train);
    R.Ft[dst][i] = R.n_test > 0 ? sqrt(st / (double)R.n_test) : 0.0;
  }
}

// Local search fitness: each offspring's least-squares scaling and the RMSE
// of its scaled semantics, in closed form from its chunk sums (o, o^2, o * t
// over the real cases; laid out [chunk][3][m]) and the run's target sums.
// With n cases, D = So2 - So^2 / n (n times the variance of o) and
// Sxy = Sot - So * St / n:
//   beta = Sxy / D,  alpha = (St - beta * So) / n,
//   SSE_train = (Stt - St^2 / n) - beta * Sxy   (residual orthogonal to 1, o),
//   SSE_test = sum (alpha + beta o - t)^2 expanded over the test sums.
// A numerically constant offspring (D <= 1e-10 * So2) keeps alpha = 0,
// beta = 1 and SSE = So2 - 2 Sot + Stt.  Chunk sums combine as in k_fitness.
// The scaling goes to the table row of the offspring generation.
__global__ __launch_bounds__(kFitWaves * 64) void k_fitness_ls(const RunDev* __restrict__ runs, Params p,
                                                                int32_t blocks_per_run) {
  __shared__ double sh[6][kFitWaves][kWave];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int run = blockIdx.x / blocks_per_run;
  const int i = (blockIdx.x - run * blocks_per_run) * kWave + lane;
  const RunDev& R = runs[run];
  const bool live = i < p.m;
  const int ii = live ? i : 0;
  const int64_t m = p.m;
  const int nt = R.nch_tr, ne = R.nch - R.nch_tr;
  const int a0 = (int)((int64_t)nt * wave / kFitWaves), a1 = (int)((int64_t)nt * (wave + 1) / kFitWaves);
  const int b0 = nt + (int)((int64_t)ne * wave / kFitWaves), b1 = nt + (int)((int64_t)ne * (wave + 1) / kFitWaves);
  for (int q = 0; q < 3; ++q) {
    double s = 0.0, st = 0.0;
    for (int c = a0; c < a1; ++c) s += R.part[((int64_t)c * 3 + q) * m + ii];
    for (int c = b0; c < b1; ++c) st += R.part[((int64_t)c * 3 + q) * m + ii];
    sh[q][wave][lane] = s;
    sh[3 + q][wave][lane] = st;
  }
  __syncthreads();
  if (wave == 0 && live) {
    double v[6];
    for (int q = 0; q < 6; ++q) {
      v[q] = sh[q][0][lane];
      for (int w = 1; w < kFitWaves; ++w) v[q] += sh[q][w][lane];
    }
    const double n = (double)R.n_train, So = v[0], Soo = v[1], Sot = v[2];
    const double St = R.tsum[0], Stt = R.tsum[1];
    const double D = Soo - So * So / n;
    double alpha = 0.0, beta = 1.0, sse;
    if (D > 1e-10 * Soo) {
      const double Sxy = Sot - So * St / n;
      beta = Sxy / D;
      alpha = (St - beta * So) / n;
      sse = (Stt - St * St / n) - beta * Sxy;
    } else {
      sse = Soo - 2.0 * Sot + Stt;
    }
    sse = sse > 0.0 ? sse : 0.0;
    double sse_te = 0.0;
    if (R.n_test > 0) {
      const double ne_ = (double)R.n_test, Se = v[3], See = v[4], Set = v[5];
      const double Ste = R.tsum[2], Stte = R.tsum[3];
      // sum (alpha + beta o - t)^2 = beta^2 See + sum (alpha - t)^2 + 2 beta sum o (alpha - t)
      sse_te = beta * beta * See + (ne_ * alpha * alpha - 2.0 * alpha * Ste + Stte) +
               2.0 * beta * (alpha * Se - Set);
      sse_te = sse_te > 0.0 ? sse_te : 0.0;
    }
    const int g1 = R.state[kStGen] + 1;
    const int dst = g1 & 1;
    R.F[dst][i] = sqrt(sse / n);
    R.Ft[dst][i] = R.n_test > 0 ? sqrt(sse_te / (double)R.n_test) : 0.0;
    R.ls[((int64_t)g1 * m + i) * 2] = alpha;
    R.ls[((int64_t)g1 * m + i) * 2 + 1] = beta;
  }
}

// Local search: sums of the stored target over a run's real train and test
// cases (one block per run; thread-strided FP64 sums, then a fixed-order LDS
// tree, so the bits never vary).  Also writes generation 0's scaling table
// row (alpha = 0, beta = 1).
template <typename T>
__global__ __launch_bounds__(256) void k_target_sums(const RunDev* __restrict__ runs, Params p) {
  __shared__ double sh[4][256];
  const RunDev& R = runs[blockIdx.x];
  const T* y = (const T*)R.y;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int64_t k = threadIdx.x; k < R.n_train; k += blockDim.x) {
    const double v = (double)y[k];
    a += v;
    b += v * v;
  }
  for (int64_t k = threadIdx.x; k < R.n_test; k += blockDim.x) {
    const double v = (double)y[R.tr_pad + k];
    c += v;
    d += v * v;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  sh[3][threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) R.tsum[threadIdx.x] = sh[threadIdx.x][0];
  for (int i = threadIdx.x; i < p.m; i += blockDim.x) {
    R.ls[2 * (int64_t)i] = 0.0;
    R.ls[2 * (int64_t)i + 1] = 1.0;
  }
}

// ---------------------------------------------------------------------------
// Survival, summary and the next generation's variation draws.
struct ValIdx {
  double v;
  int i;
};

__device__ __forceinline__ ValIdx pick_min(ValIdx a, ValIdx b) {
  return (b.v < a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}
__device__ __forceinline__ ValIdx pick_max(ValIdx a, ValIdx b) {
  return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}

template <bool MAX, typename View>
__device__ ValIdx block_arg(int m, View F, ValIdx* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  ValIdx x{MAX ? -INFINITY : INFINITY, 0x7fffffff};
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const ValIdx y{F(i), i};
    x = MAX ? pick_max(x, y) : pick_min(x, y);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const ValIdx y{__shfl_xor(x.v, o, kWave), __shfl_xor(x.i, o, kWave)};
    x = MAX ? pick_max(x, y) : pick_min(x, y);
  }
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  ValIdx r = sh[0];
  for (int w = 1; w < nw; ++w) r = MAX ? pick_max(r, sh[w]) : pick_min(r, sh[w]);
  __syncthreads();
  if (r.i < 0 || r.i >= m) r.i = 0;  // fitness is always finite; keep indices in range regardless
  return r;
}

// Sequential access to the Philox words W[0], W[1], ... of one offspring:
// word w is lane w % 4 of Philox(counter (i, w / 4, gen, 3)).
struct WordStream {
  uint32_t i, gen, k0, k1;
  int block;
  Words4 cur;
  __device__ uint32_t at(int w) {
    const int b = w >> 2;
    if (b != block) {
      cur = philox4x32_10(i, (uint32_t)b, gen, 3u, k0, k1);
      block = b;
    }
    const int s = w & 3;
    return s == 0 ? cur.w0 : (s == 1 ? cur.w1 : (s == 2 ? cur.w2 : cur.w3));
  }
};

// Tournament: s uniform candidates, the first with strictly smaller fitness
// wins (ties go to the earlier draw).
template <typename View>
__device__ __forceinline__ int32_t tournament(WordStream& ws, int first, int s, int m, View F) {
  int32_t best = draw_below(ws.at(first), (uint32_t)m);
  double fb = F(best);
  for (int j = 1; j < s; ++j) {
    const int32_t c = draw_below(ws.at(first + j), (uint32_t)m);
    const double fc = F(c);
    if (fc < fb) {
      best = c;
      fb = fc;
    }
  }
  return best;
}

template <typename View>
__device__ gsgp_record draw_record(const Params& p, uint32_t run_id, int gen_draw, int i, View F) {
  WordStream ws{(uint32_t)i, (uint32_t)gen_draw, p.seed, run_id, -1, Words4{0, 0, 0, 0}};
  const uint32_t w0 = ws.at(0), w1 = ws.at(1), w2 = ws.at(2), w3 = ws.at(3), w4 = ws.at(4);
  gsgp_record rc;
  rc.reserved = 0;
  if (p.tsize > 0 && (uint64_t)w0 < p.t_xo) {
    rc.op = 1;
    rc.p1 = tournament(ws, 5, p.tsize, p.m, F);
    rc.p2 = tournament(ws, 5 + p.tsize, p.tsize, p.m, F);
    rc.r1 = draw_below(w1, (uint32_t)p.r);
    rc.r2 = -1;
    rc.ms = 0.0;
  } else {
    rc.op = 0;
    rc.p1 = p.tsize > 0 ? tournament(ws, 5, p.tsize, p.m, F) : i;
    rc.p2 = -1;
    rc.r1 = draw_below(w1, (uint32_t)p.r);
    rc.r2 = draw_below(w2, (uint32_t)p.r);
    rc.ms = p.ms_random ? p.ms * draw_u53(w3, w4) : p.ms;
  }
  return rc;
}

// Block-wide reduction of three extrema in one pass: argmin of a, argmin of
// b, argmax of b (lowest index on ties).
template <typename A, typename B>
__device__ void block_arg3(int m, A fa, B fb, ValIdx* sh, ValIdx& min_a, ValIdx& min_b, ValIdx& max_b) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  ValIdx x{INFINITY, 0x7fffffff}, y{INFINITY, 0x7fffffff}, z{-INFINITY, 0x7fffffff};
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double va = fa(i), vb = fb(i);
    x = pick_min(x, ValIdx{va, i});
    y = pick_min(y, ValIdx{vb, i});
    z = pick_max(z, ValIdx{vb, i});
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    x = pick_min(x, ValIdx{__shfl_xor(x.v, o, kWave), __shfl_xor(x.i, o, kWave)});
    y = pick_min(y, ValIdx{__shfl_xor(y.v, o, kWave), __shfl_xor(y.i, o, kWave)});
    z = pick_max(z, ValIdx{__shfl_xor(z.v, o, kWave), __shfl_xor(z.i, o, kWave)});
  }
  if (lane == 0) {
    sh[wave] = x;
    sh[8 + wave] = y;
    sh[16 + wave] = z;
  }
  __syncthreads();
  min_a = sh[0];
  min_b = sh[8];
  max_b = sh[16];
  for (int w = 1; w < nw; ++w) {
    min_a = pick_min(min_a, sh[w]);
    min_b = pick_min(min_b, sh[8 + w]);
    max_b = pick_max(max_b, sh[16 + w]);
  }
  __syncthreads();
  // fitness is always finite; keep indices in range regardless
  if (min_a.i < 0 || min_a.i >= m) min_a.i = 0;
  if (min_b.i < 0 || min_b.i >= m) min_b.i = 0;
  if (max_b.i < 0 || max_b.i >= m) max_b.i = 0;
}

constexpr int kSurvLdsMaxM = 4096;  // parents + offspring fitness staged in LDS up to this m

// Survival with elitism (Section 2.2 "Survival"; Algorithm 1): offspring
// replace parents; when the best parent is strictly better than the best
// offspring it overwrites the worst offspring (lowest index on ties, as the
// first extremum that I?AMIN / I?AMAX return).  Then the summary and the next
// generation's draws.  surv_blks blocks per run share the elite row copy and
// the draws; each block stages the fitness arrays in LDS (LDS = true) and
// takes the survival decision redundantly; the last block to arrive
// publishes the elite fitness and advances the generation counter.
template <typename T, bool LDS>
__global__ __launch_bounds__(256) void k_survive(const RunDev* __restrict__ runs, Params p,
                                                 int32_t total, int mode) {
  extern __shared__ double fit[];  // [2 m] when LDS: parents, then offspring
  __shared__ ValIdx sh[24];
  __shared__ int is_last;
  const int run = find_run(p.n_runs, (int64_t)blockIdx.x, [&](int r) { return (int64_t)runs[r].surv_blk0; });
  const RunDev& R = runs[run];
  const int bl = blockIdx.x - R.surv_blk0;
  const int nb = R.surv_blks;
  const int m = p.m;
  const int gen = (mode == kSurvInit) ? 0 : R.state[kStGen];
  const int replay_elite = R.state[kStReplayElite];
  const int replay_select = R.state[kStReplaySelect];
  const int cur = gen & 1, nxt = cur ^ 1;
  const double* FP = R.F[cur];
  const double* FtP = R.Ft[cur];
  double* FO = R.F[nxt];
  double* FtO = R.Ft[nxt];
  const bool gen_mode = mode == kSurvGen;
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      fit[i] = FP[i];
      if (gen_mode) fit[m + i] = FO[i];
    }
    __syncthreads();
  }
  const double* fP = LDS ? fit : FP;
  const double* fO = LDS ? fit + m : FO;
  int copied = 0, src = -1, dst = -1;
  ValIdx bp, bo, wo;
  block_arg3(m, [&](int i) { return fP[i]; }, [&](int i) { return gen_mode ? fO[i] : fP[i]; }, sh, bp, bo, wo);
  if (gen_mode) {
    if (replay_elite) {
      const gsgp_gen_stats e = R.elite_in[gen];
      copied = e.elite_copied;
      src = e.elite_src;
      dst = e.elite_dst;
    } else if (bp.v < bo.v) {
      copied = 1;
      src = bp.i;
      dst = wo.i;
    }
    if (copied) {
      typedef typename VecOf<T>::type VT;
      constexpr int N = VecOf<T>::N;
      constexpr int64_t CH = chunk_cases(sizeof(T));
      const int64_t nvec = R.ld / N;
      const int64_t per = (nvec + nb - 1) / nb;
      const int64_t v0 = per * bl;
      const int64_t v1 = (v0 + per) < nvec ? (v0 + per) : nvec;
      const T* from = (const T*)R.S[cur];
      T* to = (T*)R.S[nxt];
      // four vectors in flight per thread; all N cases of a vector lie in one chunk.
      // With more than one wave, wave 0 takes the draws below while the
      // other waves copy, so the copy's memory latency overlaps the draws.
      constexpr int U = 4;
      const bool split = blockDim.x > kWave;
      const int ct = split ? (int)threadIdx.x - kWave : (int)threadIdx.x;
      const int cn = split ? (int)blockDim.x - kWave : (int)blockDim.x;
      const int64_t step = (int64_t)cn * U;
      if (ct >= 0) {
        for (int64_t v = v0 + ct; v < v1; v += step) {
          VT buf[U];
          int64_t at[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t w = v + (int64_t)u * cn;
            if (w < v1) {
              const int64_t col = w * N;
              buf[u] = *(const VT*)(from + tiled_index(R.tr_pad, R.te_pad, R.nch_tr, CH, m, src, col));
              at[u] = tiled_index(R.tr_pad, R.te_pad, R.nch_tr, CH, m, dst, col);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (v + (int64_t)u * cn < v1) *(VT*)(to + at[u]) = buf[u];
        }
      }
    }
  }
  // when the other waves copied the elite row, wave 0 alone takes the draws
  const bool draw_split = copied && blockDim.x > kWave;
  // fitness of the individuals the next draw selects from
  auto view_new = [&](int i) { return (copied && i == dst) ? fP[src] : fO[i]; };
  auto view_cur = [&](int i) { return fP[i]; };
  if (bl == 0 && mode != kSurvSelectOnly) {
    ValIdx b;
    if (gen_mode) {
      if (replay_elite) {
        b = block_arg<false>(m, view_new, sh);
      } else {
        // an elite copy is strictly better than every offspring
        b = copied ? ValIdx{fP[src], dst} : bo;
      }
    } else {
      b = bp;
    }
    if (threadIdx.x == 0) {
      gsgp_gen_stats st;
      st.best_train_rmse = b.v;
      st.best_test_rmse = gen_mode ? ((copied && b.i == dst) ? FtP[src] : FtO[b.i]) : FtP[b.i];
      st.best_index = b.i;
      st.elite_copied = copied;
      st.elite_src = src;
      st.elite_dst = dst;
      R.stats[gen_mode ? gen + 1 : 0] = st;
    }
  }
  const int gen_draw = gen_mode ? gen + 2 : gen + 1;
  if (!replay_select && gen_draw <= p.gmax) {
    const int per = (m + nb - 1) / nb;
    const int i0 = per * bl;
    const int i1 = (i0 + per) < m ? (i0 + per) : m;
    gsgp_record* out = R.rec + (int64_t)(gen_draw - 1) * m;
    const int dn = draw_split ? kWave : (int)blockDim.x;  // threads taking draws
    for (int i = i0 + (int)threadIdx.x; (int)threadIdx.x < dn && i < i1; i += dn) {
      out[i] = gen_mode ? draw_record(p, R.run_id, gen_draw, i, view_new)
                        : draw_record(p, R.run_id, gen_draw, i, view_cur);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int old = atomicAdd(&R.state[kStDone], 1);
    is_last = (old == nb - 1);
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    R.state[kStDone] = 0;
    if (gen_mode) {
      if (copied) {
        FO[dst] = FP[src];
        FtO[dst] = FtP[src];
        if (p.ls) {  // the copy keeps its source's scaling
          const int64_t m64 = m;
          R.ls[((int64_t)(gen + 1) * m64 + dst) * 2] = R.ls[((int64_t)gen * m64 + src) * 2];
          R.ls[((int64_t)(gen + 1) * m64 + dst) * 2 + 1] = R.ls[((int64_t)gen * m64 + src) * 2 + 1];
        }
      }
      R.state[kStGen] = gen + 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Lineage reconstruction helpers (all FP64).
__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ X, int64_t n, int32_t l,
                                                   double* __restrict__ Xfm, int64_t ld) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ld) return;
  for (int f = 0; f < l; ++f) Xfm[(int64_t)f * ld + c] = c < n ? X[c * l + f] : 0.0;
}

__global__ __launch_bounds__(256) void k_replay_nodes(const ReplayNode* __restrict__ nodes,
                                                      const double* __restrict__ prev,
                                                      const double* __restrict__ pool,
                                                      double* __restrict__ next, int64_t ld, int64_t n) {
  const ReplayNode nd = nodes[blockIdx.y];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double a = prev[(int64_t)nd.a * ld + c];
  double o;
  if (nd.op == 0) {
    o = a + nd.ms * (pool[(int64_t)nd.r1 * ld + c] - pool[(int64_t)nd.r2 * ld + c]);
  } else if (nd.op == 1) {
    const double r = pool[(int64_t)nd.r1 * ld + c];
    o = a * r + prev[(int64_t)nd.b * ld + c] * (1.0 - r);
  } else {
    o = a;
  }
  // local search: the offspring's recorded scaling (never for copies, and
  // skipped when it is the identity so that unscaled runs keep their bits)
  if (nd.op != 2 && (nd.alpha != 0.0 || nd.beta != 1.0)) o = nd.alpha + nd.beta * o;
  next[(int64_t)nd.out * ld + c] = o;
}

// Writes one state word of every run (generation counter, replay flags...).
__global__ void k_set_state(const RunDev* __restrict__ runs, int32_t n_runs, int32_t word, int32_t value) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_runs) runs[r].state[word] = value;
}



}  // namespace

hipError_t launch_set_state(const RunDev* d_runs, int32_t n_runs, int32_t word, int32_t value,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(blocks_for(n_runs, 256)), dim3(256), 0, s, d_runs, n_runs, word,
                     value);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
hipError_t launch_prep(const RunDev* d_runs, const Params& p, int64_t total_cols,
                       const double* const* Xsrc, const double* const* /*unused*/, hipStream_t s) {
  if (total_cols <= 0) return hipSuccess;
  if (p.precision == GSGP_FP64)
    hipLaunchKernelGGL(k_prep<double>, dim3(blocks_for(total_cols, 256)), dim3(256), 0, s, d_runs, p,
                       total_cols, Xsrc);
  else
    hipLaunchKernelGGL(k_prep<float>, dim3(blocks_for(total_cols, 256)), dim3(256), 0, s, d_runs, p,
                       total_cols, Xsrc);
  return hipGetLastError();
}

hipError_t launch_genome(const RunDev* d_runs, const Params& p, hipStream_t s) {
  const int64_t total = (int64_t)p.n_runs * (p.m + p.r) * p.k;
  hipLaunchKernelGGL(k_genome, dim3(blocks_for(total, 256)), dim3(256), 0, s, d_runs, p, total);
  return hipGetLastError();
}

template <typename T, int PREC>
void launch_vary_as(const RunDev* d_runs, const Params& p, const VaryLaunch& lc, bool rows_only, bool one_shot,
                    dim3 grid, dim3 block, hipStream_t s) {
  if (rows_only) {
    if (one_shot)
      hipLaunchKernelGGL((k_vary<T, PREC, true, false, false>), grid, block, 0, s, d_runs, p, lc);
    else
      hipLaunchKernelGGL((k_vary<T, PREC, true, true, false>), grid, block, 0, s, d_runs, p, lc);
  } else if (p.ls) {
    // local search sums are FP64 in every form, so one instance per storage type
    if constexpr (PREC != GSGP_FP32_KAHAN) {
      if (one_shot)
        hipLaunchKernelGGL((k_vary<T, PREC, false, false, true>), grid, block, 0, s, d_runs, p, lc);
      else
        hipLaunchKernelGGL((k_vary<T, PREC, false, true, true>), grid, block, 0, s, d_runs, p, lc);
    } else {
      launch_vary_as<T, GSGP_FP32>(d_runs, p, lc, rows_only, one_shot, grid, block, s);
    }
  } else {
    if (one_shot)
      hipLaunchKernelGGL((k_vary<T, PREC, false, false, false>), grid, block, 0, s, d_runs, p, lc);
    else
      hipLaunchKernelGGL((k_vary<T, PREC, false, true, false>), grid, block, 0, s, d_runs, p, lc);
  }
}

hipError_t launch_vary(const RunDev* d_runs, const Params& p, const VaryLaunch& lc, bool rows_only,
                       hipStream_t s) {
  if (lc.total_tasks <= 0) return hipSuccess;
  const dim3 grid((unsigned)lc.grid), block(lc.waves * kWave);
  // every task in the first sweep of the grid: the loop-free instance
  const int64_t sweep = lc.remap == 2 ? (lc.total_tasks + 8 * (int64_t)lc.ogroups - 1) / (8 * (int64_t)lc.ogroups) *
                                            (8 * (int64_t)lc.ogroups)
                                      : lc.total_tasks;
  const bool one_shot = lc.grid >= sweep;
  switch (p.precision) {
    case GSGP_FP64:
      launch_vary_as<double, GSGP_FP64>(d_runs, p, lc, rows_only, one_shot, grid, block, s);
      break;
    case GSGP_FP32:
      launch_vary_as<float, GSGP_FP32>(d_runs, p, lc, rows_only, one_shot, grid, block, s);
      break;
    default:
      launch_vary_as<float, GSGP_FP32_KAHAN>(d_runs, p, lc, rows_only, one_shot, grid, block, s);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_fitness(const RunDev* d_runs, const Params& p, bool init, hipStream_t s) {
  const int32_t per_run = (p.m + kWave - 1) / kWave;
  if (p.ls && !init)
    hipLaunchKernelGGL(k_fitness_ls, dim3((unsigned)(per_run * p.n_runs)), dim3(kFitWaves * kWave), 0, s, d_runs,
                       p, per_run);
  else
    hipLaunchKernelGGL(k_fitness, dim3((unsigned)(per_run * p.n_runs)), dim3(kFitWaves * kWave), 0, s, d_runs, p,
                       per_run, init ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_target_sums(const RunDev* d_runs, const Params& p, hipStream_t s) {
  if (p.precision == GSGP_FP64)
    hipLaunchKernelGGL(k_target_sums<double>, dim3((unsigned)p.n_runs), dim3(256), 0, s, d_runs, p);
  else
    hipLaunchKernelGGL(k_target_sums<float>, dim3((unsigned)p.n_runs), dim3(256), 0, s, d_runs, p);
  return hipGetLastError();
}

hipError_t launch_survive(const RunDev* d_runs, const Params& p, int32_t total_blocks, int mode,
                          hipStream_t s) {
  const bool lds = p.m <= kSurvLdsMaxM;
  const size_t shmem = lds ? (size_t)2 * p.m * sizeof(double) : 0;
  const dim3 grid(total_blocks), block(256);
  if (p.precision == GSGP_FP64) {
    if (lds)
      hipLaunchKernelGGL((k_survive<double, true>), grid, block, shmem, s, d_runs, p, total_blocks, mode);
    else
      hipLaunchKernelGGL((k_survive<double, false>), grid, block, 0, s, d_runs, p, total_blocks, mode);
  } else {
    if (lds)
      hipLaunchKernelGGL((k_survive<float, true>), grid, block, shmem, s, d_runs, p, total_blocks, mode);
    else
      hipLaunchKernelGGL((k_survive<float, false>), grid, block, 0, s, d_runs, p, total_blocks, mode);
  }
  return hipGetLastError();
}

hipError_t launch_transpose(const double* X, int64_t n, int32_t l, double* Xfm, int64_t ld,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3(blocks_for(ld, 256)), dim3(256), 0, s, X, n, l, Xfm, ld);
  return hipGetLastError();
}

hipError_t launch_replay_nodes(const ReplayNode* nodes, int32_t nnodes, const double* prev,
                               const double* pool, double* next, int64_t ld, int64_t n,
                               hipStream_t s) {
  if (nnodes <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_replay_nodes, dim3(blocks_for(n, 256), (unsigned)nnodes), dim3(256), 0, s, nodes,
                     prev, pool, next, ld, n);
  return hipGetLastError();
}

}  // namespace gsgp
