// Internal structures shared by the HIP kernels and the host runtime of
// libgsgp.so.  Nothing here is part of the public ABI (include/gsgp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsgp.h"

namespace gsgp {

// Canonical case chunk: fitness partial sums are formed over these runs of
// consecutive cases of one segment (train or test), in a fixed order, and
// combined in FP64 in chunk order.  Launch shapes never change the chunking,
// so fitness bits (and therefore selection) do not depend on tuning.  A
// chunk is 2 KiB of one semantic row (512 FP32 or 256 FP64 cases): each
// offspring task then reads and writes 2 KiB contiguous per row, which keeps
// HBM efficient under the random row order of the operators, and one chunk
// column of a large population (its distinct parent and pool rows) stays
// closer to an XCD's L2 (2 KiB against 4 KiB chunks: 1-2 % less time per
// generation on 256-, 1,024- and 2,048-row populations).
constexpr int kChunkBytes = 2048;
constexpr int chunk_cases(int storage_bytes) { return kChunkBytes / storage_bytes; }
// Each segment (train, test) of a semantic row is padded with zeros to a
// multiple of this many cases; rows therefore start 256-byte aligned.
constexpr int kSegPad = 64;
constexpr int kWave = 64;
// Interpreter work unit: a block of kInterpCases cases (kWave lanes x 2 cases).
constexpr int kInterpCases = 128;
// X is stored in tiles of kXTile cases, each tile feature-major: element
// (case c, feature f) at ((c / kXTile) * l + f) * kXTile + c % kXTile.  One
// tile's features (l x 2 KiB) are contiguous, so the rows an interpreter
// block reads spread over every L2 channel and few pages, where a
// feature-major [l][ld] layout put them ld x 8 bytes apart.
constexpr int kXTile = 256;
__host__ __device__ constexpr int64_t x_index(int64_t c, int64_t f, int64_t l) {
  return ((c / kXTile) * l + f) * kXTile + c % kXTile;
}
constexpr int kMaxTournament = 64;
// The interpreter keeps the top two stack values in registers and the rest
// (depth - 2 values per lane) in a lane-strided column: in LDS up to this
// many values (63 x 2 cases x 64 lanes x 8 B = 63 KiB, one wave per block),
// beyond it in a global-memory region of the workspace that a spill pass of
// kSpillWaves waves shares, one column per wave.
constexpr int kMaxLdsSlots = 63;
constexpr int kSpillWaves = 128;
// Stack values below the top two that a genome of k genes can need: its
// deepest stack up to its last valid function is at most k - 1 values.
constexpr int64_t max_need(int64_t k) { return k > 3 ? k - 3 : 0; }
// The interpreter runs in passes by stack need (LDS values per lane below
// the two stack values kept in registers), each with the smallest LDS
// column that holds its programs, so that a CU keeps as many waves resident
// as the column allows: the compile step files each run's programs into
// kLists lists; list b < kLists - 1 holds the programs whose need lies in
// (kListSlots[b - 1], kListSlots[b]] (list 0: need <= kListSlots[0]); the
// last list holds every deeper program (two-cases-per-lane passes with
// columns up to kMaxLdsSlots, then the spill pass).
constexpr int kLists = 5;
constexpr int kListSlots[kLists - 1] = {2, 3, 4, 6};
__host__ __device__ constexpr int list_of(int need) {
  return need <= 2 ? 0 : need == 3 ? 1 : need == 4 ? 2 : need <= 6 ? 3 : 4;
}
static_assert(list_of(kListSlots[0]) == 0 && list_of(kListSlots[1]) == 1 && list_of(kListSlots[2]) == 2 &&
                  list_of(kListSlots[3]) == 3 && list_of(kListSlots[3] + 1) == kLists - 1,
              "list_of must follow kListSlots");
// The interpreter reads a program's ops eight at a time; the compiled-op
// buffers carry this many entries of padding after the last program.
constexpr int kOpPad = 8;

// Compiled genome op word:
//   bits 0..1   the function (OpFn), or for a push which terminal (OpPush);
//   bits 2..3   the class (OpClass);
//   bits 4..15  stack depth before the op (values, top included);
//   bits 16..31 feature index.
// A push directly followed by a function it feeds is compiled into one op
// (kClsFeature / kClsConst) that applies the function to the top of the
// stack and the terminal, leaving the rest of the stack untouched.  The op's
// constant slot holds the constant of a constant op and, for a feature op,
// the bits of the absolute address of the feature's row in the run's X.  The
// word after a program's last op is an end word (push class, bit 1 set).
enum OpClass : int32_t { kClsPush = 0, kClsStack = 1, kClsFeature = 2, kClsConst = 3 };
enum OpFn : int32_t { kFnAdd = 0, kFnSub = 1, kFnMul = 2, kFnDiv = 3 };
enum OpPush : int32_t { kPushFeature = 0, kPushConst = 1 };
constexpr int kOpDepthMax = 0xFFF;

// Per-run device state words.
enum StateWord : int {
  kStGen = 0,           // last completed generation
  kStDone = 1,          // arrival counter of the survival kernel's blocks
  kStReplaySelect = 2,  // 1: variation draws are supplied, do not draw
  kStReplayElite = 3,   // 1: survival decisions are supplied
  kStMaxDepth = 4,      // deepest stack of the compiled genomes
  kStNonFinite = 5,     // set when X or y holds NaN / Inf
  kStList0 = 6,         // kLists words: the number of programs in each stack-need list
  kStXBig = 11,         // set when X holds a value beyond 2^128 in magnitude
  kStWords = 12
};

// Everything a kernel needs to know about one run; lives in the workspace.
struct RunDev {
  void* S[2];               // population semantics ping-pong, [m][ld], storage type
  void* sigR;               // squashed pool semantics, [r][ld]
  void* y;                  // target, [ld], storage type, zero pads
  double* X;                // features in case tiles, [ceil(ld / kXTile)][l][kXTile], zero pads
  double* part;             // chunk partial sums of squared residuals, [nch][m]; with local
                            // search the generation's sums of o, o^2 and o * t, [nch][3][m]
  double* F[2];             // train RMSE ping-pong, [m]
  double* Ft[2];            // test RMSE ping-pong, [m]
  gsgp_record* rec;         // variation draws, [gmax][m]; generation g at g - 1
  gsgp_gen_stats* stats;    // [gmax + 1]
  gsgp_gen_stats* elite_in; // supplied survival decisions, [gmax]
  int32_t* code;            // genomes, [m + r][k]
  double* cval;             // [m + r][k]
  int32_t* ops;             // compiled genomes, [m + r][k] + kOpPad
  double* opv;              // [m + r][k] + kOpPad
  double* opy;              // per compiled op: a constant divisor's refined reciprocal, else 0, [m + r][k] + kOpPad
  int32_t* nops;            // [m + r]
  int32_t* need;            // LDS stack values per lane each program needs, [m + r]
  int32_t* lists;           // programs by stack need, [kLists][m + r] (counts in kStList0 ..)
  int32_t* state;           // [kStWords]
  double* ls;               // local search: (alpha, beta) of every individual, [gmax + 1][m][2]
  double* tsum;             // local search: sum t and sum t^2 over train, then over test cases
  int64_t n_train, n_test;  // real cases
  int64_t tr_pad, te_pad;   // padded segment lengths
  int64_t ld;               // row stride (tr_pad + te_pad)
  int32_t l;                // features
  int32_t nch_tr, nch_te, nch;  // chunks per segment and in total
  uint32_t run_id;
  int32_t surv_blk0, surv_blks; // survival kernel blocks of this run
  int32_t x_big;            // X holds a value beyond 2^128 in magnitude (no short division by features)
  int64_t vary_task0;       // first task of this run in the variation launch
  int64_t cblk0;            // first 128-case block of this run (interpreter)
  int64_t cblk0w;           // first 256-case block of this run (wide interpreter)
  int64_t col0;             // first padded column of this run (data prep)
};

// Run-independent parameters, passed by value to every kernel.
struct Params {
  int32_t m, r, k, gmax;
  int32_t tsize, ms_random;
  int32_t n_runs, precision;
  int32_t ls, pad1;                // ls: least-squares scaling of every variation offspring
  uint64_t t_xo, t_func, t_feat;  // event thresholds floor(p * 2^32)
  double ms, erc_lo, erc_hi;
  uint32_t seed;
  int32_t pad;
};

// Chunk-tiled layout of every semantic buffer (population, pool): the
// padded columns of a run are cut into chunks (train segment first, then
// test), and each chunk stores the slices of all rows one after another.
// Element (row i, column col) of a buffer with `rows` rows lives at
//   rows * cs + i * len + (col - cs)
// where cs and len are the first column and the length of col's chunk.  One
// chunk's parents, pool trees and offspring thus sit in three contiguous
// blocks, which keeps address translation and DRAM pages local while the
// operators pick rows at random.
struct ChunkGeom {
  int64_t cs;   // first padded column of the chunk
  int64_t len;  // columns in the chunk (a multiple of kSegPad)
};

__host__ __device__ inline ChunkGeom chunk_geom(int64_t tr_pad, int64_t te_pad, int32_t nch_tr, int32_t c,
                                                int64_t chunk) {
  ChunkGeom g;
  if (c < nch_tr) {
    g.cs = (int64_t)c * chunk;
    g.len = tr_pad - g.cs;
  } else {
    const int64_t k = (int64_t)(c - nch_tr) * chunk;
    g.cs = tr_pad + k;
    g.len = te_pad - k;
  }
  if (g.len > chunk) g.len = chunk;
  return g;
}

// Index of (row i, padded column col) in a chunk-tiled buffer of `rows` rows.
__host__ __device__ inline int64_t tiled_index(int64_t tr_pad, int64_t te_pad, int32_t nch_tr, int64_t chunk,
                                               int64_t rows, int64_t i, int64_t col) {
  const int32_t c = col < tr_pad ? (int32_t)(col / chunk) : nch_tr + (int32_t)((col - tr_pad) / chunk);
  const ChunkGeom g = chunk_geom(tr_pad, te_pad, nch_tr, c, chunk);
  return rows * g.cs + i * g.len + (col - g.cs);
}

// Launch shape of the variation kernel.
struct VaryLaunch {
  int32_t waves;         // waves per block
  int32_t opb;           // offspring per block task
  int32_t ogroups;       // ceil(m / opb)
  int32_t remap;         // 1: XCD-aware block order
  int64_t total_tasks;   // sum over runs of nch * ogroups
  int64_t grid;          // blocks launched
};

enum SurviveMode : int32_t { kSurvInit = 0, kSurvGen = 1, kSurvSelectOnly = 2 };

// Host-side launchers (kernels.hip).  All enqueue on `s` and return the
// launch status.
hipError_t launch_prep(const RunDev* d_runs, const Params& p, int64_t total_cols,
                       const double* const* Xsrc, const double* const* ysrc, hipStream_t s);
hipError_t launch_set_state(const RunDev* d_runs, int32_t n_runs, int32_t word, int32_t value,
                            hipStream_t s);
hipError_t launch_genome(const RunDev* d_runs, const Params& p, hipStream_t s);
hipError_t launch_compile(const RunDev* d_runs, const Params& p, hipStream_t s);
// Interpreter passes: each takes the programs of stack-need list `list` (at
// most `progs` per run) with lo < need <= slots.  launch_interpret: two
// cases per lane, any slots up to kMaxLdsSlots, case_blocks blocks of
// kInterpCases cases; launch_interpret_wide: list < kLists - 1, whose
// programs need at most kListSlots[list] values, two or four cases per lane
// (blocks of kInterpCases or kXTile cases over all runs: blocks128,
// blocks256).
hipError_t launch_interpret(const RunDev* d_runs, const Params& p, int64_t case_blocks, int lo, int slots,
                            int list, int32_t progs, hipStream_t s);
hipError_t launch_interpret_wide(const RunDev* d_runs, const Params& p, int64_t blocks256, int64_t blocks128, int lo,
                                 int list, int32_t progs, hipStream_t s);
// Last pass: every program of the last list whose need exceeds kMaxLdsSlots,
// with its stack in `spill` (kSpillWaves columns of slots x 2 x 64 doubles).
hipError_t launch_interpret_spill(const RunDev* d_runs, const Params& p, double* spill, int slots,
                                  hipStream_t s);
hipError_t launch_vary(const RunDev* d_runs, const Params& p, const VaryLaunch& lc, bool rows_only,
                       hipStream_t s);
hipError_t launch_fitness(const RunDev* d_runs, const Params& p, bool init, hipStream_t s);
// Local search: sums of the stored target over each run's train and test cases.
hipError_t launch_target_sums(const RunDev* d_runs, const Params& p, hipStream_t s);
hipError_t launch_survive(const RunDev* d_runs, const Params& p, int32_t total_blocks, int mode,
                          hipStream_t s);
// Reconstruction helpers.
hipError_t launch_transpose(const double* X, int64_t n, int32_t l, double* Xfm, int64_t ld,
                            hipStream_t s);
hipError_t launch_interpret_list(const int32_t* ops, const double* opv, const int32_t* nops,
                                 int32_t k, const int32_t* prog, const int32_t* squash,
                                 int32_t nprog, const double* Xfm, int64_t ld, int64_t n,
                                 double* out, int slots, double* spill, hipStream_t s);
struct ReplayNode {
  int32_t op;     // 0 mutation, 1 crossover, 2 copy
  int32_t a, b;   // source slots (previous generation); b = -1 unless crossover
  int32_t r1, r2; // pool slots
  int32_t out;    // destination slot
  double ms;
  double alpha, beta;  // local search: the offspring is alpha + beta * (operator output)
};
hipError_t launch_replay_nodes(const ReplayNode* nodes, int32_t nnodes, const double* prev,
                               const double* pool, double* next, int64_t ld, int64_t n,
                               hipStream_t s);

}  // namespace gsgp
