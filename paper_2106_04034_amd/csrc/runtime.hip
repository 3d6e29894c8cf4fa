// Host runtime of libgsgp.so: argument validation, workspace carving,
// launch planning, HIP graph capture of a generation, inspection and lineage
// reconstruction.  Implements the C ABI declared in include/gsgp.h.
//
// Algorithm 1 of the GSGP-CUDA paper (arXiv 2106.04034) is the control flow:
// gsgp_eval_population runs its set-up (CreatePopulation x2,
// ComputeSemantics x2, ComputeFitness) and gsgp_generation its loop body.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "common.hpp"

using namespace gsgp;

// Device scratch of gsgp_reconstruct_static, for callers that cannot
// allocate: one copy of this array on every GPU the library runs on, held
// until the process ends.  Host code never uses the array's name as an
// address; it uses the per-device address that hipGetSymbolAddress returns.
constexpr size_t kStaticScratchBytes = GSGP_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
struct StaticScratch {
  std::mutex call;       // one reconstruction at a time on this device
  char* ptr = nullptr;   // device address of `scratch` on this device
};
StaticScratch g_static[kMaxDevices];
std::mutex g_static_setup;

// Resolves the device's copy of `scratch` once, with that device current.
hipError_t resolve_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipSuccess;  // the static entry point refuses such devices
  std::lock_guard<std::mutex> lock(g_static_setup);
  if (g_static[device].ptr) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_static[device].ptr = (char*)p;
  return hipSuccess;
}

thread_local std::string g_last_error;

gsgp_status fail(gsgp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
inline int64_t pad_to(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

uint64_t event_threshold(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

size_t storage_bytes(int32_t precision) { return precision == GSGP_FP64 ? 8 : 4; }

// Byte offsets of one run's buffers inside the workspace.
struct RunPlan {
  int64_t n_train, n_test, tr_pad, te_pad, ld;
  int32_t l, nch_tr, nch_te;
  size_t X, y, S0, S1, sigR, part, F0, F1, Ft0, Ft1, rec, stats, elite_in, code, cval, ops, opv, opy, nops, need, lists;
  size_t ls, tsum;
  size_t end;
};

// With GSGP_FLAG_GUARDS every buffer is followed by kGuardBytes of a fixed
// pattern, checked after every call that launches kernels.
constexpr size_t kGuardBytes = 256;
constexpr uint32_t kGuardWord = 0xC0FFEE5Au;

struct Guard {
  size_t at;         // byte offset of the guard in the workspace
  int32_t run;       // -1 for the shared buffers
  const char* after; // the buffer it follows
};

struct Plan {
  size_t runs_dev, src_ptrs, state, spill, spill_bytes, total;
  std::vector<RunPlan> runs;
  std::vector<Guard> guards;
};

// Flags that change what a run computes (the others change only how).
constexpr uint32_t kResultFlags = GSGP_FLAG_LOCAL_SEARCH;

gsgp_status validate_config(const gsgp_config* c) {
  if (!c) return fail(GSGP_ERR_ARG, "config is NULL");
  if (c->pop_size < 1 || c->pop_size > (1 << 22)) return fail(GSGP_ERR_ARG, "pop_size %d out of [1, 2^22]", c->pop_size);
  if (c->pool_size < 1 || c->pool_size > (1 << 22)) return fail(GSGP_ERR_ARG, "pool_size %d out of [1, 2^22]", c->pool_size);
  if (c->genome_len < 1 || c->genome_len > 4096) return fail(GSGP_ERR_ARG, "genome_len %d out of [1, 4096]", c->genome_len);
  if (c->n_generations_max < 1 || c->n_generations_max > (1 << 24))
    return fail(GSGP_ERR_ARG, "n_generations_max %d out of [1, 2^24]", c->n_generations_max);
  if (c->tournament_size < 0 || c->tournament_size > kMaxTournament)
    return fail(GSGP_ERR_ARG, "tournament_size %d out of [0, %d]", c->tournament_size, kMaxTournament);
  if (c->ms_random != 0 && c->ms_random != 1) return fail(GSGP_ERR_ARG, "ms_random must be 0 or 1");
  if (!(c->p_crossover >= 0.0 && c->p_crossover <= 1.0)) return fail(GSGP_ERR_ARG, "p_crossover out of [0, 1]");
  if (c->tournament_size == 0 && c->p_crossover != 0.0)
    return fail(GSGP_ERR_ARG, "tournament_size 0 (mutate every individual) requires p_crossover == 0");
  if (!(c->mutation_step >= 0.0 && c->mutation_step <= 1e6)) return fail(GSGP_ERR_ARG, "mutation_step out of [0, 1e6]");
  if (!(c->p_function >= 0.0 && c->p_function <= 1.0) || !(c->p_feature >= 0.0 && c->p_feature <= 1.0) ||
      !(c->p_function + c->p_feature <= 1.0 + 1e-12))
    return fail(GSGP_ERR_ARG, "gene probabilities must lie in [0, 1] and sum to at most 1");
  if (!std::isfinite(c->erc_lo) || !std::isfinite(c->erc_hi) || c->erc_lo > c->erc_hi ||
      std::fabs(c->erc_lo) > 3.0e38 || std::fabs(c->erc_hi) > 3.0e38)
    return fail(GSGP_ERR_ARG, "constant range must be finite with erc_lo <= erc_hi");
  if (c->precision < GSGP_FP64 || c->precision > GSGP_FP32_KAHAN) return fail(GSGP_ERR_ARG, "unknown precision %d", c->precision);
  if ((c->flags & ~(GSGP_FLAG_NO_GRAPH | GSGP_FLAG_GUARDS | GSGP_FLAG_LOCAL_SEARCH)) != 0)
    return fail(GSGP_ERR_ARG, "unknown flags 0x%x", c->flags);
  if (c->reserved != 0) return fail(GSGP_ERR_ARG, "reserved config field must be 0");
  return GSGP_OK;
}

gsgp_status make_plan(const gsgp_config* c, const gsgp_run* runs, int32_t n_runs, Plan* plan) {
  gsgp_status st = validate_config(c);
  if (st != GSGP_OK) return st;
  if (!runs || n_runs < 1 || n_runs > 65536) return fail(GSGP_ERR_ARG, "need 1..65536 runs");
  const int64_t m = c->pop_size, r = c->pool_size, k = c->genome_len, G = c->n_generations_max;
  const size_t s = storage_bytes(c->precision);
  const bool guarded = (c->flags & GSGP_FLAG_GUARDS) != 0;
  const bool ls = (c->flags & GSGP_FLAG_LOCAL_SEARCH) != 0;
  plan->guards.clear();
  size_t off = 0;
  // reserves `bytes` at the next aligned offset, plus a guard when asked
  auto take_at = [&](size_t bytes, int32_t run, const char* name) {
    const size_t at = off;
    if (guarded) {
      plan->guards.push_back(Guard{at + bytes, run, name});
      bytes += kGuardBytes;
    }
    off = align_up(off + bytes);
    return at;
  };
  plan->runs_dev = take_at(sizeof(RunDev) * n_runs, -1, "run descriptors");
  plan->src_ptrs = take_at(sizeof(double*) * 4 * n_runs, -1, "input pointers");
  plan->state = take_at(sizeof(int32_t) * kStWords * n_runs, -1, "state words");
  // stack columns of the interpreter's spill pass, sized for the deepest
  // stack a genome of k genes can need; none when every stack fits in LDS
  const int64_t need_cap = max_need(k);
  plan->spill_bytes = need_cap > kMaxLdsSlots ? sizeof(double) * kSpillWaves * need_cap * 2 * kWave : 0;
  plan->spill = take_at(plan->spill_bytes, -1, "interpreter spill stacks");
  plan->runs.resize(n_runs);
  for (int32_t i = 0; i < n_runs; ++i) {
    const gsgp_run& d = runs[i];
    if (d.n_train < 1) return fail(GSGP_ERR_ARG, "run %d: n_train must be >= 1", i);
    if (d.n_test < 0) return fail(GSGP_ERR_ARG, "run %d: n_test must be >= 0", i);
    if (d.n_train > ((int64_t)1 << 40) || d.n_test > ((int64_t)1 << 40)) return fail(GSGP_ERR_ARG, "run %d: too many cases", i);
    if (d.n_features < 1 || d.n_features > 65535) return fail(GSGP_ERR_ARG, "run %d: n_features out of [1, 65535]", i);
    if (d.reserved != 0) return fail(GSGP_ERR_ARG, "run %d: reserved field must be 0", i);
    if (!d.X_train || !d.y_train) return fail(GSGP_ERR_ARG, "run %d: NULL train data", i);
    if ((d.n_test > 0) != (d.X_test != nullptr) || (d.n_test > 0) != (d.y_test != nullptr))
      return fail(GSGP_ERR_ARG, "run %d: test pointers must be non-NULL iff n_test > 0", i);
    RunPlan& p = plan->runs[i];
    p.n_train = d.n_train;
    p.n_test = d.n_test;
    p.l = d.n_features;
    p.tr_pad = pad_to(d.n_train, kSegPad);
    p.te_pad = pad_to(d.n_test, kSegPad);
    p.ld = p.tr_pad + p.te_pad;
    const int64_t chunk = chunk_cases((int)s);
    p.nch_tr = (int32_t)((p.tr_pad + chunk - 1) / chunk);
    p.nch_te = (int32_t)((p.te_pad + chunk - 1) / chunk);
    p.X = take_at(sizeof(double) * p.l * ((p.ld + kXTile - 1) / kXTile) * kXTile, i, "X");
    p.y = take_at(s * p.ld, i, "y");
    p.S0 = take_at(s * m * p.ld, i, "S[0]");
    p.S1 = take_at(s * m * p.ld, i, "S[1]");
    p.sigR = take_at(s * r * p.ld, i, "sigmoid(S_R)");
    // chunk partial sums: one per individual, three with local search
    p.part = take_at(sizeof(double) * (p.nch_tr + p.nch_te) * m * (ls ? 3 : 1), i, "chunk partial sums");
    p.F0 = take_at(8 * m, i, "F[0]");
    p.F1 = take_at(8 * m, i, "F[1]");
    p.Ft0 = take_at(8 * m, i, "Ft[0]");
    p.Ft1 = take_at(8 * m, i, "Ft[1]");
    p.rec = take_at(sizeof(gsgp_record) * G * m, i, "variation records");
    p.stats = take_at(sizeof(gsgp_gen_stats) * (G + 1), i, "summaries");
    p.elite_in = take_at(sizeof(gsgp_gen_stats) * G, i, "supplied survival decisions");
    p.code = take_at(4 * (m + r) * k, i, "genome codes");
    p.cval = take_at(8 * (m + r) * k, i, "genome constants");
    p.ops = take_at(4 * ((m + r) * k + kOpPad), i, "compiled ops");
    p.opv = take_at(8 * ((m + r) * k + kOpPad), i, "compiled constants");
    p.opy = take_at(8 * ((m + r) * k + kOpPad), i, "compiled reciprocals");
    p.nops = take_at(4 * (m + r), i, "program lengths");
    p.need = take_at(4 * (m + r), i, "program stack needs");
    p.lists = take_at(4 * kLists * (m + r), i, "program lists by stack need");
    // local search: the scaling table of every generation and the target sums
    p.ls = take_at(ls ? sizeof(double) * 2 * (G + 1) * m : 0, i, "scaling table");
    p.tsum = take_at(ls ? sizeof(double) * 4 : 0, i, "target sums");
    p.end = off;
  }
  plan->total = off;
  return GSGP_OK;
}

}  // namespace

struct gsgp_handle {
  gsgp_config cfg;
  int32_t n_runs = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  char* ws = nullptr;
  Plan plan;
  std::vector<RunDev> runs_h;
  RunDev* runs_d = nullptr;
  Params params;
  VaryLaunch vary{}, rows{};
  int64_t interp_tasks = 0;  // interpreter case blocks over all runs
  int64_t interp_tasks_w = 0;  // wide interpreter case blocks over all runs
  int32_t surv_blocks = 0;
  int32_t slots = 1;         // interpreter stack values per lane in LDS
  int32_t max_blocks = 0;
  int32_t gen = 0;
  bool evaluated = false;
  bool poisoned = false;
  hipGraph_t graph = nullptr;       // one generation
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_k = nullptr;     // kGraphGens generations back to back
  hipGraphExec_t exec_k = nullptr;
  int32_t* pinned = nullptr;  // state read-back, [n_runs][kStWords]
  int device = 0;
};

namespace {

gsgp_status hip_fail(gsgp_handle* h, hipError_t e, const char* what) {
  if (h) h->poisoned = true;
  return fail(GSGP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(h, call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
  } while (0)

gsgp_status usable(gsgp_handle* h) {
  if (!h) return fail(GSGP_ERR_ARG, "handle is NULL");
  if (h->poisoned) return fail(GSGP_ERR_STATE, "handle is poisoned by an earlier error");
  return GSGP_OK;
}

// Writes the guard pattern after every buffer (GSGP_FLAG_GUARDS).
gsgp_status arm_guards(gsgp_handle* h) {
  std::vector<uint32_t> pat(kGuardBytes / 4, kGuardWord);
  for (const Guard& g : h->plan.guards)
    HIPCHK(h, hipMemcpy(h->ws + g.at, pat.data(), kGuardBytes, hipMemcpyHostToDevice));
  return GSGP_OK;
}

// After a call that launched kernels: `st` unless a guard was overwritten,
// which poisons the handle and names the buffer it follows.
gsgp_status check_guards(gsgp_handle* h, gsgp_status st) {
  if (st != GSGP_OK || h->plan.guards.empty()) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::vector<uint32_t> got(kGuardBytes / 4);
  for (const Guard& g : h->plan.guards) {
    HIPCHK(h, hipMemcpy(got.data(), h->ws + g.at, kGuardBytes, hipMemcpyDeviceToHost));
    for (uint32_t w : got) {
      if (w != kGuardWord) {
        h->poisoned = true;
        if (g.run < 0) return fail(GSGP_ERR_STATE, "workspace guard after the %s was overwritten", g.after);
        return fail(GSGP_ERR_STATE, "workspace guard after %s of run %d was overwritten", g.after, g.run);
      }
    }
  }
  return GSGP_OK;
}

void drop_graph(gsgp_handle* h) {
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->exec_k) (void)hipGraphExecDestroy(h->exec_k);
  if (h->graph_k) (void)hipGraphDestroy(h->graph_k);
  h->exec = nullptr;
  h->graph = nullptr;
  h->exec_k = nullptr;
  h->graph_k = nullptr;
}

// Variation launch for the current shape.  With remap the grid is a multiple
// of 8 so that logical blocks can be spread XCD by XCD.
void plan_vary(gsgp_handle* h, int32_t waves, int32_t opb, int32_t remap, int32_t max_blocks) {
  VaryLaunch& v = h->vary;
  v.waves = waves;
  v.opb = opb;
  h->max_blocks = max_blocks;
  v.ogroups = (h->cfg.pop_size + opb - 1) / opb;
  v.remap = remap;
  int64_t t = 0;
  for (int32_t i = 0; i < h->n_runs; ++i) {
    h->runs_h[i].vary_task0 = t;
    t += (int64_t)h->runs_h[i].nch * v.ogroups;
  }
  v.total_tasks = t;
  // max_blocks > 0 makes the launch persistent: blocks loop over tasks
  int64_t need = t;
  // remap 2 walks super-groups of 8 * ogroups tasks, one group per XCD
  if (remap == 2) need = pad_to(t, 8 * (int64_t)v.ogroups);
  int64_t grid = std::min<int64_t>(need, max_blocks > 0 ? max_blocks : ((int64_t)1 << 30));
  if (remap) grid = pad_to(grid, 8);
  v.grid = grid;
}

// The generation-0 partial sums use one task per (chunk, individual group)
// with the same indexing; offspring groups of the vary plan are reused.
void plan_rows(gsgp_handle* h) {
  h->rows = h->vary;
  h->rows.remap = 0;
  h->rows.grid = h->vary.total_tasks;
}

hipError_t upload_runs(gsgp_handle* h) {
  return hipMemcpyAsync(h->runs_d, h->runs_h.data(), sizeof(RunDev) * h->n_runs, hipMemcpyHostToDevice,
                        h->stream);
}

hipError_t enqueue_generation(gsgp_handle* h, hipStream_t s) {
  hipError_t e = launch_vary(h->runs_d, h->params, h->vary, false, s);
  if (e != hipSuccess) return e;
  e = launch_fitness(h->runs_d, h->params, false, s);
  if (e != hipSuccess) return e;
  return launch_survive(h->runs_d, h->params, h->surv_blocks, kSurvGen, s);
}

// Generations per graph of the long form.  Every kernel reads the generation
// counter from device memory, so a graph of any number of generations
// replays anywhere in a run.  Consecutive graph launches leave a longer gap
// between generations than consecutive kernels inside one graph: 1,000
// generations of single_fp32_100k take 246.6 ms with one generation per
// graph and 242.9 / 242.1 / 241.9 / 241.8 ms with 4 / 8 / 16 / 32.
constexpr int32_t kGraphGens = 16;

gsgp_status capture(gsgp_handle* h, int32_t n, hipGraph_t* graph, hipGraphExec_t* exec) {
  HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int32_t i = 0; i < n && e == hipSuccess; ++i) e = enqueue_generation(h, h->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
  if (e != hipSuccess) return hip_fail(h, e, "capturing generations");
  if (e2 != hipSuccess) return hip_fail(h, e2, "hipStreamEndCapture");
  *graph = g;
  HIPCHK(h, hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  return GSGP_OK;
}

gsgp_status ensure_graph(gsgp_handle* h) {
  if (!h->exec) {
    gsgp_status st = capture(h, 1, &h->graph, &h->exec);
    if (st != GSGP_OK) return st;
  }
  if (!h->exec_k) return capture(h, kGraphGens, &h->graph_k, &h->exec_k);
  return GSGP_OK;
}

gsgp_status run_generations(gsgp_handle* h, int32_t n_gens) {
  const bool graph = !(h->cfg.flags & GSGP_FLAG_NO_GRAPH);
  if (graph) {
    gsgp_status st = ensure_graph(h);
    if (st != GSGP_OK) return st;
    int32_t g = 0;
    for (; g + kGraphGens <= n_gens; g += kGraphGens) HIPCHK(h, hipGraphLaunch(h->exec_k, h->stream));
    for (; g < n_gens; ++g) HIPCHK(h, hipGraphLaunch(h->exec, h->stream));
  } else {
    for (int32_t g = 0; g < n_gens; ++g) HIPCHK(h, enqueue_generation(h, h->stream));
  }
  h->gen += n_gens;
  return GSGP_OK;
}

gsgp_status copy_stats(gsgp_handle* h, int32_t gen0, int32_t n, gsgp_gen_stats* out, int32_t stride) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int32_t r = 0; r < h->n_runs; ++r)
    HIPCHK(h, hipMemcpy(out + (size_t)r * stride, h->runs_h[r].stats + gen0, sizeof(gsgp_gen_stats) * n,
                        hipMemcpyDeviceToHost));
  return GSGP_OK;
}

gsgp_status check_run(gsgp_handle* h, int32_t run) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (run < 0 || run >= h->n_runs) return fail(GSGP_ERR_ARG, "run %d out of [0, %d)", run, h->n_runs);
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  return GSGP_OK;
}

// Local search: rows row0 .. row0 + n_rows - 1 of the current population
// are stored unscaled; their semantics are alpha + beta * S with the current
// generation's scaling (FP64, the same operations the variation kernel
// applies when it reads a parent).  out holds n_rows rows of `cols` values.
gsgp_status apply_scaling(gsgp_handle* h, int32_t run, int32_t row0, int32_t n_rows, int64_t cols, double* out) {
  if (!(h->cfg.flags & GSGP_FLAG_LOCAL_SEARCH)) return GSGP_OK;
  std::vector<double> ab((size_t)2 * n_rows);
  const double* table = h->runs_h[run].ls + ((int64_t)h->gen * h->cfg.pop_size + row0) * 2;
  HIPCHK(h, hipMemcpy(ab.data(), table, sizeof(double) * ab.size(), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < n_rows; ++i) {
    const double a = ab[2 * i], b = ab[2 * i + 1];
    if (a == 0.0 && b == 1.0) continue;
    double* row = out + (int64_t)i * cols;
    for (int64_t c = 0; c < cols; ++c) row[c] = a + b * row[c];
  }
  return GSGP_OK;
}

// Unpacks a chunk-tiled semantic buffer (see chunk_geom) into FP64 rows of
// n_train + n_test cases.
template <typename T>
void to_f64(const std::vector<char>& raw, int64_t rows, const RunDev& R, double* out) {
  const T* s = (const T*)raw.data();
  const int64_t n_all = R.n_train + R.n_test;
  const int64_t CH = chunk_cases((int)sizeof(T));
  for (int32_t c = 0; c < R.nch; ++c) {
    const ChunkGeom g = chunk_geom(R.tr_pad, R.te_pad, R.nch_tr, c, CH);
    const bool train = c < R.nch_tr;
    const int64_t first = train ? g.cs : g.cs - R.tr_pad;              // case index in its segment
    const int64_t real = (train ? R.n_train : R.n_test) - first;      // real cases left in the segment
    const int64_t used = std::min<int64_t>(g.len, std::max<int64_t>(real, 0));
    const int64_t out0 = train ? first : R.n_train + first;
    for (int64_t i = 0; i < rows; ++i) {
      const T* src = s + rows * g.cs + i * g.len;
      for (int64_t k = 0; k < used; ++k) out[i * n_all + out0 + k] = (double)src[k];
    }
  }
}

}  // namespace

extern "C" {

const char* gsgp_status_string(gsgp_status s) {
  switch (s) {
    case GSGP_OK: return "ok";
    case GSGP_ERR_ARG: return "invalid argument";
    case GSGP_ERR_STATE: return "invalid state";
    case GSGP_ERR_WORKSPACE: return "workspace too small or misaligned";
    case GSGP_ERR_NONFINITE: return "non-finite input";
    case GSGP_ERR_HIP: return "HIP error";
    case GSGP_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* gsgp_last_error(void) { return g_last_error.c_str(); }

gsgp_status gsgp_workspace_size(const gsgp_config* cfg, const gsgp_run* runs, int32_t n_runs, size_t* bytes) {
  if (!bytes) return fail(GSGP_ERR_ARG, "bytes is NULL");
  Plan plan;
  gsgp_status st = make_plan(cfg, runs, n_runs, &plan);
  if (st != GSGP_OK) return st;
  *bytes = plan.total;
  return GSGP_OK;
}

gsgp_status gsgp_init(const gsgp_config* cfg, const gsgp_run* runs, int32_t n_runs, void* d_workspace,
                      size_t ws_bytes, void* hip_stream, gsgp_handle** out) {
  if (!out) return fail(GSGP_ERR_ARG, "out is NULL");
  *out = nullptr;
  Plan plan;
  gsgp_status st = make_plan(cfg, runs, n_runs, &plan);
  if (st != GSGP_OK) return st;
  if (!d_workspace) return fail(GSGP_ERR_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)d_workspace) % kAlign) return fail(GSGP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < plan.total)
    return fail(GSGP_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, plan.total);

  gsgp_handle* h = new gsgp_handle();
  h->cfg = *cfg;
  h->n_runs = n_runs;
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char*)d_workspace;
  h->plan = plan;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = resolve_static_scratch(h->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->pinned, sizeof(int32_t) * kStWords * n_runs, hipHostMallocDefault);
  if (e != hipSuccess) {
    gsgp_status s2 = fail(GSGP_ERR_HIP, "creating handle resources: %s", hipGetErrorString(e));
    gsgp_destroy(h);
    return s2;
  }
  Params& p = h->params;
  p.m = cfg->pop_size;
  p.r = cfg->pool_size;
  p.k = cfg->genome_len;
  p.gmax = cfg->n_generations_max;
  p.tsize = cfg->tournament_size;
  p.ms_random = cfg->ms_random;
  p.n_runs = n_runs;
  p.precision = cfg->precision;
  p.t_xo = event_threshold(cfg->p_crossover);
  p.t_func = event_threshold(cfg->p_function);
  p.t_feat = event_threshold(cfg->p_function + cfg->p_feature);
  p.ms = cfg->mutation_step;
  p.erc_lo = cfg->erc_lo;
  p.erc_hi = cfg->erc_hi;
  p.seed = cfg->seed;
  p.pad = 0;
  p.ls = (cfg->flags & GSGP_FLAG_LOCAL_SEARCH) ? 1 : 0;
  p.pad1 = 0;

  char* ws = h->ws;
  h->runs_d = (RunDev*)(ws + plan.runs_dev);
  int32_t* state = (int32_t*)(ws + plan.state);
  h->runs_h.resize(n_runs);
  int64_t col = 0, itask = 0, itask_w = 0;
  int32_t sblk = 0;
  for (int32_t i = 0; i < n_runs; ++i) {
    const RunPlan& q = plan.runs[i];
    RunDev& R = h->runs_h[i];
    memset(&R, 0, sizeof R);
    R.S[0] = ws + q.S0;
    R.S[1] = ws + q.S1;
    R.sigR = ws + q.sigR;
    R.y = ws + q.y;
    R.X = (double*)(ws + q.X);
    R.part = (double*)(ws + q.part);
    R.F[0] = (double*)(ws + q.F0);
    R.F[1] = (double*)(ws + q.F1);
    R.Ft[0] = (double*)(ws + q.Ft0);
    R.Ft[1] = (double*)(ws + q.Ft1);
    R.rec = (gsgp_record*)(ws + q.rec);
    R.stats = (gsgp_gen_stats*)(ws + q.stats);
    R.elite_in = (gsgp_gen_stats*)(ws + q.elite_in);
    R.code = (int32_t*)(ws + q.code);
    R.cval = (double*)(ws + q.cval);
    R.ops = (int32_t*)(ws + q.ops);
    R.opv = (double*)(ws + q.opv);
    R.opy = (double*)(ws + q.opy);
    R.nops = (int32_t*)(ws + q.nops);
    R.need = (int32_t*)(ws + q.need);
    R.lists = (int32_t*)(ws + q.lists);
    R.ls = (double*)(ws + q.ls);
    R.tsum = (double*)(ws + q.tsum);
    R.state = state + (size_t)kStWords * i;
    R.n_train = q.n_train;
    R.n_test = q.n_test;
    R.tr_pad = q.tr_pad;
    R.te_pad = q.te_pad;
    R.ld = q.ld;
    R.l = q.l;
    R.nch_tr = q.nch_tr;
    R.nch_te = q.nch_te;
    R.nch = q.nch_tr + q.nch_te;
    R.run_id = (uint32_t)i;
    R.col0 = col;
    col += q.ld;
    R.cblk0 = itask;
    itask += (q.ld + kInterpCases - 1) / kInterpCases;
    R.cblk0w = itask_w;
    itask_w += (q.ld + 4 * kWave - 1) / (4 * kWave);
    R.surv_blk0 = sblk;
    // survival blocks per run: each copies about 16 KiB of an elite row
    const int64_t nb = ((int64_t)storage_bytes(cfg->precision) * q.ld + 16383) / 16384;
    R.surv_blks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nb, 64));
    sblk += R.surv_blks;
  }
  h->interp_tasks = itask;
  h->interp_tasks_w = itask_w;
  h->surv_blocks = sblk;
  plan_vary(h, 4, 16, 1, 0);
  plan_rows(h);

  std::vector<const double*> src(4 * (size_t)n_runs);
  for (int32_t i = 0; i < n_runs; ++i) {
    src[4 * i + 0] = runs[i].X_train;
    src[4 * i + 1] = runs[i].y_train;
    src[4 * i + 2] = runs[i].X_test;
    src[4 * i + 3] = runs[i].y_test;
  }
  const double* const* d_src = (const double* const*)(ws + plan.src_ptrs);
  std::vector<int32_t> zeros((size_t)kStWords * n_runs, 0);
  if (!h->plan.guards.empty() && arm_guards(h) != GSGP_OK) {
    gsgp_status s2 = fail(GSGP_ERR_HIP, "gsgp_init: writing the workspace guards");
    gsgp_destroy(h);
    return s2;
  }
  e = upload_runs(h);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void*)d_src, src.data(), sizeof(double*) * src.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(state, zeros.data(), sizeof(int32_t) * zeros.size(), hipMemcpyHostToDevice, h->stream);
  // X's last tile of each run is whole: its columns past the padded cases
  // are read by interpreter lanes whose values are never stored; zeros
  for (int32_t i = 0; i < n_runs && e == hipSuccess; ++i) {
    const RunPlan& q = plan.runs[i];
    e = hipMemsetAsync(ws + q.X, 0, sizeof(double) * q.l * ((q.ld + kXTile - 1) / kXTile) * kXTile, h->stream);
  }
  if (e == hipSuccess) e = launch_prep(h->runs_d, p, col, d_src, nullptr, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->pinned, state, sizeof(int32_t) * kStWords * n_runs, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    gsgp_status s2 = fail(GSGP_ERR_HIP, "gsgp_init: %s", hipGetErrorString(e));
    gsgp_destroy(h);
    return s2;
  }
  for (int32_t i = 0; i < n_runs; ++i) {
    if (h->pinned[kStWords * i + kStNonFinite]) {
      gsgp_destroy(h);
      return fail(GSGP_ERR_NONFINITE, "run %d: X or y holds NaN/Inf (or |y| > FLT_MAX)", i);
    }
    h->runs_h[i].x_big = h->pinned[kStWords * i + kStXBig];
  }
  e = upload_runs(h);
  if (e != hipSuccess) {
    gsgp_status s2 = fail(GSGP_ERR_HIP, "gsgp_init: %s", hipGetErrorString(e));
    gsgp_destroy(h);
    return s2;
  }
  if (check_guards(h, GSGP_OK) != GSGP_OK) {
    const std::string why = g_last_error;
    gsgp_destroy(h);
    return fail(GSGP_ERR_STATE, "gsgp_init: %s", why.c_str());
  }
  *out = h;
  return GSGP_OK;
}

gsgp_status gsgp_destroy(gsgp_handle* h) {
  if (!h) return GSGP_OK;
  drop_graph(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->pinned) (void)hipHostFree(h->pinned);
  delete h;
  return GSGP_OK;
}

namespace {

// ComputeSemantics of every compiled program, in one pass per stack-need
// list, each with the smallest LDS column that holds its programs (more
// resident waves for the shallow lists): the first kLists - 1 lists with the
// wide kernel, then the last list with columns up to kMaxLdsSlots, then the
// programs beyond any LDS column (spill stacks).  counts[b]: the longest
// list b over the runs.
hipError_t interpret_all(gsgp_handle* h, const int32_t (&counts)[kLists], hipStream_t s) {
  const Params& p = h->params;
  hipError_t e = hipSuccess;
  for (int b = 0; b < kLists - 1 && e == hipSuccess; ++b) {
    const int lo = b == 0 ? -1 : kListSlots[b - 1];
    e = launch_interpret_wide(h->runs_d, p, h->interp_tasks_w, h->interp_tasks, lo, b, counts[b], s);
  }
  if (e == hipSuccess && h->slots > kListSlots[kLists - 2])
    e = launch_interpret(h->runs_d, p, h->interp_tasks, kListSlots[kLists - 2], std::min(h->slots, kMaxLdsSlots),
                         kLists - 1, counts[kLists - 1], s);
  if (e == hipSuccess && h->slots > kMaxLdsSlots)
    e = launch_interpret_spill(h->runs_d, p, (double*)(h->ws + h->plan.spill), h->slots, s);
  return e;
}

// Algorithm 1 before the loop.  ev (nullable) receives four events: start,
// after the genomes, after the semantics (compile + interpret), and after
// the initial fitness and first draws.
gsgp_status eval_impl(gsgp_handle* h, const int32_t* h_codes, const double* h_consts, hipEvent_t* ev) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if ((h_codes == nullptr) != (h_consts == nullptr)) return fail(GSGP_ERR_ARG, "give both codes and constants, or neither");
  const Params& p = h->params;
  const int64_t per = (int64_t)(p.m + p.r) * p.k;
  if (h_codes) {
    for (int32_t r = 0; r < h->n_runs; ++r) {
      const int32_t l = h->runs_h[r].l;
      for (int64_t q = 0; q < per; ++q) {
        const int32_t c = h_codes[r * per + q];
        if (c < -5 || c >= l) return fail(GSGP_ERR_ARG, "run %d gene %lld: code %d out of [-5, %d)", r, (long long)q, c, l);
        if (!std::isfinite(h_consts[r * per + q])) return fail(GSGP_ERR_ARG, "run %d gene %lld: constant not finite", r, (long long)q);
      }
    }
  }
  if (ev) HIPCHK(h, hipEventRecord(ev[0], h->stream));
  for (int32_t w : {kStGen, kStDone, kStReplaySelect, kStReplayElite, kStMaxDepth})
    HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, w, 0, h->stream));
  for (int32_t b = 0; b < kLists; ++b) HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStList0 + b, 0, h->stream));
  if (h_codes) {
    for (int32_t r = 0; r < h->n_runs; ++r) {
      HIPCHK(h, hipMemcpyAsync(h->runs_h[r].code, h_codes + r * per, 4 * per, hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, hipMemcpyAsync(h->runs_h[r].cval, h_consts + r * per, 8 * per, hipMemcpyHostToDevice, h->stream));
    }
  } else {
    HIPCHK(h, launch_genome(h->runs_d, p, h->stream));
  }
  if (ev) HIPCHK(h, hipEventRecord(ev[1], h->stream));
  HIPCHK(h, launch_compile(h->runs_d, p, h->stream));
  int32_t* state = (int32_t*)(h->ws + h->plan.state);
  HIPCHK(h, hipMemcpyAsync(h->pinned, state, sizeof(int32_t) * kStWords * h->n_runs, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int32_t deepest = 0, counts[kLists] = {0, 0, 0, 0, 0};
  for (int32_t r = 0; r < h->n_runs; ++r) {
    deepest = std::max(deepest, h->pinned[kStWords * r + kStMaxDepth]);
    for (int32_t b = 0; b < kLists; ++b) counts[b] = std::max(counts[b], h->pinned[kStWords * r + kStList0 + b]);
  }
  h->slots = std::max(1, deepest - 2);  // the top two values live in registers
  // the deepest stack up to a genome's last valid function is at most k - 1
  // values, which sized the spill stacks; anything else is a broken invariant
  if ((int64_t)h->slots > std::max<int64_t>(1, max_need(p.k))) {
    h->poisoned = true;
    return fail(GSGP_ERR_STATE, "compiled stack depth %d exceeds the bound for genomes of %d genes", deepest, p.k);
  }
  HIPCHK(h, interpret_all(h, counts, h->stream));

  if (ev) HIPCHK(h, hipEventRecord(ev[2], h->stream));
  if (p.ls) HIPCHK(h, launch_target_sums(h->runs_d, p, h->stream));  // and generation 0's scaling
  HIPCHK(h, launch_vary(h->runs_d, p, h->rows, true, h->stream));
  HIPCHK(h, launch_fitness(h->runs_d, p, true, h->stream));
  HIPCHK(h, launch_survive(h->runs_d, p, h->surv_blocks, kSurvInit, h->stream));
  if (ev) HIPCHK(h, hipEventRecord(ev[3], h->stream));
  h->gen = 0;
  h->evaluated = true;
  return GSGP_OK;
}

}  // namespace

static gsgp_status eval_population_body(gsgp_handle* h, const int32_t* h_codes, const double* h_consts) {
  return eval_impl(h, h_codes, h_consts, nullptr);
}

static gsgp_status time_eval_body(gsgp_handle* h, double* h_ms) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h_ms) return fail(GSGP_ERR_ARG, "h_ms is NULL");
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  for (auto& e : ev) {
    hipError_t x = hipEventCreate(&e);
    if (x != hipSuccess) {
      for (auto& f : ev)
        if (f) (void)hipEventDestroy(f);
      return hip_fail(h, x, "hipEventCreate");
    }
  }
  st = eval_impl(h, nullptr, nullptr, ev);
  if (st == GSGP_OK) {
    hipError_t x = hipEventSynchronize(ev[3]);
    float a = 0, b = 0, c = 0, d = 0;
    if (x == hipSuccess) x = hipEventElapsedTime(&a, ev[0], ev[1]);
    if (x == hipSuccess) x = hipEventElapsedTime(&b, ev[1], ev[2]);
    if (x == hipSuccess) x = hipEventElapsedTime(&c, ev[2], ev[3]);
    if (x == hipSuccess) x = hipEventElapsedTime(&d, ev[0], ev[3]);
    if (x != hipSuccess) {
      st = hip_fail(h, x, "timing the initialisation");
    } else {
      h_ms[0] = a;
      h_ms[1] = b;
      h_ms[2] = c;
      h_ms[3] = d;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return st;
}

static gsgp_status generation_body(gsgp_handle* h, int32_t n_gens, gsgp_gen_stats* h_stats) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  if (n_gens < 1) return fail(GSGP_ERR_ARG, "n_gens must be >= 1");
  if ((int64_t)h->gen + n_gens > h->cfg.n_generations_max)
    return fail(GSGP_ERR_ARG, "generation %d + %d exceeds n_generations_max %d", h->gen, n_gens, h->cfg.n_generations_max);
  const int32_t g0 = h->gen;
  st = run_generations(h, n_gens);
  if (st != GSGP_OK) return st;
  if (h_stats) return copy_stats(h, g0 + 1, n_gens, h_stats, n_gens);
  return GSGP_OK;
}

static gsgp_status generation_replay_body(gsgp_handle* h, int32_t n_gens, const gsgp_record* h_records,
                                          const gsgp_gen_stats* h_elite, gsgp_gen_stats* h_stats) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  if (n_gens < 1 || !h_records) return fail(GSGP_ERR_ARG, "need n_gens >= 1 and records");
  if ((int64_t)h->gen + n_gens > h->cfg.n_generations_max)
    return fail(GSGP_ERR_ARG, "generation %d + %d exceeds n_generations_max %d", h->gen, n_gens, h->cfg.n_generations_max);
  const int32_t m = h->cfg.pop_size, r = h->cfg.pool_size;
  for (int64_t q = 0; q < (int64_t)h->n_runs * n_gens * m; ++q) {
    const gsgp_record& d = h_records[q];
    const bool ok = (d.op == 0 && d.p1 >= 0 && d.p1 < m && d.r1 >= 0 && d.r1 < r && d.r2 >= 0 && d.r2 < r &&
                     std::isfinite(d.ms)) ||
                    (d.op == 1 && d.p1 >= 0 && d.p1 < m && d.p2 >= 0 && d.p2 < m && d.r1 >= 0 && d.r1 < r);
    if (!ok) return fail(GSGP_ERR_ARG, "record %lld is not a valid mutation or crossover", (long long)q);
  }
  if (h_elite) {
    for (int64_t q = 0; q < (int64_t)h->n_runs * n_gens; ++q) {
      const gsgp_gen_stats& e = h_elite[q];
      if (e.elite_copied != 0 && e.elite_copied != 1) return fail(GSGP_ERR_ARG, "elite decision %lld: elite_copied must be 0/1", (long long)q);
      if (e.elite_copied && (e.elite_src < 0 || e.elite_src >= m || e.elite_dst < 0 || e.elite_dst >= m))
        return fail(GSGP_ERR_ARG, "elite decision %lld: index out of range", (long long)q);
    }
  }
  const int32_t g0 = h->gen;
  for (int32_t run = 0; run < h->n_runs; ++run) {
    HIPCHK(h, hipMemcpyAsync(h->runs_h[run].rec + (int64_t)g0 * m, h_records + (int64_t)run * n_gens * m,
                             sizeof(gsgp_record) * n_gens * m, hipMemcpyHostToDevice, h->stream));
    if (h_elite)
      HIPCHK(h, hipMemcpyAsync(h->runs_h[run].elite_in + g0, h_elite + (int64_t)run * n_gens,
                               sizeof(gsgp_gen_stats) * n_gens, hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStReplaySelect, 1, h->stream));
  HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStReplayElite, h_elite ? 1 : 0, h->stream));
  st = run_generations(h, n_gens);
  if (st != GSGP_OK) return st;
  HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStReplaySelect, 0, h->stream));
  HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStReplayElite, 0, h->stream));
  HIPCHK(h, launch_survive(h->runs_d, h->params, h->surv_blocks, kSurvSelectOnly, h->stream));
  if (h_stats) return copy_stats(h, g0 + 1, n_gens, h_stats, n_gens);
  return GSGP_OK;
}

gsgp_status gsgp_current_generation(gsgp_handle* h, int32_t* gen) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!gen) return fail(GSGP_ERR_ARG, "gen is NULL");
  *gen = h->gen;
  return GSGP_OK;
}

gsgp_status gsgp_get_fitness(gsgp_handle* h, int32_t run, double* h_train, double* h_test) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const RunDev& R = h->runs_h[run];
  const int cur = h->gen & 1;
  if (h_train) HIPCHK(h, hipMemcpy(h_train, R.F[cur], 8 * h->cfg.pop_size, hipMemcpyDeviceToHost));
  if (h_test) HIPCHK(h, hipMemcpy(h_test, R.Ft[cur], 8 * h->cfg.pop_size, hipMemcpyDeviceToHost));
  return GSGP_OK;
}

gsgp_status gsgp_get_semantics_rows(gsgp_handle* h, int32_t run, int32_t which, int32_t row0, int32_t n_rows,
                                    double* h_out) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (which != 0 && which != 1) return fail(GSGP_ERR_ARG, "which must be 0 (population) or 1 (pool)");
  if (!h_out) return fail(GSGP_ERR_ARG, "h_out is NULL");
  const int64_t rows = which == 0 ? h->cfg.pop_size : h->cfg.pool_size;
  if (row0 < 0 || n_rows < 1 || (int64_t)row0 + n_rows > rows)
    return fail(GSGP_ERR_ARG, "rows %d..%d not in [0, %lld)", row0, row0 + n_rows - 1, (long long)rows);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const RunDev& R = h->runs_h[run];
  const size_t s = storage_bytes(h->cfg.precision);
  const int64_t CH = chunk_cases((int)s);
  // gather the rows' part of every chunk block into a tiled buffer of n_rows rows
  std::vector<char> raw((size_t)n_rows * R.ld * s);
  const char* from = (const char*)(which == 0 ? R.S[h->gen & 1] : R.sigR);
  for (int32_t c = 0; c < R.nch; ++c) {
    const ChunkGeom g = chunk_geom(R.tr_pad, R.te_pad, R.nch_tr, c, CH);
    HIPCHK(h, hipMemcpy(raw.data() + (size_t)n_rows * g.cs * s, from + (size_t)(rows * g.cs + row0 * g.len) * s,
                        (size_t)n_rows * g.len * s, hipMemcpyDeviceToHost));
  }
  if (s == 8)
    to_f64<double>(raw, n_rows, R, h_out);
  else
    to_f64<float>(raw, n_rows, R, h_out);
  if (which == 0) return apply_scaling(h, run, row0, n_rows, R.n_train + R.n_test, h_out);
  return GSGP_OK;
}

gsgp_status gsgp_get_semantics_cases(gsgp_handle* h, int32_t run, int32_t which, int64_t case0, int64_t n_cases,
                                     double* h_out) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (which != 0 && which != 1) return fail(GSGP_ERR_ARG, "which must be 0 (population) or 1 (pool)");
  if (!h_out) return fail(GSGP_ERR_ARG, "h_out is NULL");
  const RunDev& R = h->runs_h[run];
  const int64_t n_all = R.n_train + R.n_test;
  if (case0 < 0 || n_cases < 1 || case0 + n_cases > n_all)
    return fail(GSGP_ERR_ARG, "cases %lld..%lld not in [0, %lld)", (long long)case0, (long long)(case0 + n_cases - 1),
                (long long)n_all);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int64_t rows = which == 0 ? h->cfg.pop_size : h->cfg.pool_size;
  const size_t s = storage_bytes(h->cfg.precision);
  const int64_t CH = chunk_cases((int)s);
  const char* from = (const char*)(which == 0 ? R.S[h->gen & 1] : R.sigR);
  // the requested cases as padded-column ranges: train part, then test part
  struct Piece {
    int64_t col0, col1, out0;
  };
  Piece pieces[2];
  int np = 0;
  const int64_t c1 = case0 + n_cases;
  if (case0 < R.n_train) pieces[np++] = Piece{case0, std::min(c1, R.n_train), 0};
  if (c1 > R.n_train) {
    const int64_t t0 = std::max(case0, R.n_train) - R.n_train, t1 = c1 - R.n_train;
    pieces[np++] = Piece{R.tr_pad + t0, R.tr_pad + t1, std::max(case0, R.n_train) - case0};
  }
  std::vector<char> buf;
  for (int q = 0; q < np; ++q) {
    const Piece& pc = pieces[q];
    const int32_t first = pc.col0 < R.tr_pad ? (int32_t)(pc.col0 / CH) : R.nch_tr + (int32_t)((pc.col0 - R.tr_pad) / CH);
    for (int32_t c = first; c < R.nch; ++c) {
      const ChunkGeom g = chunk_geom(R.tr_pad, R.te_pad, R.nch_tr, c, CH);
      const int64_t lo = std::max(pc.col0, g.cs), hi = std::min(pc.col1, g.cs + g.len);
      if (g.cs >= pc.col1) break;
      if (lo >= hi) continue;
      // rows x (hi - lo) sub-block of the chunk block: row i at rows * cs + i * len + (lo - cs)
      const int64_t w = hi - lo;
      buf.resize((size_t)rows * w * s);
      HIPCHK(h, hipMemcpy2D(buf.data(), (size_t)w * s, from + (size_t)(rows * g.cs + (lo - g.cs)) * s, (size_t)g.len * s,
                            (size_t)w * s, (size_t)rows, hipMemcpyDeviceToHost));
      const int64_t o = pc.out0 + (lo - pc.col0);
      for (int64_t i = 0; i < rows; ++i) {
        double* dst = h_out + i * n_cases + o;
        if (s == 8) {
          const double* src = (const double*)buf.data() + i * w;
          for (int64_t k = 0; k < w; ++k) dst[k] = src[k];
        } else {
          const float* src = (const float*)buf.data() + i * w;
          for (int64_t k = 0; k < w; ++k) dst[k] = (double)src[k];
        }
      }
    }
  }
  if (which == 0) return apply_scaling(h, run, 0, (int32_t)rows, n_cases, h_out);
  return GSGP_OK;
}

gsgp_status gsgp_get_semantics(gsgp_handle* h, int32_t run, int32_t which, double* h_out) {
  if (which != 0 && which != 1) return fail(GSGP_ERR_ARG, "which must be 0 (population) or 1 (pool)");
  return gsgp_get_semantics_rows(h, run, which, 0, which == 0 ? h->cfg.pop_size : h->cfg.pool_size, h_out);
}

gsgp_status gsgp_get_records(gsgp_handle* h, int32_t run, int32_t gen0, int32_t n_gens, int32_t raw,
                             gsgp_record* h_out) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (!h_out || n_gens < 1 || gen0 < 1 || (int64_t)gen0 + n_gens - 1 > h->gen)
    return fail(GSGP_ERR_ARG, "records of generations %d..%d are not available (current %d)", gen0, gen0 + n_gens - 1, h->gen);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int32_t m = h->cfg.pop_size;
  const RunDev& R = h->runs_h[run];
  HIPCHK(h, hipMemcpy(h_out, R.rec + (int64_t)(gen0 - 1) * m, sizeof(gsgp_record) * n_gens * m, hipMemcpyDeviceToHost));
  if (!raw) {
    std::vector<gsgp_gen_stats> s(n_gens);
    HIPCHK(h, hipMemcpy(s.data(), R.stats + gen0, sizeof(gsgp_gen_stats) * n_gens, hipMemcpyDeviceToHost));
    for (int32_t g = 0; g < n_gens; ++g) {
      if (!s[g].elite_copied) continue;
      gsgp_record& d = h_out[(int64_t)g * m + s[g].elite_dst];
      d = gsgp_record{2, s[g].elite_src, -1, -1, -1, 0, 0.0};
    }
  }
  return GSGP_OK;
}

gsgp_status gsgp_get_stats(gsgp_handle* h, int32_t run, int32_t gen0, int32_t n_gens, gsgp_gen_stats* h_out) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (!h_out || n_gens < 1 || gen0 < 0 || (int64_t)gen0 + n_gens - 1 > h->gen)
    return fail(GSGP_ERR_ARG, "summaries of generations %d..%d are not available (current %d)", gen0, gen0 + n_gens - 1, h->gen);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(h_out, h->runs_h[run].stats + gen0, sizeof(gsgp_gen_stats) * n_gens, hipMemcpyDeviceToHost));
  return GSGP_OK;
}

gsgp_status gsgp_get_scaling(gsgp_handle* h, int32_t run, int32_t gen0, int32_t n_gens, double* h_out) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (!h_out || n_gens < 1 || gen0 < 0 || (int64_t)gen0 + n_gens - 1 > h->gen)
    return fail(GSGP_ERR_ARG, "scaling of generations %d..%d is not available (current %d)", gen0, gen0 + n_gens - 1, h->gen);
  const int64_t m = h->cfg.pop_size;
  if (!(h->cfg.flags & GSGP_FLAG_LOCAL_SEARCH)) {
    for (int64_t q = 0; q < (int64_t)n_gens * m; ++q) {
      h_out[2 * q] = 0.0;
      h_out[2 * q + 1] = 1.0;
    }
    return GSGP_OK;
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(h_out, h->runs_h[run].ls + (int64_t)gen0 * m * 2, sizeof(double) * 2 * m * n_gens,
                      hipMemcpyDeviceToHost));
  return GSGP_OK;
}

gsgp_status gsgp_get_genomes(gsgp_handle* h, int32_t run, int32_t* h_codes, double* h_consts) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int64_t per = (int64_t)(h->cfg.pop_size + h->cfg.pool_size) * h->cfg.genome_len;
  if (h_codes) HIPCHK(h, hipMemcpy(h_codes, h->runs_h[run].code, 4 * per, hipMemcpyDeviceToHost));
  if (h_consts) HIPCHK(h, hipMemcpy(h_consts, h->runs_h[run].cval, 8 * per, hipMemcpyDeviceToHost));
  return GSGP_OK;
}

static gsgp_status time_stages_body(gsgp_handle* h, int32_t n_gens, double* h_ms) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  if (!h_ms || n_gens < 1) return fail(GSGP_ERR_ARG, "need n_gens >= 1 and an output array");
  if ((int64_t)h->gen + n_gens > h->cfg.n_generations_max)
    return fail(GSGP_ERR_ARG, "generation %d + %d exceeds n_generations_max %d", h->gen, n_gens, h->cfg.n_generations_max);
  std::vector<hipEvent_t> ev((size_t)4 * n_gens, nullptr);
  gsgp_status result = GSGP_OK;
  for (auto& e : ev) {
    hipError_t x = hipEventCreate(&e);
    if (x != hipSuccess) {
      result = hip_fail(h, x, "hipEventCreate");
      break;
    }
  }
  double acc[4] = {0, 0, 0, 0};
  if (result == GSGP_OK) {
    for (int32_t g = 0; g < n_gens && result == GSGP_OK; ++g) {
      hipEvent_t* e = &ev[(size_t)4 * g];
      hipError_t x = hipEventRecord(e[0], h->stream);
      if (x == hipSuccess) x = launch_vary(h->runs_d, h->params, h->vary, false, h->stream);
      if (x == hipSuccess) x = hipEventRecord(e[1], h->stream);
      if (x == hipSuccess) x = launch_fitness(h->runs_d, h->params, false, h->stream);
      if (x == hipSuccess) x = hipEventRecord(e[2], h->stream);
      if (x == hipSuccess) x = launch_survive(h->runs_d, h->params, h->surv_blocks, kSurvGen, h->stream);
      if (x == hipSuccess) x = hipEventRecord(e[3], h->stream);
      if (x != hipSuccess) result = hip_fail(h, x, "timed generation");
    }
    if (result == GSGP_OK) {
      h->gen += n_gens;
      hipError_t x = hipStreamSynchronize(h->stream);
      if (x != hipSuccess) result = hip_fail(h, x, "hipStreamSynchronize");
    }
    for (int32_t g = 0; g < n_gens && result == GSGP_OK; ++g) {
      hipEvent_t* e = &ev[(size_t)4 * g];
      float a = 0, b = 0, c = 0, d = 0;
      hipError_t x = hipEventElapsedTime(&a, e[0], e[1]);
      if (x == hipSuccess) x = hipEventElapsedTime(&b, e[1], e[2]);
      if (x == hipSuccess) x = hipEventElapsedTime(&c, e[2], e[3]);
      if (x == hipSuccess) x = hipEventElapsedTime(&d, e[0], e[3]);
      if (x != hipSuccess) {
        result = hip_fail(h, x, "hipEventElapsedTime");
        break;
      }
      acc[0] += c;
      acc[1] += a;
      acc[2] += b;
      acc[3] += d;
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (result == GSGP_OK)
    for (int i = 0; i < 4; ++i) h_ms[i] = acc[i] / n_gens;
  return result;
}

gsgp_status gsgp_set_launch(gsgp_handle* h, int32_t waves_per_block, int32_t offspring_per_block, int32_t xcd_remap,
                            int32_t max_blocks) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  const int32_t w = waves_per_block ? waves_per_block : h->vary.waves;
  const int32_t o = offspring_per_block ? offspring_per_block : h->vary.opb;
  if (w < 1 || w > 8) return fail(GSGP_ERR_ARG, "waves_per_block must be in [1, 8]");
  if (o < 1 || o > 4096) return fail(GSGP_ERR_ARG, "offspring_per_block must be in [1, 4096]");
  if (xcd_remap < 0 || xcd_remap > 2) return fail(GSGP_ERR_ARG, "xcd_remap must be 0, 1 or 2");
  if (max_blocks < 0) return fail(GSGP_ERR_ARG, "max_blocks must be >= 0");
  plan_vary(h, w, o, xcd_remap, max_blocks);
  plan_rows(h);
  HIPCHK(h, upload_runs(h));
  drop_graph(h);
  return GSGP_OK;
}

static gsgp_status autotune_body(gsgp_handle* h, int32_t* h_best) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  // the trial launches read the next generation's records
  if (h->gen >= h->cfg.n_generations_max)
    return fail(GSGP_ERR_STATE, "no generation left to time (%d of %d done)", h->gen, h->cfg.n_generations_max);
  // The variation kernel is idempotent for a fixed generation (it reads the
  // parents and writes the offspring buffer), so shapes can be timed on the
  // live buffers without advancing the run.
  const VaryLaunch keep = h->vary;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  float best_ms = 1e30f;
  int32_t best[4] = {keep.waves, keep.opb, keep.remap, h->max_blocks};
  const int32_t wave_opts[] = {2, 4, 8};
  const int32_t opb_mult[] = {1, 2, 4, 8};
  const int32_t grid_opts[] = {0, 1024, 2048, 4096};
  gsgp_status result = GSGP_OK;
  for (int32_t w : wave_opts) {
    for (int32_t mult : opb_mult) {
      for (int32_t trial = 0; trial < 12 && result == GSGP_OK; ++trial) {
        const int32_t remap = trial % 3;
        const int32_t cap = grid_opts[trial / 3];
        plan_vary(h, w, w * mult, remap, cap);
        hipError_t x = upload_runs(h);
        for (int rep = 0; rep < 2 && x == hipSuccess; ++rep) x = launch_vary(h->runs_d, h->params, h->vary, false, h->stream);
        if (x == hipSuccess) x = hipEventRecord(e0, h->stream);
        for (int rep = 0; rep < 5 && x == hipSuccess; ++rep) x = launch_vary(h->runs_d, h->params, h->vary, false, h->stream);
        if (x == hipSuccess) x = hipEventRecord(e1, h->stream);
        if (x == hipSuccess) x = hipEventSynchronize(e1);
        float ms = 0;
        if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
        if (x != hipSuccess) {
          result = hip_fail(h, x, "autotune trial");
          break;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best[0] = w;
          best[1] = w * mult;
          best[2] = remap;
          best[3] = cap;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result != GSGP_OK) return result;
  plan_vary(h, best[0], best[1], best[2], best[3]);
  plan_rows(h);
  HIPCHK(h, upload_runs(h));
  drop_graph(h);
  if (h_best) memcpy(h_best, best, sizeof best);
  return GSGP_OK;
}

// ---------------------------------------------------------------------------
// Lineage reconstruction.
namespace {

struct Lineage {
  std::vector<std::vector<int32_t>> need;  // need[g]: individuals of generation g, sorted
  std::vector<int32_t> pool;               // pool trees used, sorted
  std::vector<gsgp_record> rec;            // [gen][m]
  std::vector<gsgp_gen_stats> stats;       // [gen + 1]
  std::vector<double> ls;                  // local search: [gen + 1][m][2] scaling, else empty
  size_t max_slots = 1, total_nodes = 0;
  int64_t ld = 0;
  size_t off_X = 0, off_pool = 0, off_A = 0, off_B = 0, off_prog = 0, off_nodes = 0, off_spill = 0, total = 0;
};

gsgp_status walk_lineage(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, int64_t n, Lineage* L) {
  const int32_t m = h->cfg.pop_size;
  const RunDev& R = h->runs_h[run];
  HIPCHK(h, hipStreamSynchronize(h->stream));
  L->rec.resize((size_t)gen * m);
  L->stats.resize((size_t)gen + 1);
  if (gen > 0) {
    HIPCHK(h, hipMemcpy(L->rec.data(), R.rec, sizeof(gsgp_record) * gen * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(L->stats.data(), R.stats, sizeof(gsgp_gen_stats) * (gen + 1), hipMemcpyDeviceToHost));
    if (h->cfg.flags & GSGP_FLAG_LOCAL_SEARCH) {
      L->ls.resize((size_t)(gen + 1) * m * 2);
      HIPCHK(h, hipMemcpy(L->ls.data(), R.ls, sizeof(double) * L->ls.size(), hipMemcpyDeviceToHost));
    }
  }
  std::vector<std::set<int32_t>> need(gen + 1);
  std::set<int32_t> pool;
  need[gen].insert(individual);
  for (int32_t g = gen; g >= 1; --g) {
    const gsgp_gen_stats& s = L->stats[g];
    for (int32_t i : need[g]) {
      if (s.elite_copied && i == s.elite_dst) {
        need[g - 1].insert(s.elite_src);
        continue;
      }
      const gsgp_record& d = L->rec[(size_t)(g - 1) * m + i];
      need[g - 1].insert(d.p1);
      pool.insert(d.r1);
      if (d.op == 1)
        need[g - 1].insert(d.p2);
      else
        pool.insert(d.r2);
    }
  }
  L->need.resize(gen + 1);
  L->max_slots = 1;
  L->total_nodes = 0;
  for (int32_t g = 0; g <= gen; ++g) {
    L->need[g].assign(need[g].begin(), need[g].end());
    L->max_slots = std::max(L->max_slots, L->need[g].size());
    if (g > 0) L->total_nodes += L->need[g].size();
  }
  L->pool.assign(pool.begin(), pool.end());
  L->ld = pad_to(n, kSegPad);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L->off_X = take(sizeof(double) * R.l * L->ld);
  L->off_pool = take(sizeof(double) * std::max<size_t>(1, L->pool.size()) * L->ld);
  L->off_A = take(sizeof(double) * L->max_slots * L->ld);
  L->off_B = take(sizeof(double) * L->max_slots * L->ld);
  L->off_prog = take(sizeof(int32_t) * 2 * (L->need[0].size() + L->pool.size() + 2));
  L->off_nodes = take(sizeof(ReplayNode) * std::max<size_t>(1, L->total_nodes));
  // stack columns for programs deeper than an LDS column (spill interpreter)
  L->off_spill = take(h->slots > kMaxLdsSlots ? sizeof(double) * kSpillWaves * h->slots * 2 * kWave : 0);
  L->total = off;
  return GSGP_OK;
}

}  // namespace

gsgp_status gsgp_reconstruct_scratch_size(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, int64_t n,
                                          size_t* bytes) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (!bytes) return fail(GSGP_ERR_ARG, "bytes is NULL");
  if (gen < 0 || gen > h->gen) return fail(GSGP_ERR_ARG, "generation %d not in [0, %d]", gen, h->gen);
  if (individual < 0 || individual >= h->cfg.pop_size) return fail(GSGP_ERR_ARG, "individual out of range");
  if (n < 1 || n > ((int64_t)1 << 40)) return fail(GSGP_ERR_ARG, "n must be >= 1");
  Lineage L;
  st = walk_lineage(h, run, gen, individual, n, &L);
  if (st != GSGP_OK) return st;
  *bytes = L.total;
  return GSGP_OK;
}

gsgp_status gsgp_export_linear(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, int32_t* h_tree,
                               double* h_affine, double* h_weights) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (gen < 0 || gen > h->gen) return fail(GSGP_ERR_ARG, "generation %d not in [0, %d]", gen, h->gen);
  if (individual < 0 || individual >= h->cfg.pop_size) return fail(GSGP_ERR_ARG, "individual out of range");
  if (!h_tree || !h_affine || !h_weights) return fail(GSGP_ERR_ARG, "NULL output pointer");
  const int32_t m = h->cfg.pop_size, r = h->cfg.pool_size;
  const bool scaled = (h->cfg.flags & GSGP_FLAG_LOCAL_SEARCH) != 0;
  const RunDev& R = h->runs_h[run];
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::vector<gsgp_record> rec((size_t)gen * m);
  std::vector<gsgp_gen_stats> stats((size_t)gen + 1);
  std::vector<double> ls;
  if (gen > 0) {
    HIPCHK(h, hipMemcpy(rec.data(), R.rec, sizeof(gsgp_record) * gen * m, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(stats.data(), R.stats, sizeof(gsgp_gen_stats) * (gen + 1), hipMemcpyDeviceToHost));
    if (scaled) {
      ls.resize((size_t)(gen + 1) * m * 2);
      HIPCHK(h, hipMemcpy(ls.data(), R.ls, sizeof(double) * ls.size(), hipMemcpyDeviceToHost));
    }
  }
  // walk back to the generation-0 tree, keeping the mutations in order with
  // the generation and index of the offspring each one made
  struct Step {
    const gsgp_record* d;
    int32_t g, i;
  };
  std::vector<Step> steps;
  int32_t i = individual;
  for (int32_t g = gen; g >= 1; --g) {
    const gsgp_gen_stats& s = stats[g];
    if (s.elite_copied && i == s.elite_dst) {
      i = s.elite_src;
      continue;
    }
    const gsgp_record& d = rec[(size_t)(g - 1) * m + i];
    if (d.op == 1) return fail(GSGP_ERR_UNSUPPORTED, "the lineage contains a crossover at generation %d", g);
    steps.push_back(Step{&d, g, i});
    i = d.p1;
  }
  // forward, generation by generation: with the step's scaling (alpha, beta)
  // (0 and 1 without local search), c = alpha + beta c, b = beta b,
  // w = beta w, then w[r1] += beta ms and w[r2] -= beta ms
  std::vector<double> w(r, 0.0);
  double c = 0.0, b = 1.0;
  for (auto it = steps.rbegin(); it != steps.rend(); ++it) {
    double alpha = 0.0, beta = 1.0;
    if (scaled) {
      alpha = ls[((size_t)it->g * m + it->i) * 2];
      beta = ls[((size_t)it->g * m + it->i) * 2 + 1];
    }
    c = alpha + beta * c;
    b = beta * b;
    for (double& x : w) x = beta * x;
    w[it->d->r1] += beta * it->d->ms;
    w[it->d->r2] -= beta * it->d->ms;
  }
  *h_tree = i;
  h_affine[0] = c;
  h_affine[1] = b;
  std::copy(w.begin(), w.end(), h_weights);
  return GSGP_OK;
}

}  // extern "C"

namespace {

gsgp_status check_reconstruct_args(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, const double* d_X,
                                   int64_t n, double* d_out) {
  gsgp_status st = check_run(h, run);
  if (st != GSGP_OK) return st;
  if (gen < 0 || gen > h->gen) return fail(GSGP_ERR_ARG, "generation %d not in [0, %d]", gen, h->gen);
  if (individual < 0 || individual >= h->cfg.pop_size) return fail(GSGP_ERR_ARG, "individual out of range");
  if (n < 1 || n > ((int64_t)1 << 40)) return fail(GSGP_ERR_ARG, "n must be >= 1");
  if (!d_X || !d_out) return fail(GSGP_ERR_ARG, "NULL data or output pointer");
  return GSGP_OK;
}

// Lineage reconstruction into `scratch_bytes` of device scratch at `sc`;
// `whose` names it in errors.
gsgp_status reconstruct_with(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, const double* d_X,
                             int64_t n, double* d_out, char* sc, size_t scratch_bytes, const char* whose) {
  Lineage L;
  gsgp_status st = walk_lineage(h, run, gen, individual, n, &L);
  if (st != GSGP_OK) return st;
  if (scratch_bytes < L.total)
    return fail(GSGP_ERR_WORKSPACE, "%s has %zu bytes, this reconstruction needs %zu", whose, scratch_bytes, L.total);
  const RunDev& R = h->runs_h[run];
  const int32_t m = h->cfg.pop_size;
  double* Xfm = (double*)(sc + L.off_X);
  double* pool = (double*)(sc + L.off_pool);
  double* bufA = (double*)(sc + L.off_A);
  double* bufB = (double*)(sc + L.off_B);
  int32_t* prog = (int32_t*)(sc + L.off_prog);
  ReplayNode* nodes = (ReplayNode*)(sc + L.off_nodes);
  double* spill = h->slots > kMaxLdsSlots ? (double*)(sc + L.off_spill) : nullptr;

  // host-side lists: generation-0 programs, pool programs, replay nodes
  const size_t n0 = L.need[0].size(), np = L.pool.size();
  std::vector<int32_t> lists(2 * (n0 + np + 2), 0);
  int32_t* prog0 = lists.data();
  int32_t* sq0 = prog0 + n0 + 1;
  int32_t* progp = sq0 + n0 + 1;
  int32_t* sqp = progp + np + 1;
  for (size_t j = 0; j < n0; ++j) prog0[j] = L.need[0][j];
  for (size_t j = 0; j < np; ++j) {
    progp[j] = m + L.pool[j];
    sqp[j] = 1;
  }
  std::map<int32_t, int32_t> pool_slot;
  for (size_t j = 0; j < np; ++j) pool_slot[L.pool[j]] = (int32_t)j;
  std::vector<ReplayNode> all_nodes;
  all_nodes.reserve(L.total_nodes);
  std::vector<size_t> node_begin(gen + 2, 0);
  for (int32_t g = 1; g <= gen; ++g) {
    node_begin[g] = all_nodes.size();
    std::map<int32_t, int32_t> prev_slot;
    for (size_t j = 0; j < L.need[g - 1].size(); ++j) prev_slot[L.need[g - 1][j]] = (int32_t)j;
    const gsgp_gen_stats& s = L.stats[g];
    for (size_t j = 0; j < L.need[g].size(); ++j) {
      const int32_t i = L.need[g][j];
      ReplayNode nd{};
      nd.out = (int32_t)j;
      nd.b = -1;
      nd.r1 = -1;
      nd.r2 = -1;
      nd.ms = 0.0;
      nd.alpha = 0.0;
      nd.beta = 1.0;
      if (s.elite_copied && i == s.elite_dst) {
        nd.op = 2;
        nd.a = prev_slot.at(s.elite_src);
      } else {
        const gsgp_record& d = L.rec[(size_t)(g - 1) * m + i];
        nd.op = d.op;
        nd.a = prev_slot.at(d.p1);
        nd.r1 = pool_slot.at(d.r1);
        if (d.op == 1) {
          nd.b = prev_slot.at(d.p2);
        } else {
          nd.r2 = pool_slot.at(d.r2);
          nd.ms = d.ms;
        }
        if (!L.ls.empty()) {
          nd.alpha = L.ls[((size_t)g * m + i) * 2];
          nd.beta = L.ls[((size_t)g * m + i) * 2 + 1];
        }
      }
      all_nodes.push_back(nd);
    }
  }
  node_begin[gen + 1] = all_nodes.size();
  HIPCHK(h, hipMemcpyAsync(prog, lists.data(), sizeof(int32_t) * lists.size(), hipMemcpyHostToDevice, h->stream));
  if (!all_nodes.empty())
    HIPCHK(h, hipMemcpyAsync(nodes, all_nodes.data(), sizeof(ReplayNode) * all_nodes.size(), hipMemcpyHostToDevice,
                             h->stream));
  const int32_t* d_prog0 = prog;
  const int32_t* d_sq0 = prog + n0 + 1;
  const int32_t* d_progp = d_sq0 + n0 + 1;
  const int32_t* d_sqp = d_progp + np + 1;
  HIPCHK(h, launch_transpose(d_X, n, R.l, Xfm, L.ld, h->stream));
  HIPCHK(h, launch_interpret_list(R.ops, R.opv, R.nops, h->cfg.genome_len, d_prog0, d_sq0, (int32_t)n0, Xfm, L.ld, n,
                                  bufA, h->slots, spill, h->stream));
  HIPCHK(h, launch_interpret_list(R.ops, R.opv, R.nops, h->cfg.genome_len, d_progp, d_sqp, (int32_t)np, Xfm, L.ld, n,
                                  pool, h->slots, spill, h->stream));
  double* cur = bufA;
  double* nxt = bufB;
  for (int32_t g = 1; g <= gen; ++g) {
    const size_t b = node_begin[g], e = node_begin[g + 1];
    HIPCHK(h, launch_replay_nodes(nodes + b, (int32_t)(e - b), cur, pool, nxt, L.ld, n, h->stream));
    std::swap(cur, nxt);
  }
  const auto& last = L.need[gen];
  const int32_t slot = (int32_t)(std::lower_bound(last.begin(), last.end(), individual) - last.begin());
  HIPCHK(h, hipMemcpyAsync(d_out, cur + (int64_t)slot * L.ld, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return GSGP_OK;
}

}  // namespace

extern "C" {

gsgp_status gsgp_reconstruct(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, const double* d_X,
                             int64_t n, double* d_out, void* d_scratch, size_t scratch_bytes) {
  gsgp_status st = check_reconstruct_args(h, run, gen, individual, d_X, n, d_out);
  if (st != GSGP_OK) return st;
  if (!d_scratch || ((uintptr_t)d_scratch) % kAlign) return fail(GSGP_ERR_WORKSPACE, "scratch must be non-NULL and 256-byte aligned");
  return reconstruct_with(h, run, gen, individual, d_X, n, d_out, (char*)d_scratch, scratch_bytes, "the scratch");
}

gsgp_status gsgp_reconstruct_static(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual, const double* d_X,
                                    int64_t n, double* d_out) {
  gsgp_status st = check_reconstruct_args(h, run, gen, individual, d_X, n, d_out);
  if (st != GSGP_OK) return st;
  if (h->device < 0 || h->device >= kMaxDevices || !g_static[h->device].ptr)
    return fail(GSGP_ERR_UNSUPPORTED, "no static scratch on device %d", h->device);
  std::lock_guard<std::mutex> lock(g_static[h->device].call);
  return reconstruct_with(h, run, gen, individual, d_X, n, d_out, g_static[h->device].ptr, kStaticScratchBytes,
                          "the static scratch");
}



// The entry points that launch kernels check the workspace guards
// (GSGP_FLAG_GUARDS) before returning.
gsgp_status gsgp_eval_population(gsgp_handle* h, const int32_t* h_codes, const double* h_consts) {
  return check_guards(h, eval_population_body(h, h_codes, h_consts));
}

gsgp_status gsgp_time_eval(gsgp_handle* h, double* h_ms) { return check_guards(h, time_eval_body(h, h_ms)); }

gsgp_status gsgp_generation(gsgp_handle* h, int32_t n_gens, gsgp_gen_stats* h_stats) {
  return check_guards(h, generation_body(h, n_gens, h_stats));
}

gsgp_status gsgp_generation_replay(gsgp_handle* h, int32_t n_gens, const gsgp_record* h_records,
                                   const gsgp_gen_stats* h_elite, gsgp_gen_stats* h_stats) {
  return check_guards(h, generation_replay_body(h, n_gens, h_records, h_elite, h_stats));
}

gsgp_status gsgp_time_stages(gsgp_handle* h, int32_t n_gens, double* h_ms) {
  return check_guards(h, time_stages_body(h, n_gens, h_ms));
}

gsgp_status gsgp_autotune(gsgp_handle* h, int32_t* h_best) { return check_guards(h, autotune_body(h, h_best)); }

// ---- checkpoint / resume ---------------------------------------------------
// A checkpoint holds, per run, the current population semantics and fitness,
// the squashed pool, the genomes and their compiled form, the ancestry record
// (draws of generations 1 .. gen + 1, summaries 0 .. gen) and the state
// words; every later draw is a function of (seed, run, offspring, generation)
// and the fitness, so a loaded handle continues bit for bit.
}  // extern "C"

namespace {

constexpr uint64_t kCkptMagic = 0x5450434B50475347ull;  // "GSGPCKPT"

// Everything that decides a run's draws and values is in the header and
// must match the loading handle: sizes, precision, seed and every operator
// setting (tournament, crossover probability, step and its randomness, gene
// probabilities, constant range, the flags that change results).
struct CkptHeader {
  uint64_t magic;
  int32_t version, n_runs, m, r, k, G, precision, gen, slots, tsize, ms_random, pad;
  uint32_t seed, result_flags;
  double p_crossover, mutation_step, p_function, p_feature, erc_lo, erc_hi;
};
constexpr int32_t kCkptVersion = 6;  // 5: genomes recompiled on load; 6: twelve state words per run
static_assert(sizeof(CkptHeader) == 112, "no padding between header fields");

struct CkptPiece {
  size_t off;    // workspace offset
  size_t bytes;
};

std::vector<CkptPiece> ckpt_pieces(const gsgp_handle* h) {
  std::vector<CkptPiece> out;
  const int64_t m = h->cfg.pop_size, r = h->cfg.pool_size, k = h->cfg.genome_len;
  const int64_t G = h->cfg.n_generations_max;
  const size_t s = storage_bytes(h->cfg.precision);
  const int cur = h->gen & 1;
  const int64_t n_rec = std::min<int64_t>(h->gen + 1, G);
  out.push_back({h->plan.state, sizeof(int32_t) * kStWords * h->n_runs});
  for (int32_t i = 0; i < h->n_runs; ++i) {
    const RunPlan& q = h->plan.runs[i];
    out.push_back({cur ? q.S1 : q.S0, s * m * q.ld});
    out.push_back({q.sigR, s * r * q.ld});
    out.push_back({cur ? q.F1 : q.F0, 8 * (size_t)m});
    out.push_back({cur ? q.Ft1 : q.Ft0, 8 * (size_t)m});
    out.push_back({q.rec, sizeof(gsgp_record) * (size_t)(n_rec * m)});
    out.push_back({q.stats, sizeof(gsgp_gen_stats) * (size_t)(h->gen + 1)});
    // the genomes; their compiled form holds addresses in this workspace
    // and is rebuilt by the loading handle
    out.push_back({q.code, 4 * (size_t)((m + r) * k)});
    out.push_back({q.cval, 8 * (size_t)((m + r) * k)});
    if (h->cfg.flags & GSGP_FLAG_LOCAL_SEARCH) {
      out.push_back({q.ls, sizeof(double) * 2 * (size_t)(m * (h->gen + 1))});
      out.push_back({q.tsum, sizeof(double) * 4});
    }
  }
  return out;
}

CkptHeader ckpt_header(const gsgp_handle* h) {
  CkptHeader c;
  std::memset(&c, 0, sizeof c);  // padding included: headers compare bytewise
  c.magic = kCkptMagic;
  c.version = kCkptVersion;
  c.n_runs = h->n_runs;
  c.m = h->cfg.pop_size;
  c.r = h->cfg.pool_size;
  c.k = h->cfg.genome_len;
  c.G = h->cfg.n_generations_max;
  c.precision = h->cfg.precision;
  c.gen = h->gen;
  c.slots = h->slots;
  c.tsize = h->cfg.tournament_size;
  c.ms_random = h->cfg.ms_random;
  c.seed = h->cfg.seed;
  c.result_flags = h->cfg.flags & kResultFlags;
  c.p_crossover = h->cfg.p_crossover;
  c.mutation_step = h->cfg.mutation_step;
  c.p_function = h->cfg.p_function;
  c.p_feature = h->cfg.p_feature;
  c.erc_lo = h->cfg.erc_lo;
  c.erc_hi = h->cfg.erc_hi;
  return c;
}

// The run-defining part of two headers is equal (the generation and the
// compiled stack depth are the saved state, not configuration).
bool same_configuration(CkptHeader a, CkptHeader b) {
  a.gen = b.gen;
  a.slots = b.slots;
  return std::memcmp(&a, &b, sizeof a) == 0;
}

size_t ckpt_bytes(const gsgp_handle* h, const std::vector<CkptPiece>& pieces) {
  size_t total = sizeof(CkptHeader) + sizeof(int64_t) * 2 * h->n_runs;  // header, per-run (ld, l)
  for (const CkptPiece& p : pieces) total += p.bytes;
  return total;
}

}  // namespace

extern "C" {

gsgp_status gsgp_checkpoint_size(gsgp_handle* h, size_t* bytes) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!bytes) return fail(GSGP_ERR_ARG, "bytes is NULL");
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  *bytes = ckpt_bytes(h, ckpt_pieces(h));
  return GSGP_OK;
}

gsgp_status gsgp_checkpoint_save(gsgp_handle* h, void* h_buf, size_t bytes) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h_buf) return fail(GSGP_ERR_ARG, "h_buf is NULL");
  if (!h->evaluated) return fail(GSGP_ERR_STATE, "gsgp_eval_population has not run");
  const std::vector<CkptPiece> pieces = ckpt_pieces(h);
  const size_t need = ckpt_bytes(h, pieces);
  if (bytes < need) return fail(GSGP_ERR_ARG, "checkpoint buffer has %zu bytes, needs %zu", bytes, need);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  char* out = (char*)h_buf;
  const CkptHeader c = ckpt_header(h);
  std::memcpy(out, &c, sizeof c);
  out += sizeof c;
  for (int32_t i = 0; i < h->n_runs; ++i) {
    const int64_t shape[2] = {h->plan.runs[i].ld, h->plan.runs[i].l};
    std::memcpy(out, shape, sizeof shape);
    out += sizeof shape;
  }
  for (const CkptPiece& p : pieces) {
    HIPCHK(h, hipMemcpy(out, h->ws + p.off, p.bytes, hipMemcpyDeviceToHost));
    out += p.bytes;
  }
  return GSGP_OK;
}

gsgp_status gsgp_checkpoint_load(gsgp_handle* h, const void* h_buf, size_t bytes) {
  gsgp_status st = usable(h);
  if (st != GSGP_OK) return st;
  if (!h_buf || bytes < sizeof(CkptHeader)) return fail(GSGP_ERR_ARG, "no checkpoint");
  CkptHeader c;
  std::memcpy(&c, h_buf, sizeof c);
  if (c.magic != kCkptMagic || c.version != kCkptVersion) return fail(GSGP_ERR_ARG, "not a checkpoint of this library");
  if (!same_configuration(c, ckpt_header(h)))
    return fail(GSGP_ERR_ARG, "the checkpoint was taken with another configuration (sizes, precision, seed or "
                              "operator settings differ)");
  if (c.gen < 0 || c.gen > h->cfg.n_generations_max || c.slots < 1 ||
      (int64_t)c.slots > std::max<int64_t>(1, max_need(h->cfg.genome_len)))
    return fail(GSGP_ERR_ARG, "corrupt checkpoint header");
  const char* in = (const char*)h_buf + sizeof c;
  if (bytes < sizeof c + sizeof(int64_t) * 2 * h->n_runs) return fail(GSGP_ERR_ARG, "truncated checkpoint");
  for (int32_t i = 0; i < h->n_runs; ++i) {
    int64_t shape[2];
    std::memcpy(shape, in, sizeof shape);
    in += sizeof shape;
    if (shape[0] != h->plan.runs[i].ld || shape[1] != h->plan.runs[i].l)
      return fail(GSGP_ERR_ARG, "run %d: the checkpoint was taken on data of another shape", i);
  }
  // the pieces depend on the generation: plan them as of the saved one
  const int32_t keep_gen = h->gen;
  h->gen = c.gen;
  const std::vector<CkptPiece> pieces = ckpt_pieces(h);
  h->gen = keep_gen;
  if (bytes < ckpt_bytes(h, pieces)) return fail(GSGP_ERR_ARG, "truncated checkpoint");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (const CkptPiece& p : pieces) {
    HIPCHK(h, hipMemcpy(h->ws + p.off, in, p.bytes, hipMemcpyHostToDevice));
    in += p.bytes;
  }
  // compile the loaded genomes for this workspace (the depth words restart)
  HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStMaxDepth, 0, h->stream));
  for (int32_t b = 0; b < kLists; ++b) HIPCHK(h, launch_set_state(h->runs_d, h->n_runs, kStList0 + b, 0, h->stream));
  HIPCHK(h, launch_compile(h->runs_d, h->params, h->stream));
  int32_t* state = (int32_t*)(h->ws + h->plan.state);
  HIPCHK(h, hipMemcpyAsync(h->pinned, state, sizeof(int32_t) * kStWords * h->n_runs, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int32_t deepest = 0;
  for (int32_t r = 0; r < h->n_runs; ++r) deepest = std::max(deepest, h->pinned[kStWords * r + kStMaxDepth]);
  h->gen = c.gen;
  h->slots = std::max(1, deepest - 2);
  if (h->slots != c.slots) {
    h->poisoned = true;
    return fail(GSGP_ERR_STATE, "the loaded genomes compile to another stack depth (%d, saved %d)", h->slots, c.slots);
  }
  h->evaluated = true;
  return check_guards(h, GSGP_OK);
}

gsgp_status gsgp_guard_offsets(gsgp_handle* h, int64_t* h_offsets, int32_t max, int32_t* n) {
  if (!h) return fail(GSGP_ERR_ARG, "handle is NULL");
  if (!n || (max > 0 && !h_offsets) || max < 0) return fail(GSGP_ERR_ARG, "bad output arguments");
  const int32_t total = (int32_t)h->plan.guards.size();
  *n = total;
  for (int32_t i = 0; i < total && i < max; ++i) h_offsets[i] = (int64_t)h->plan.guards[i].at;
  return GSGP_OK;
}

}  // extern "C"
