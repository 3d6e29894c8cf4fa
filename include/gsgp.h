/*
 * gsgp.h -- C ABI of the MI355X (gfx950) GSGP hot-path library, libgsgp.so.
 *
 * The library runs Geometric Semantic Genetic Programming as stated in
 * "GSGP-CUDA - a CUDA framework for Geometric Semantic Genetic Programming"
 * (Trujillo et al., arXiv 2106.04034), Algorithm 1: given population size m,
 * random-tree pool size r, fitness cases (n x l) with target t, program size k
 * and a number of generations g, build random linear genomes, interpret them
 * once into semantic matrices, then evolve by geometric semantic operators
 * acting on semantic vectors only, with RMSE fitness and elitist survival.
 *
 * Conventions shared by every entry point:
 *  - Every call returns a gsgp_status; nothing throws across the ABI.
 *  - Arguments are validated before any device work; a rejected call
 *    changes no state.
 *  - Device memory is owned by the caller.  The library never calls
 *    hipMalloc/hipFree; it carves the caller's workspace.  The handle owns
 *    only host memory and a HIP graph cache.  The one device array of the
 *    library's own is the static scratch of gsgp_reconstruct_static
 *    (GSGP_STATIC_SCRATCH_BYTES on each GPU it runs on).
 *  - All device work is enqueued on the HIP stream given to gsgp_init (NULL
 *    is the legacy default stream).  Calls that return host data (getters,
 *    h_stats != NULL) synchronise that stream.  A handle is not thread safe.
 *  - After a HIP error the handle is poisoned: later calls return
 *    GSGP_ERR_STATE until gsgp_destroy.
 *  - gsgp_last_error() returns a thread-local message for the last failure.
 *
 * One handle holds n_runs >= 1 independent runs that share a gsgp_config
 * but may differ in data (n_train, n_test, n_features).  n_runs == 1 is the
 * plain single-run form; n_runs > 1 is the batched form, where every stage of
 * a generation is one launch over all runs.
 */
#ifndef GSGP_H
#define GSGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GSGP_OK = 0,
  GSGP_ERR_ARG = -1,         /* invalid argument or configuration            */
  GSGP_ERR_STATE = -2,       /* wrong call order, or handle poisoned         */
  GSGP_ERR_WORKSPACE = -3,   /* workspace too small or misaligned            */
  GSGP_ERR_NONFINITE = -4,   /* NaN or Inf in X or y                         */
  GSGP_ERR_HIP = -5,         /* a HIP runtime call failed (handle poisoned)  */
  GSGP_ERR_UNSUPPORTED = -6  /* valid input beyond what this build supports  */
} gsgp_status;

/* Storage/arithmetic precision of semantic vectors in the generation loop.
 * The interpreter, fitness combination and reconstruction are FP64 in every
 * form; the FP32 forms round semantics once when they are stored.
 *   GSGP_FP64        : FP64 semantics, FP64 arithmetic.
 *   GSGP_FP32        : FP32 semantics and arithmetic, plain FP32 sums of
 *                      squared residuals within each 512-case chunk.
 *   GSGP_FP32_KAHAN  : as GSGP_FP32 with compensated (Kahan / two-sum)
 *                      chunk sums.
 * Chunk sums are combined in FP64 in a fixed order in every form. */
typedef enum { GSGP_FP64 = 0, GSGP_FP32 = 1, GSGP_FP32_KAHAN = 2 } gsgp_precision;

/* gsgp_config.flags */
#define GSGP_FLAG_NO_GRAPH 1u  /* launch generations one by one, no HIP graph */
#define GSGP_FLAG_GUARDS 2u    /* debug: a 256-byte guard pattern after every workspace
                                  buffer (gsgp_workspace_size grows accordingly), checked
                                  after every call that launches kernels; an overwritten
                                  guard poisons the handle (GSGP_ERR_STATE) */
#define GSGP_FLAG_LOCAL_SEARCH 4u /* GSGP with local search (named in Sections 3.2 and 5 of
                                  the paper, not defined there): every offspring O of a
                                  variation operator becomes alpha + beta * O, with
                                  (alpha, beta) the least-squares fit of the training
                                  target on O over the training cases; the same scaling
                                  applies to the offspring's test cases.  A numerically
                                  constant offspring (sum (o - mean o)^2 <= 1e-10 *
                                  sum o^2) is kept (alpha = 0, beta = 1).  The scaling
                                  of every individual is kept (gsgp_get_scaling) and
                                  followed by reconstruction and export. */

/* Run parameters: the inputs of Algorithm 1 plus operator settings.
 * Defaults used by the project's workloads are given in brackets. */
typedef struct {
  int32_t pop_size;          /* m, >= 1                                         */
  int32_t pool_size;         /* r, >= 1 random trees for the operators         */
  int32_t genome_len;        /* k, 1..4096 genes per linear genome [127]       */
  int32_t n_generations_max; /* capacity of the ancestry record, >= 1          */
  int32_t tournament_size;   /* 1..64 [4]; 0 = the paper's loop: every
                                individual is mutated once, no selection
                                (requires p_crossover == 0)                    */
  int32_t ms_random;         /* 0: step = mutation_step; 1: step drawn
                                uniformly in [0, mutation_step) per offspring  */
  double p_crossover;        /* probability of crossover per offspring [0.5]   */
  double mutation_step;      /* ms [0.1], >= 0                                 */
  double p_function;         /* gene is a function [0.80]                      */
  double p_feature;          /* gene is a feature [0.14]; constant otherwise   */
  double erc_lo, erc_hi;     /* ephemeral random constant range [-1, 1]        */
  int32_t precision;         /* gsgp_precision                                  */
  uint32_t seed;             /* Philox key word 0; key word 1 is the run index */
  uint32_t flags;            /* GSGP_FLAG_*                                     */
  int32_t reserved;          /* must be 0                                       */
} gsgp_config;

/* Data of one run.  Pointers are DEVICE pointers to FP64 arrays in the
 * layout of the paper's train/test files (Section 3.3): row-major, one row
 * per fitness case.  They are read only during gsgp_init, which copies them
 * into the workspace; the caller may free them afterwards. */
typedef struct {
  int64_t n_train;           /* >= 1                                            */
  int64_t n_test;            /* >= 0                                            */
  int32_t n_features;        /* l >= 1                                          */
  int32_t reserved;          /* must be 0                                       */
  const double* X_train;     /* n_train x n_features                            */
  const double* y_train;     /* n_train                                         */
  const double* X_test;      /* n_test x n_features; NULL iff n_test == 0       */
  const double* y_test;      /* n_test; NULL iff n_test == 0                    */
} gsgp_run;

/* Variation draws of one offspring (what the paper's two auxiliary kernels
 * store before GSM, Section 2.2, extended with crossover parents).
 *   op 0 = mutation  O = S[p1] + ms * (sigma(R[r1]) - sigma(R[r2]))   (p2 = -1)
 *   op 1 = crossover O = S[p1] * sigma(R[r1]) + S[p2] * (1 - sigma(R[r1]))
 *                                                          (r2 = -1, ms = 0)
 *   op 2 = elite copy of parent p1 (only in the lineage view of
 *          gsgp_get_records, never stored on the device)                   */
typedef struct {
  int32_t op, p1, p2, r1, r2, reserved;
  double ms;
} gsgp_record;

/* Per-generation summary (the paper's two output files, Section 3.3: best
 * train fitness and the same individual's test fitness), plus the survival
 * decision: when elite_copied, parent elite_src replaced offspring elite_dst. */
typedef struct {
  double best_train_rmse;
  double best_test_rmse;     /* 0 when the run has no test cases               */
  int32_t best_index;
  int32_t elite_copied;
  int32_t elite_src;
  int32_t elite_dst;
} gsgp_gen_stats;

typedef struct gsgp_handle gsgp_handle;

/* Bytes of device workspace gsgp_init needs for these runs (Section 2.3's
 * memory complexity: O(mk + rk + 2mn + rn + nl), plus the ancestry record of
 * n_generations_max generations).  Pure host computation.
 * Errors: GSGP_ERR_ARG for an invalid config or run description. */
gsgp_status gsgp_workspace_size(const gsgp_config* cfg, const gsgp_run* runs, int32_t n_runs,
                                size_t* bytes);

/* Algorithm 1 set-up (Section 2.1 stages 1-2: work ranges and memory).
 * Validates cfg and runs, carves d_workspace (device, >= gsgp_workspace_size
 * bytes, 256-byte aligned), copies X into padded case tiles and y
 * into the storage precision, checks that X and y are finite, and synchronises
 * the stream.  hip_stream is a hipStream_t (NULL = default stream).
 * Errors: GSGP_ERR_ARG, GSGP_ERR_WORKSPACE (too small / misaligned),
 * GSGP_ERR_NONFINITE (no handle is returned), GSGP_ERR_HIP. */
gsgp_status gsgp_init(const gsgp_config* cfg, const gsgp_run* runs, int32_t n_runs,
                      void* d_workspace, size_t ws_bytes, void* hip_stream, gsgp_handle** out);

/* Algorithm 1 before the loop: CreatePopulation(m), CreatePopulation(r),
 * ComputeSemantics(P), ComputeSemantics(R), ComputeFitness (Section 2.2,
 * "Initialization", "Interpreter", "Fitness computation").  Starts (or
 * restarts) every run at generation 0 and draws generation 1's variation.
 * Genomes are drawn from Philox unless h_codes/h_consts (HOST arrays,
 * [n_runs][m + r][k], population rows then pool rows; code >= 0 is a feature,
 * -1 +, -2 -, -3 *, -4 protected /, -5 constant with its value in h_consts)
 * are given; both or neither.  Every genome is accepted: stacks that do not
 * fit a wavefront's LDS column are kept in the workspace's spill stacks
 * (sized by gsgp_workspace_size for genome_len), so no population is refused
 * once the arguments are valid.  Arguments (genome codes in range, finite
 * constants) are checked on the host before any device work, so a rejected
 * call leaves the current run untouched.  Asynchronous apart from one small
 * read-back.
 * Errors: GSGP_ERR_ARG (bad genome code or constant), GSGP_ERR_STATE,
 * GSGP_ERR_HIP. */
gsgp_status gsgp_eval_population(gsgp_handle* h, const int32_t* h_codes, const double* h_consts);

/* Algorithm 1's loop body, n_gens times: variation draws (tournaments),
 * GSM/GSC on train and test semantics, ComputeFitness, survival with
 * elitism (Section 2.2).  h_stats (HOST, nullable) receives
 * [n_runs][n_gens] summaries and synchronises the stream.  Unless
 * GSGP_FLAG_NO_GRAPH is set, one generation and a block of 16 generations
 * are each captured once in a HIP graph and replayed (16 at a time, then one
 * at a time for the rest).
 * Errors: GSGP_ERR_ARG (n_gens < 1 or beyond n_generations_max),
 * GSGP_ERR_STATE (before gsgp_eval_population), GSGP_ERR_HIP. */
gsgp_status gsgp_generation(gsgp_handle* h, int32_t n_gens, gsgp_gen_stats* h_stats);

/* As gsgp_generation, but the variation draws are given instead of drawn:
 * h_records (HOST, [n_runs][n_gens][m]) must hold op 0 or 1 entries with
 * indices in range.  h_elite (HOST, nullable, [n_runs][n_gens]) dictates the
 * survival decision through its elite_copied/elite_src/elite_dst fields;
 * when NULL the device decides.  Used to follow a given lineage, e.g. to
 * evaluate one lineage at another precision.
 * Errors: as gsgp_generation, plus GSGP_ERR_ARG for an invalid record. */
gsgp_status gsgp_generation_replay(gsgp_handle* h, int32_t n_gens, const gsgp_record* h_records,
                                   const gsgp_gen_stats* h_elite, gsgp_gen_stats* h_stats);

/* Device scratch bytes gsgp_reconstruct needs for (run, gen, individual) on
 * n new cases (the lineage's generation-0 and pool programs on n cases, two
 * generations of its ancestors, the replay lists, and spill stacks when a
 * program's stack exceeds an LDS column).  Reads the ancestry record
 * (synchronises the stream).
 * Errors: GSGP_ERR_ARG, GSGP_ERR_STATE. */
gsgp_status gsgp_reconstruct_scratch_size(gsgp_handle* h, int32_t run, int32_t gen,
                                          int32_t individual, int64_t n, size_t* bytes);

/* "Return: best individual found" (Algorithm 1) as a model: the FP64
 * semantics of individual `individual` of generation `gen` (<= the current
 * generation) of run `run` on n new cases d_X (DEVICE, row-major n x l, FP64).
 * Walks the ancestry record (Section 2.1 stage 3, lineage structures) back to
 * the generation-0 genomes and pool trees, interprets them on d_X and replays
 * the recorded combinations forward.  d_out (DEVICE, n FP64) receives the
 * result; d_scratch (DEVICE, >= gsgp_reconstruct_scratch_size bytes, 256-byte
 * aligned) is caller-owned scratch.  Synchronises the stream.
 * Errors: GSGP_ERR_ARG, GSGP_ERR_WORKSPACE, GSGP_ERR_STATE, GSGP_ERR_HIP. */
gsgp_status gsgp_reconstruct(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual,
                             const double* d_X, int64_t n, double* d_out, void* d_scratch,
                             size_t scratch_bytes);

/* Bytes of the device scratch array that gsgp_reconstruct_static uses on
 * each GPU (64 MiB). */
#define GSGP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reconstruction as gsgp_reconstruct, with its scratch taken from an array
 * of GSGP_STATIC_SCRATCH_BYTES that the library keeps on each GPU it runs on
 * for the life of the process, instead of caller scratch.  The caller still
 * passes d_X and d_out (DEVICE).  The call makes no device allocation.  A
 * reconstruction that needs more scratch than the array holds (see
 * gsgp_reconstruct_scratch_size) is refused with GSGP_ERR_WORKSPACE before
 * any device work.  All calls on one GPU share its array, which keeps the
 * last call's contents (every byte a call reads it has written first): the
 * library serialises such calls within a process with a lock, and the call
 * returns only after its work is done (it synchronises the stream).  Work on
 * other streams that overlapped one of these calls could not touch the
 * array, which is internal to the library.
 * Errors: as gsgp_reconstruct; GSGP_ERR_UNSUPPORTED for a device index
 * beyond 63. */
gsgp_status gsgp_reconstruct_static(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual,
                                    const double* d_X, int64_t n, double* d_out);

/* Compact model of a mutation-only lineage (the paper's own loop; GSM,
 * Section 2, and the lineage structures of Section 2.1 stage 3): individual
 * `individual` of generation `gen` of run `run` equals
 * c + b * T(x) + sum_j w_j * sigmoid(R_j(x)), with T the generation-0
 * population tree *h_tree (HOST) and R_j the pool trees (genomes from
 * gsgp_get_genomes).  h_affine (HOST, 2 doubles) receives (c, b), which are
 * (0, 1) without local search; h_weights (HOST, r doubles) receives w.  Both
 * are accumulated forward generation by generation: with the step's
 * offspring scaling (alpha, beta) ((0, 1) without local search),
 * c = alpha + beta c, b = beta b, w = beta w, then w[r1] += beta ms and
 * w[r2] -= beta ms.  Reads the ancestry record (synchronises the stream).
 * Errors: GSGP_ERR_ARG, GSGP_ERR_STATE, GSGP_ERR_UNSUPPORTED (the lineage
 * contains a crossover), GSGP_ERR_HIP. */
gsgp_status gsgp_export_linear(gsgp_handle* h, int32_t run, int32_t gen, int32_t individual,
                               int32_t* h_tree, double* h_affine, double* h_weights);

/* ---- inspection (HOST outputs; each synchronises the stream) ---------- */
/* These return the state Algorithm 1 keeps between its steps: the
 * population's fitness and semantics (the S_P matrix and the fitness vector
 * of Algorithm 1's loop, Section 2.2), the squashed pool (the random
 * functions R_u of GSM, Section 2), the variation draws and survival
 * decisions that form the lineage structures (Section 2.1 stage 3), the
 * per-generation summaries the paper writes to its two output files
 * (Section 3.3) and the generation-0 genomes (CreatePopulation, Section 2.2
 * "Initialization"). */

/* Current generation number (0 after gsgp_eval_population); Algorithm 1's
 * generation counter. */
gsgp_status gsgp_current_generation(gsgp_handle* h, int32_t* gen);

/* Train and test RMSE of the current population of `run` (m FP64 each):
 * ComputeFitness's output (Section 2.2 "Fitness computation"). */
gsgp_status gsgp_get_fitness(gsgp_handle* h, int32_t run, double* h_train, double* h_test);

/* Semantics of `run` as FP64: which = 0 the current population
 * [m][n_train + n_test], which = 1 the squashed pool sigma(S_R)
 * [r][n_train + n_test]; train cases then test cases in each row
 * (ComputeSemantics / GSM outputs, Algorithm 1). */
gsgp_status gsgp_get_semantics(gsgp_handle* h, int32_t run, int32_t which, double* h_out);

/* Rows row0 .. row0 + n_rows - 1 of the same (h_out: [n_rows][n_train +
 * n_test] FP64), copying only those rows from the device: for inspecting a
 * few individuals of a large run. */
gsgp_status gsgp_get_semantics_rows(gsgp_handle* h, int32_t run, int32_t which, int32_t row0, int32_t n_rows,
                                    double* h_out);

/* Cases case0 .. case0 + n_cases - 1 (train cases first, then test cases, as
 * in a row of gsgp_get_semantics) of every row (h_out: [m or r][n_cases]
 * FP64), copying only those cases from the device: for inspecting a slice of
 * the fitness cases of a large run.
 * Errors: GSGP_ERR_ARG (range outside [0, n_train + n_test)), GSGP_ERR_STATE,
 * GSGP_ERR_HIP. */
gsgp_status gsgp_get_semantics_cases(gsgp_handle* h, int32_t run, int32_t which, int64_t case0, int64_t n_cases,
                                     double* h_out);

/* Variation records of generations gen0 .. gen0 + n_gens - 1 (1-based,
 * <= current), [n_gens][m]: the draws of the paper's auxiliary kernels
 * before GSM (Section 2.2) that, with the survival decisions, make up the
 * lineage structures (Section 2.1 stage 3).  raw = 1 returns the draws as
 * made; raw = 0 returns the lineage view, where the offspring replaced by an
 * elite copy shows op 2 with p1 = the elite parent. */
gsgp_status gsgp_get_records(gsgp_handle* h, int32_t run, int32_t gen0, int32_t n_gens,
                             int32_t raw, gsgp_record* h_out);

/* Summaries of generations gen0 .. gen0 + n_gens - 1 (0 = initial): best
 * train RMSE and the same individual's test RMSE, the two values per
 * generation the paper writes to its output files (Section 3.3), plus the
 * survival decision. */
gsgp_status gsgp_get_stats(gsgp_handle* h, int32_t run, int32_t gen0, int32_t n_gens,
                           gsgp_gen_stats* h_out);

/* Local search scaling (GSGP_FLAG_LOCAL_SEARCH) of every individual of
 * generations gen0 .. gen0 + n_gens - 1 (0 = initial, <= current):
 * h_out [n_gens][m][2] (alpha, beta); the individual's semantics are
 * alpha + beta * (its operator's output), an elite copy carries its source's
 * scaling, and generation 0 is (0, 1).  Without local search every entry is
 * (0, 1). */
gsgp_status gsgp_get_scaling(gsgp_handle* h, int32_t run, int32_t gen0, int32_t n_gens, double* h_out);

/* Generation-0 genomes of `run`: [m + r][k] codes and constants
 * (CreatePopulation's output, Section 2.2 "Initialization"). */
gsgp_status gsgp_get_genomes(gsgp_handle* h, int32_t run, int32_t* h_codes, double* h_consts);

/* ---- measurement ------------------------------------------------------ */

/* Runs n_gens generations without a graph, timing every stage with HIP
 * events on the library stream, and writes the mean milliseconds per launch
 * to h_ms[0..3]: selection+survival, variation (GSM/GSC + fitness partials),
 * fitness combination, and the whole generation.  Advances the runs. */
gsgp_status gsgp_time_stages(gsgp_handle* h, int32_t n_gens, double* h_ms);

/* Runs gsgp_eval_population (Philox genomes) with HIP events between its
 * stages and writes the milliseconds of each to h_ms[0..3]: CreatePopulation
 * (genomes), ComputeSemantics (genome compilation and interpretation of
 * population and pool, including one small read-back), initial fitness and
 * the first variation draws, and the whole initialisation -- the stage
 * categories of the paper's speed-up study (Section 3.1).  Restarts the runs
 * at generation 0.  Errors: as gsgp_eval_population. */
gsgp_status gsgp_time_eval(gsgp_handle* h, double* h_ms);

/* Launch shape of the variation kernel: waves per block (1..8) and
 * offspring per block task (0 keeps the current value for either), XCD-aware
 * block order (0 none; 1 each XCD takes a contiguous range of tasks; 2 the
 * XCDs take neighbouring case chunks side by side), and max_blocks (0 = one block per task; > 0 = a
 * persistent grid of at most that many blocks looping over tasks).  Shapes
 * never change results: partial sums follow a fixed chunking of the cases.
 * Errors: GSGP_ERR_ARG. */
gsgp_status gsgp_set_launch(gsgp_handle* h, int32_t waves_per_block, int32_t offspring_per_block,
                            int32_t xcd_remap, int32_t max_blocks);

/* Times candidate launch shapes of the variation kernel on the live buffers
 * (the kernel is idempotent within a generation, so the runs do not
 * advance) and keeps the fastest.  h_best (HOST, nullable) receives
 * {waves_per_block, offspring_per_block, xcd_remap, max_blocks}.
 * Errors: GSGP_ERR_STATE (also when no generation is left to run),
 * GSGP_ERR_HIP. */
gsgp_status gsgp_autotune(gsgp_handle* h, int32_t* h_best);

/* ---- checkpoint / resume ---------------------------------------------- */

/* Size of a checkpoint of every run at the current generation (after
 * gsgp_eval_population).  Errors: GSGP_ERR_ARG, GSGP_ERR_STATE. */
gsgp_status gsgp_checkpoint_size(gsgp_handle* h, size_t* bytes);

/* Writes the checkpoint into h_buf (HOST, >= gsgp_checkpoint_size bytes):
 * the current population semantics and fitness, the squashed pool, the
 * genomes (the loading handle compiles them for its own workspace), the
 * ancestry record so far (including the next generation's draws), the
 * scaling table and target sums with local search, and the state words.  Every later draw is a
 * function of (seed, run, offspring, generation) and the fitness (Philox
 * counters), so a handle that loads it continues bit for bit.  Synchronises
 * the stream.  Errors: GSGP_ERR_ARG, GSGP_ERR_STATE, GSGP_ERR_HIP. */
gsgp_status gsgp_checkpoint_save(gsgp_handle* h, void* h_buf, size_t bytes);

/* Restores a checkpoint into a handle made with the same configuration
 * (sizes, generations, precision, seed, every operator setting and the
 * local-search flag; launch and debug flags may differ) on data of the same
 * shapes (the data itself is the caller's); the handle is then at the saved
 * generation, as if gsgp_eval_population and those generations had run.  A
 * later gsgp_eval_population restarts from generation 0.
 * Errors: GSGP_ERR_ARG (not a checkpoint, other configuration, truncated,
 * or written by another checkpoint version of the library), GSGP_ERR_STATE,
 * GSGP_ERR_HIP. */
gsgp_status gsgp_checkpoint_load(gsgp_handle* h, const void* h_buf, size_t bytes);

/* Byte offsets (within the workspace) of the guards that GSGP_FLAG_GUARDS
 * places after every buffer: *n receives their number, h_offsets (HOST,
 * nullable when max = 0) the first min(max, *n) offsets.  For diagnostics
 * and tests of the guard check itself.  Errors: GSGP_ERR_ARG. */
gsgp_status gsgp_guard_offsets(gsgp_handle* h, int64_t* h_offsets, int32_t max, int32_t* n);

/* Releases host resources.  The workspace stays the caller's. */
gsgp_status gsgp_destroy(gsgp_handle* h);

const char* gsgp_status_string(gsgp_status s);
const char* gsgp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GSGP_H */
