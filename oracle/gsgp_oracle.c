/*
 * gsgp_oracle.c -- plain FP64 CPU oracle of one GSGP run (test infrastructure).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test
 * suite, the package smoke check and the benchmark's CPU-baseline leg load
 * it.  It shares no code, header, table or constant generator with the HIP
 * library; the two agree only because each follows the method's definition.
 *
 * Method: Geometric Semantic Genetic Programming as described in
 * "GSGP-CUDA - a CUDA framework for Geometric Semantic Genetic Programming"
 * (Trujillo et al., arXiv 2106.04034):
 *   - Section 2 (software description): fitness cases, semantics, fitness as
 *     a distance to the target, the mutation operator with logistic-squashed
 *     random trees;
 *   - Section 2.2 / Algorithm 1: CreatePopulation, ComputeSemantics,
 *     ComputeFitness, GSM, survival with elitism;
 *   - Section 2.2 "Initialization" and "Interpreter" paragraphs: the linear
 *     genome and its stack interpreter with the Out register.
 * Readings where the paper is silent or ambiguous (crossover formula, the
 * sign in the mutation operator, tournament selection, protected-division
 * threshold, overflow clamp, random-number mapping) are listed in the
 * project's design notes and repeated at each function below.
 *
 * Everything is written as plain loops in the order the definitions give.
 * Rows (trees, individuals) are independent, so an OpenMP loop over rows
 * changes no result bit.  Build: gcc -O2 -fopenmp -ffp-contract=off.
 *
 * Parity pins (tests/test_oracle_*.py): Philox known-answer vectors and a
 * pure-Python twin; gene-type frequencies; hand-worked interpreter programs
 * (tests/golden/interpreter_programs.txt); random skip-free programs checked
 * against infix evaluation; sigmoid closed forms; RMSE against numpy; operator
 * identities and bounds; brute-force tournaments and rank frequencies;
 * elitism invariants; brute-force lineage reconstruction; least-squares
 * scaling against hand-worked rows, numpy's least squares, exact linear
 * targets and the optimality of the fit.  No function here is "parity
 * unpinned".
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Gene codes of the linear genome.  code >= 0 is an input feature index. */
#define ORC_ADD (-1)
#define ORC_SUB (-2)
#define ORC_MUL (-3)
#define ORC_DIV (-4)
#define ORC_CONST (-5)

#define ORC_OP_MUT 0
#define ORC_OP_XO 1

/* One offspring's variation draws (what the two auxiliary kernels of the
 * paper store, Section 2.2 "Geometric Semantic Mutation", extended with the
 * crossover parents). */
typedef struct {
  int32_t op, p1, p2, r1, r2, pad;
  double ms;
} orc_record;

typedef struct {
  int32_t pop_size, pool_size, genome_len, tournament_size;
  double p_crossover, mutation_step;
  int32_t ms_random, pad0;
  double p_function, p_feature, erc_lo, erc_hi;
  uint32_t seed, run_id;
} orc_config;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel Random
 * Numbers: As Easy as 1, 2, 3" (SC 2011): ten rounds of two 32x32->64
 * multiplies with the round multipliers below, xor of the high halves with
 * the other counter words and the key, and a Weyl-sequence key bump. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  int round;
  for (round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Integer in [0, n) from one 32-bit word by multiply-shift. */
static uint32_t orc_below(uint32_t w, uint32_t n) {
  return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* Uniform double in [0, 1) on the 2^-53 grid from two 32-bit words. */
static double orc_u53(uint32_t wa, uint32_t wb) {
  double hi = (double)(wa >> 5);  /* 27 bits */
  double lo = (double)(wb >> 6);  /* 26 bits */
  return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* Threshold T(p) so that a 32-bit word w is an event with probability p
 * when w < T(p); T(1) = 2^32 makes p = 1 certain. */
static uint64_t orc_threshold(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

uint64_t orc_event_threshold(double p) { return orc_threshold(p); }

/* ------------------------------------------------------------------------ */
/* CreatePopulation (Algorithm 1; Section 2.2 "Initialization"): every gene is
 * drawn independently: a function with probability p_function, a feature
 * with probability p_feature, otherwise an ephemeral random constant.  The
 * paper's three probabilities (0.8 / 0.14 / 0.04) do not sum to one; the
 * constant takes the remainder.  Functions and features are uniform.
 * Gene q of tree t uses Philox counter (q, t, 0, tag), key (seed, run_id);
 * tag 1 is the population, tag 2 the random-tree pool. */
void orc_genomes(const orc_config* cfg, int32_t n_features, uint32_t tag, int32_t rows,
                 int32_t* code, double* cval) {
  const int32_t k = cfg->genome_len;
  const uint64_t t_func = orc_threshold(cfg->p_function);
  const uint64_t t_feat = orc_threshold(cfg->p_function + cfg->p_feature);
  const uint32_t key[2] = {cfg->seed, cfg->run_id};
  int32_t t;
#pragma omp parallel for schedule(static)
  for (t = 0; t < rows; ++t) {
    int32_t q;
    for (q = 0; q < k; ++q) {
      uint32_t ctr[4], w[4];
      int64_t at = (int64_t)t * k + q;
      ctr[0] = (uint32_t)q;
      ctr[1] = (uint32_t)t;
      ctr[2] = 0;
      ctr[3] = tag;
      orc_philox(ctr, key, w);
      cval[at] = 0.0;
      if ((uint64_t)w[0] < t_func) {
        code[at] = -1 - (int32_t)(w[1] >> 30); /* +, -, *, / */
      } else if ((uint64_t)w[0] < t_feat) {
        code[at] = (int32_t)orc_below(w[1], (uint32_t)n_features);
      } else {
        double u = orc_u53(w[2], w[3]);
        double span = cfg->erc_hi - cfg->erc_lo;
        double scaled = span * u;
        code[at] = ORC_CONST;
        cval[at] = cfg->erc_lo + scaled;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* ComputeSemantics (Section 2.2 "Interpreter"): read the genome left to
 * right with a LIFO stack.  A terminal is pushed.  A function pops its two
 * operands (b is the top, a the one below) and pushes op(a, b); if fewer than
 * two values are on the stack it is skipped and the stack is left as it was.
 * Register Out keeps the latest valid function output and is returned at the
 * end (0.0 when no function ever runs).  Protected division returns 1.0 when
 * |b| < 1e-6.  Every function result is clamped to [-FLT_MAX, FLT_MAX] so a
 * finite input can never yield Inf or NaN. */
static double orc_eval_one(const int32_t* code, const double* cval, int32_t k,
                           const double* x, double* stack) {
  int32_t depth = 0, q;
  double out = 0.0;
  const double big = (double)FLT_MAX;
  for (q = 0; q < k; ++q) {
    int32_t g = code[q];
    if (g >= 0) {
      stack[depth++] = x[g];
    } else if (g == ORC_CONST) {
      stack[depth++] = cval[q];
    } else {
      double a, b, r;
      if (depth < 2) continue;
      b = stack[depth - 1];
      a = stack[depth - 2];
      depth -= 2;
      if (g == ORC_ADD) {
        r = a + b;
      } else if (g == ORC_SUB) {
        r = a - b;
      } else if (g == ORC_MUL) {
        r = a * b;
      } else {
        r = (fabs(b) < 1e-6) ? 1.0 : a / b;
      }
      if (r > big) r = big;
      if (r < -big) r = -big;
      stack[depth++] = r;
      out = r;
    }
  }
  return out;
}

/* out[t][c] = program t evaluated on case c; X is row-major n x l. */
void orc_interpret(const int32_t* code, const double* cval, int32_t rows, int32_t k,
                   const double* X, int64_t n, int32_t l, double* out) {
  int32_t t;
#pragma omp parallel for schedule(dynamic, 1)
  for (t = 0; t < rows; ++t) {
    double* stack = (double*)malloc(sizeof(double) * (size_t)(k + 1));
    int64_t c;
    for (c = 0; c < n; ++c) {
      out[(int64_t)t * n + c] =
          orc_eval_one(code + (int64_t)t * k, cval + (int64_t)t * k, k, X + c * l, stack);
    }
    free(stack);
  }
}

/* Logistic squashing of a random tree's output, R = 1 / (1 + e^{-T})
 * (Section 2, definition of the mutation operator). */
void orc_sigmoid(const double* in, double* out, int64_t count) {
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < count; ++i) out[i] = 1.0 / (1.0 + exp(-in[i]));
}

/* ComputeFitness (Section 2.2 "Fitness computation"): root mean squared
 * error of each semantic row against the target.  n == 0 (no test set)
 * gives 0. */
void orc_rmse_rows(const double* S, int32_t rows, int64_t n, const double* t, double* out) {
  int32_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < rows; ++i) {
    double sum = 0.0;
    int64_t c;
    for (c = 0; c < n; ++c) {
      double e = S[(int64_t)i * n + c] - t[c];
      sum += e * e;
    }
    out[i] = (n > 0) ? sqrt(sum / (double)n) : 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* Variation draws for generation `gen` (1-based).  Offspring i reads 32-bit
 * words W[w] = Philox(counter (i, w / 4, gen, 3))[w % 4]:
 *   W[0] crossover event, W[1] first pool tree, W[2] second pool tree,
 *   W[3], W[4] the random mutation step, W[5 .. 5+s) first tournament,
 *   W[5+s .. 5+2s) second tournament (s = tournament size).
 * A tournament takes s uniform candidates and keeps, scanning in draw order,
 * the first one with a strictly smaller fitness.  Crossover uses both
 * tournament winners and one pool tree; mutation the first winner and two
 * pool trees.  With s = 0 the paper's own loop applies: every individual is
 * mutated once (parent i), no selection (Section 2.1, stage 5). */
static int32_t orc_tournament(const uint32_t* w, int32_t s, int32_t m, const double* F) {
  int32_t best = (int32_t)orc_below(w[0], (uint32_t)m), j;
  for (j = 1; j < s; ++j) {
    int32_t cand = (int32_t)orc_below(w[j], (uint32_t)m);
    if (F[cand] < F[best]) best = cand;
  }
  return best;
}

void orc_select(const orc_config* cfg, int32_t gen, const double* F, orc_record* rec) {
  const int32_t m = cfg->pop_size, r = cfg->pool_size, s = cfg->tournament_size;
  const int32_t n_words = 5 + 2 * s;
  const uint64_t t_xo = orc_threshold(cfg->p_crossover);
  const uint32_t key[2] = {cfg->seed, cfg->run_id};
  int32_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < m; ++i) {
    uint32_t W[5 + 2 * 64 + 4];
    int32_t w;
    orc_record out;
    for (w = 0; w < n_words; w += 4) {
      uint32_t ctr[4], v[4];
      ctr[0] = (uint32_t)i;
      ctr[1] = (uint32_t)(w / 4);
      ctr[2] = (uint32_t)gen;
      ctr[3] = 3u;
      orc_philox(ctr, key, v);
      W[w] = v[0];
      W[w + 1] = v[1];
      W[w + 2] = v[2];
      W[w + 3] = v[3];
    }
    memset(&out, 0, sizeof out);
    if (s > 0 && (uint64_t)W[0] < t_xo) {
      out.op = ORC_OP_XO;
      out.p1 = orc_tournament(W + 5, s, m, F);
      out.p2 = orc_tournament(W + 5 + s, s, m, F);
      out.r1 = (int32_t)orc_below(W[1], (uint32_t)r);
      out.r2 = -1;
      out.ms = 0.0;
    } else {
      out.op = ORC_OP_MUT;
      out.p1 = (s > 0) ? orc_tournament(W + 5, s, m, F) : i;
      out.p2 = -1;
      out.r1 = (int32_t)orc_below(W[1], (uint32_t)r);
      out.r2 = (int32_t)orc_below(W[2], (uint32_t)r);
      out.ms = cfg->ms_random ? cfg->mutation_step * orc_u53(W[3], W[4]) : cfg->mutation_step;
    }
    rec[i] = out;
  }
}

/* GSM / GSC on one segment (train or test) of n cases (Section 2, and
 * Algorithm 1's GSM kernel).  Mutation: O = T + ms * (R1 - R2), with the
 * minus sign (read so that R1 == R2 leaves the parent unchanged).
 * Crossover: O = T1 * R + T2 * (1 - R).  Here sigR already holds
 * R = 1 / (1 + e^{-T_u}) for every pool tree. */
void orc_vary(const orc_record* rec, int32_t m, const double* S_P, const double* sigR,
              int64_t n, double* S_O) {
  int32_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < m; ++i) {
    const orc_record* d = &rec[i];
    int64_t c;
    double* o = S_O + (int64_t)i * n;
    if (d->op == ORC_OP_XO) {
      const double* t1 = S_P + (int64_t)d->p1 * n;
      const double* t2 = S_P + (int64_t)d->p2 * n;
      const double* rr = sigR + (int64_t)d->r1 * n;
      for (c = 0; c < n; ++c) o[c] = t1[c] * rr[c] + t2[c] * (1.0 - rr[c]);
    } else {
      const double* t = S_P + (int64_t)d->p1 * n;
      const double* ra = sigR + (int64_t)d->r1 * n;
      const double* rb = sigR + (int64_t)d->r2 * n;
      for (c = 0; c < n; ++c) o[c] = t[c] + d->ms * (ra[c] - rb[c]);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Local search (the paper's Section 3.2 names GSGP with a local search
 * method as the next step and Section 5 lists it as future work; neither
 * defines it).  Reading: every offspring O formed by a variation operator is
 * replaced by its least-squares linear scaling alpha + beta * O, with
 * (alpha, beta) the simple linear regression of the training target t on O
 * over the training cases.  The same (alpha, beta) scale the offspring's
 * test cases.  With O = T + ms (R1 - R2) this is the regression-based local
 * search of the mutation restricted to one coefficient on both mutation
 * terms.  A (numerically) constant offspring has no regression slope: when
 * sum (o - mean o)^2 <= 1e-10 * sum o^2 the offspring is kept unscaled
 * (alpha = 0, beta = 1).
 * Two-pass textbook form: means first, then centred sums. */
void orc_ls_fit(const double* O, int32_t rows, int64_t n, const double* t, double* alpha, double* beta) {
  int32_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < rows; ++i) {
    const double* o = O + (int64_t)i * n;
    double so = 0.0, st = 0.0, soo = 0.0, sxx = 0.0, sxy = 0.0, mo, mt;
    int64_t c;
    for (c = 0; c < n; ++c) {
      so += o[c];
      st += t[c];
      soo += o[c] * o[c];
    }
    mo = so / (double)n;
    mt = st / (double)n;
    for (c = 0; c < n; ++c) {
      const double dx = o[c] - mo;
      const double dy = t[c] - mt;
      sxx += dx * dx;
      sxy += dx * dy;
    }
    if (n > 0 && sxx > 1e-10 * soo) {
      beta[i] = sxy / sxx;
      alpha[i] = mt - beta[i] * mo;
    } else {
      alpha[i] = 0.0;
      beta[i] = 1.0;
    }
  }
}

/* O[i][c] <- alpha[i] + beta[i] * O[i][c]. */
void orc_ls_apply(double* O, int32_t rows, int64_t n, const double* alpha, const double* beta) {
  int32_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < rows; ++i) {
    double* o = O + (int64_t)i * n;
    int64_t c;
    for (c = 0; c < n; ++c) o[c] = alpha[i] + beta[i] * o[c];
  }
}

/* ------------------------------------------------------------------------ */
/* Survival with elitism (Section 2.2 "Survival"; Algorithm 1): the
 * offspring replace the parents, except that when the best parent is
 * strictly better than the best offspring it replaces the worst offspring.
 * Ties go to the lowest index (the first extremum).  The caller swaps the
 * buffers afterwards.  Returns 1 when the elite was copied and reports the
 * source parent and the overwritten offspring. */
int32_t orc_argmin(const double* F, int32_t m) {
  int32_t b = 0, i;
  for (i = 1; i < m; ++i)
    if (F[i] < F[b]) b = i;
  return b;
}

int32_t orc_argmax(const double* F, int32_t m) {
  int32_t b = 0, i;
  for (i = 1; i < m; ++i)
    if (F[i] > F[b]) b = i;
  return b;
}

int32_t orc_survive(int32_t m, const double* F_P, const double* Ft_P, double* F_O, double* Ft_O,
                    const double* S_P_train, double* S_O_train, int64_t n_train,
                    const double* S_P_test, double* S_O_test, int64_t n_test,
                    int32_t* elite_src, int32_t* elite_dst) {
  int32_t bP = orc_argmin(F_P, m);
  int32_t bO = orc_argmin(F_O, m);
  *elite_src = -1;
  *elite_dst = -1;
  if (F_P[bP] < F_O[bO]) {
    int32_t w = orc_argmax(F_O, m);
    memcpy(S_O_train + (int64_t)w * n_train, S_P_train + (int64_t)bP * n_train,
           sizeof(double) * (size_t)n_train);
    if (n_test > 0)
      memcpy(S_O_test + (int64_t)w * n_test, S_P_test + (int64_t)bP * n_test,
             sizeof(double) * (size_t)n_test);
    F_O[w] = F_P[bP];
    Ft_O[w] = Ft_P[bP];
    *elite_src = bP;
    *elite_dst = w;
    return 1;
  }
  return 0;
}

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
