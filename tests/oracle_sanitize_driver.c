/* Test driver for a sanitizer build of the oracle (AddressSanitizer +
 * UndefinedBehaviorSanitizer): one small GSGP run through every oracle entry
 * point, with ragged sizes, a test segment, tournaments and crossover, then
 * the paper's mutate-all loop with random steps.  Exits 0 after printing the
 * final best fitness; any sanitizer report makes the run fail. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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

void orc_genomes(const orc_config* cfg, int32_t n_features, uint32_t tag, int32_t rows, int32_t* code,
                 double* cval);
void orc_interpret(const int32_t* code, const double* cval, int32_t rows, int32_t k, const double* X, int64_t n,
                   int32_t l, double* out);
void orc_sigmoid(const double* in, double* out, int64_t count);
void orc_rmse_rows(const double* S, int32_t rows, int64_t n, const double* t, double* out);
void orc_select(const orc_config* cfg, int32_t gen, const double* F, orc_record* rec);
void orc_vary(const orc_record* rec, int32_t m, const double* S_P, const double* sigR, int64_t n, double* S_O);
int32_t orc_survive(int32_t m, const double* F_P, const double* Ft_P, double* F_O, double* Ft_O,
                    const double* S_P_train, double* S_O_train, int64_t n_train, const double* S_P_test,
                    double* S_O_test, int64_t n_test, int32_t* elite_src, int32_t* elite_dst);

static double* alloc(size_t count) {
  double* p = (double*)malloc(sizeof(double) * (count ? count : 1));
  if (!p) exit(3);
  return p;
}

static double run(int32_t m, int32_t r, int32_t k, int32_t ts, double pxo, int32_t ms_random, int64_t n_tr,
                  int64_t n_te, int32_t l, int32_t G, uint32_t seed) {
  orc_config cfg = {m, r, k, ts, pxo, 0.1, ms_random, 0, 0.80, 0.14, -1.0, 1.0, seed, 0};
  int32_t* code = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + r) * k);
  double* cval = alloc((size_t)(m + r) * k);
  orc_genomes(&cfg, l, 1u, m, code, cval);
  orc_genomes(&cfg, l, 2u, r, code + (size_t)m * k, cval + (size_t)m * k);
  double *Xtr = alloc((size_t)n_tr * l), *Xte = alloc((size_t)n_te * l), *ytr = alloc(n_tr), *yte = alloc(n_te);
  uint64_t z = 88172645463325252ull;
  for (int64_t i = 0; i < n_tr * l; ++i) Xtr[i] = (double)((z = z * 6364136223846793005ull + 1) >> 11) / 9007199254740992.0 * 2 - 1;
  for (int64_t i = 0; i < n_te * l; ++i) Xte[i] = (double)((z = z * 6364136223846793005ull + 1) >> 11) / 9007199254740992.0 * 2 - 1;
  for (int64_t i = 0; i < n_tr; ++i) ytr[i] = Xtr[i * l] * Xtr[i * l + (l - 1)] + 0.5;
  for (int64_t i = 0; i < n_te; ++i) yte[i] = Xte[i * l] * Xte[i * l + (l - 1)] + 0.5;
  double *S_tr = alloc((size_t)m * n_tr), *S_te = alloc((size_t)m * n_te);
  double *R_tr = alloc((size_t)r * n_tr), *R_te = alloc((size_t)r * n_te);
  orc_interpret(code, cval, m, k, Xtr, n_tr, l, S_tr);
  orc_interpret(code, cval, m, k, Xte, n_te, l, S_te);
  orc_interpret(code + (size_t)m * k, cval + (size_t)m * k, r, k, Xtr, n_tr, l, R_tr);
  orc_interpret(code + (size_t)m * k, cval + (size_t)m * k, r, k, Xte, n_te, l, R_te);
  orc_sigmoid(R_tr, R_tr, (int64_t)r * n_tr);
  orc_sigmoid(R_te, R_te, (int64_t)r * n_te);
  double *F = alloc(m), *Ft = alloc(m), *FO = alloc(m), *FtO = alloc(m);
  orc_rmse_rows(S_tr, m, n_tr, ytr, F);
  orc_rmse_rows(S_te, m, n_te, yte, Ft);
  orc_record* rec = (orc_record*)malloc(sizeof(orc_record) * (size_t)m);
  double *O_tr = alloc((size_t)m * n_tr), *O_te = alloc((size_t)m * n_te);
  for (int32_t g = 1; g <= G; ++g) {
    orc_select(&cfg, g, F, rec);
    orc_vary(rec, m, S_tr, R_tr, n_tr, O_tr);
    orc_vary(rec, m, S_te, R_te, n_te, O_te);
    orc_rmse_rows(O_tr, m, n_tr, ytr, FO);
    orc_rmse_rows(O_te, m, n_te, yte, FtO);
    int32_t src, dst;
    orc_survive(m, F, Ft, FO, FtO, S_tr, O_tr, n_tr, S_te, O_te, n_te, &src, &dst);
    double* t;
    t = S_tr; S_tr = O_tr; O_tr = t;
    t = S_te; S_te = O_te; O_te = t;
    t = F; F = FO; FO = t;
    t = Ft; Ft = FtO; FtO = t;
  }
  double best = INFINITY;
  for (int32_t i = 0; i < m; ++i) best = F[i] < best ? F[i] : best;
  free(code); free(cval); free(Xtr); free(Xte); free(ytr); free(yte); free(S_tr); free(S_te);
  free(R_tr); free(R_te); free(F); free(Ft); free(FO); free(FtO); free(rec); free(O_tr); free(O_te);
  return best;
}

int main(void) {
  const double a = run(17, 5, 31, 4, 0.5, 0, 203, 37, 3, 6, 7u);
  const double b = run(9, 4, 3, 0, 0.0, 1, 65, 1, 2, 5, 8u);
  if (!(isfinite(a) && isfinite(b))) return 2;
  printf("sanitized oracle ok %.17g %.17g\n", a, b);
  return 0;
}
