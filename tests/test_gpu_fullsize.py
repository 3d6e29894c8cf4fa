"""Parity at the benchmark's full size (single_fp32_100k: 100,000 train /
25,000 test cases, 20 features, m = r = 1,024, FP32, the launch shape the
benchmark uses), on sampled outputs the oracle computes one by one and on
properties that hold at any size.

Bars:
  - genomes: bit-exact (integer draws, constants from the same FP64 ops);
  - population semantics: the FP32 rounding of the oracle's FP64 value,
    bit-exact (the interpreter is bit-exact in FP64 and rounds once);
    pool: within 1 FP32 ulp (exp rounding may cross a rounding boundary);
  - generation-0 fitness of sampled individuals: 1e-4 relative (the FP32
    form's bar; storage rounding of S and t, FP32 chunk sums);
  - tournaments: every recorded winner is the first strict minimum among
    the candidates that an independent Philox twin draws, under the GPU's
    own fitness; pool indices and operator choice equal the twin's draws;
  - offspring: each sampled element equals the operator evaluated in FP32
    on the stored parent / pool values (same operations, bit-exact);
  - fitness of sampled offspring against an FP64 RMSE of the stored FP32
    row: 1e-5 relative;
  - elitism: best train RMSE never increases; an elite row is a byte copy.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2106_04034_amd import gsgp, synth
from tests import pyphilox
from tests.gpu_helpers import oracle_config

pytestmark = pytest.mark.gpu

G_TEST = 6


@pytest.fixture(scope="module")
def run():
    wl = synth.WORKLOADS["single_fp32_100k"]
    d = synth.single_run(wl.n_train, wl.n_test, wl.n_features)
    s = gsgp.Settings(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                      n_generations_max=G_TEST, tournament_size=wl.tournament_size,
                      p_crossover=wl.p_crossover, mutation_step=wl.mutation_step,
                      precision=gsgp.FP32, seed=synth.evolution_seed(1))
    R = gsgp.Runner(s, [d])
    R.set_launch(4, 4, 1, 0)
    R.eval_population()
    S0 = R.semantics(0, 0).astype(np.float32)
    sig = R.semantics(0, 1).astype(np.float32)
    F0, Ft0 = R.fitness(0)
    codes, consts = R.genomes(0)
    R.generation(1)
    S1 = R.semantics(0, 0).astype(np.float32)
    F1, Ft1 = R.fitness(0)
    rec1 = R.records(0, 1, 1)[0]
    st1 = R.stats(0, 1, 1)[0]
    R.generation(G_TEST - 1)
    stats = R.stats(0, 0, G_TEST + 1)
    yield dict(R=R, d=d, s=s, S0=S0, sig=sig, F0=F0, Ft0=Ft0, codes=codes, consts=consts,
               S1=S1, F1=F1, Ft1=Ft1, rec1=rec1, st1=st1, stats=stats)
    R.close()


def test_genomes_bit_exact(run):
    s, d = run["s"], run["d"]
    ocfg = oracle_config(s)
    cp, vp = orc.genomes(ocfg, d.n_features, orc.TAG_POPULATION, s.pop_size)
    cr, vr = orc.genomes(ocfg, d.n_features, orc.TAG_POOL, s.pool_size)
    assert np.array_equal(run["codes"], np.concatenate([cp, cr]))
    assert np.array_equal(run["consts"], np.concatenate([vp, vr]))


def test_sampled_semantics(run):
    s, d = run["s"], run["d"]
    rng = np.random.default_rng(0)
    X = np.concatenate([d.X_train, d.X_test])
    cases = np.sort(rng.choice(X.shape[0], size=1500, replace=False))
    cases[0], cases[-1] = 0, X.shape[0] - 1
    pop = rng.choice(s.pop_size, size=12, replace=False)
    pool = rng.choice(s.pool_size, size=12, replace=False)
    codes, consts = run["codes"], run["consts"]
    want = orc.interpret(codes[pop], consts[pop], X[cases]).astype(np.float32)
    got = run["S0"][pop][:, cases]
    assert np.array_equal(got, want)
    rows = s.pop_size + pool
    want_p = orc.sigmoid(orc.interpret(codes[rows], consts[rows], X[cases])).astype(np.float32)
    got_p = run["sig"][pool][:, cases]
    ulp = np.spacing(np.abs(want_p).astype(np.float32))
    assert np.all(np.abs(got_p - want_p) <= ulp)


def test_sampled_generation0_fitness(run):
    s, d = run["s"], run["d"]
    rng = np.random.default_rng(1)
    idx = rng.choice(s.pop_size, size=6, replace=False)
    codes, consts = run["codes"], run["consts"]
    S_tr = orc.interpret(codes[idx], consts[idx], d.X_train)
    S_te = orc.interpret(codes[idx], consts[idx], d.X_test)
    F = orc.rmse_rows(S_tr, d.y_train)
    Ft = orc.rmse_rows(S_te, d.y_test)
    assert np.all(np.abs(run["F0"][idx] - F) <= 1e-4 * F)
    assert np.all(np.abs(run["Ft0"][idx] - Ft) <= 1e-4 * Ft)


def test_tournaments_valid_under_gpu_fitness(run):
    s = run["s"]
    rec, F0 = run["rec1"], run["F0"]
    m, r, ts = s.pop_size, s.pool_size, s.tournament_size
    for i in range(0, m, 7):
        W = pyphilox.words(i, 1, 5 + 2 * ts, s.seed, 0)
        xo = W[0] < pyphilox.threshold(s.p_crossover)
        assert rec[i]["op"] == (1 if xo else 0)
        assert rec[i]["r1"] == pyphilox.below(W[1], r)

        def winner(ws):
            c = [pyphilox.below(w, m) for w in ws]
            b = c[0]
            for x in c[1:]:
                if F0[x] < F0[b]:
                    b = x
            return b

        assert rec[i]["p1"] == winner(W[5:5 + ts])
        if xo:
            assert rec[i]["p2"] == winner(W[5 + ts:5 + 2 * ts])
        else:
            assert rec[i]["r2"] == pyphilox.below(W[2], r)


def test_sampled_offspring_elements_and_fitness(run):
    s, d = run["s"], run["d"]
    S0, sig, S1, rec, st = run["S0"], run["sig"], run["S1"], run["rec1"], run["st1"]
    rng = np.random.default_rng(2)
    n_all = S0.shape[1]
    cols = rng.choice(n_all, size=4000, replace=False)
    one = np.float32(1.0)
    for i in rng.choice(s.pop_size, size=40, replace=False):
        if st["elite_copied"] and i == st["elite_dst"]:
            assert np.array_equal(S1[i], S0[st["elite_src"]])
            continue
        d_ = rec[i]
        if d_["op"] == 1:
            x, y, z = S0[d_["p1"], cols], S0[d_["p2"], cols], sig[d_["r1"], cols]
            want = x * z + y * (one - z)
        else:
            x, y, z = S0[d_["p1"], cols], sig[d_["r1"], cols], sig[d_["r2"], cols]
            want = x + np.float32(d_["ms"]) * (y - z)
        assert np.array_equal(S1[i, cols], want)
        row = S1[i].astype(np.float64)
        n_tr = d.X_train.shape[0]
        y32 = np.concatenate([d.y_train, d.y_test]).astype(np.float32).astype(np.float64)
        f = np.sqrt(np.mean((row[:n_tr] - y32[:n_tr]) ** 2))
        ft = np.sqrt(np.mean((row[n_tr:] - y32[n_tr:]) ** 2))
        assert abs(run["F1"][i] - f) <= 1e-5 * f
        assert abs(run["Ft1"][i] - ft) <= 1e-5 * ft


def test_elitism_invariants(run):
    best = run["stats"]["best_train_rmse"]
    assert np.all(np.diff(best) <= 0)
    assert run["stats"]["best_index"].min() >= 0
