"""Parity at the benchmark's full sizes, in the launch shapes the benchmark
uses, on sampled outputs the oracle computes one by one and on properties
that hold at any size:
  - single_fp32_100k: 100,000 / 25,000 cases, 20 features, m = r = 1,024,
    FP32, launch 4 waves x 4 offspring, XCD-contiguous order;
  - large_fp32_1m: 1,000,000 / 250,000 cases, 64 features, m = r = 2,048,
    FP32, launch 2 x 2, XCD-contiguous order;
  - batched_256: 256 runs of uneven size in one handle, FP32-Kahan, launch
    4 x 8, XCD side-by-side order; three runs are checked (the largest, the
    smallest and a middle one);
  - paper_shape_k127 (Section 3.1 shape): 102,400 cases, 1,024 features,
    m = r = 10,240, the mutate-all loop with a random step, FP32, launch
    4 x 4, hardware round-robin order.

Bars:
  - genomes: bit-exact (integer draws, constants from the same FP64 ops);
  - population semantics: the FP32 rounding of the oracle's FP64 value,
    bit-exact (the interpreter is bit-exact in FP64 and rounds once);
    pool: within 1 FP32 ulp (exp rounding may cross a rounding boundary);
  - generation-0 fitness of sampled individuals: 1e-4 relative (the FP32
    forms' bar; storage rounding of S and t, FP32 chunk sums);
  - generation-1 draws: equal to the draws an independent Philox twin makes
    on the host from the device's generation-0 fitness (operator, pool rows,
    step, and tournament winners: first strict minimum in draw order);
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

G_TEST = 4
FLT_MAX = np.float32(3.4028234663852886e38)


def _host_record(s, run_id, i, F):
    """Generation-1 draws of offspring i (same reading as the kernels and
    the oracle: W0 operator, W1/W2 pool rows, W3/W4 step, then tournaments)."""
    ts = s.tournament_size
    m, r = s.pop_size, s.pool_size
    W = pyphilox.words(i, 1, 5 + 2 * max(ts, 1), s.seed, run_id)

    def winner(ws):
        best = pyphilox.below(ws[0], m)
        for w in ws[1:]:
            c = pyphilox.below(w, m)
            if F[c] < F[best]:
                best = c
        return best

    xo = ts > 0 and W[0] < pyphilox.threshold(s.p_crossover)
    if xo:
        return dict(op=1, p1=winner(W[5:5 + ts]), p2=winner(W[5 + ts:5 + 2 * ts]), r1=pyphilox.below(W[1], r))
    ms = s.mutation_step * pyphilox.u53(W[3], W[4]) if s.ms_random else s.mutation_step
    return dict(op=0, p1=winner(W[5:5 + ts]) if ts > 0 else i, r1=pyphilox.below(W[1], r),
                r2=pyphilox.below(W[2], r), ms=ms)


def _row(R, run, which, i):
    return R.semantics_rows(run, which, int(i), 1)[0].astype(np.float32)


def _check_run(R, run, s, d, rng, n_offspring):
    """Every check on one run of a handle that has just been evaluated (at
    generation 0); leaves the handle G_TEST generations further on."""
    m, r = s.pop_size, s.pool_size
    ocfg = oracle_config(s, run_id=run)
    l = d.X_train.shape[1]
    X = np.concatenate([d.X_train, d.X_test])
    n_all = X.shape[0]
    n_tr = d.X_train.shape[0]
    # genomes
    codes, consts = R.genomes(run)
    cp, vp = orc.genomes(ocfg, l, orc.TAG_POPULATION, m)
    cr, vr = orc.genomes(ocfg, l, orc.TAG_POOL, r)
    assert np.array_equal(codes, np.concatenate([cp, cr]))
    assert np.array_equal(consts, np.concatenate([vp, vr]))
    # semantics of sampled rows on sampled cases
    cases = np.sort(rng.choice(n_all, size=min(1500, n_all), replace=False))
    cases[0], cases[-1] = 0, n_all - 1
    w0 = int(rng.integers(0, max(1, m - 12)))
    pop = np.arange(w0, min(m, w0 + 12))
    S0w = R.semantics_rows(run, 0, int(pop[0]), len(pop)).astype(np.float32)
    want = orc.interpret(codes[pop], consts[pop], X[cases]).astype(np.float32)
    assert np.array_equal(S0w[:, cases], want)
    p0 = int(rng.integers(0, max(1, r - 12)))
    pool = np.arange(p0, min(r, p0 + 12))
    sigw = R.semantics_rows(run, 1, int(pool[0]), len(pool)).astype(np.float32)
    want_p = orc.sigmoid(orc.interpret(codes[m + pool], consts[m + pool], X[cases])).astype(np.float32)
    ulp = np.spacing(np.abs(want_p).astype(np.float32))
    assert np.all(np.abs(sigw[:, cases] - want_p) <= ulp)
    # generation-0 fitness of sampled individuals, on every case
    F0, Ft0 = R.fitness(run)
    idx = rng.choice(m, size=min(4, m), replace=False)
    St = orc.interpret(codes[idx], consts[idx], d.X_train)
    assert np.all(np.abs(F0[idx] - orc.rmse_rows(St, d.y_train)) <= 1e-4 * orc.rmse_rows(St, d.y_train))
    if d.X_test.shape[0]:
        Se = orc.interpret(codes[idx], consts[idx], d.X_test)
        assert np.all(np.abs(Ft0[idx] - orc.rmse_rows(Se, d.y_test)) <= 1e-4 * orc.rmse_rows(Se, d.y_test))
    # generation 1: host twin of the draws, operands fetched before the step
    offs = rng.choice(m, size=min(n_offspring, m), replace=False)
    plan = {int(i): _host_record(s, run, int(i), F0) for i in offs}
    rows = {}
    best0 = int(np.argmin(F0))  # the elite, should survival keep it
    rows[(0, best0)] = _row(R, run, 0, best0)
    for i, rc in plan.items():
        for key, which in (("p1", 0), ("p2", 0), ("r1", 1), ("r2", 1)):
            if key in rc and (which, rc[key]) not in rows:
                rows[(which, rc[key])] = _row(R, run, which, rc[key])
    R.generation(1)
    rec1 = R.records(run, 1, 1)[0]
    st1 = R.stats(run, 1, 1)[0]
    F1, Ft1 = R.fitness(run)
    y32 = np.concatenate([d.y_train, d.y_test]).astype(np.float32).astype(np.float64)
    one = np.float32(1.0)
    for i, rc in plan.items():
        got = rec1[i]
        assert got["op"] == rc["op"] and got["p1"] == rc["p1"] and got["r1"] == rc["r1"], (run, i)
        O = _row(R, run, 0, i)
        if st1["elite_copied"] and i == st1["elite_dst"]:
            continue  # checked below against its source
        if rc["op"] == 1:
            assert got["p2"] == rc["p2"]
            x, y, z = rows[(0, rc["p1"])], rows[(0, rc["p2"])], rows[(1, rc["r1"])]
            want_o = x * z + y * (one - z)
        else:
            assert got["r2"] == rc["r2"] and got["ms"] == rc["ms"]
            x, y, z = rows[(0, rc["p1"])], rows[(1, rc["r1"])], rows[(1, rc["r2"])]
            want_o = x + np.float32(rc["ms"]) * (y - z)
        want_o = np.minimum(np.maximum(want_o, -FLT_MAX), FLT_MAX)
        assert np.array_equal(O, want_o), (run, i)
        row = O.astype(np.float64)
        f = np.sqrt(np.mean((row[:n_tr] - y32[:n_tr]) ** 2))
        assert abs(F1[i] - f) <= 1e-5 * f, (run, i)
        if n_all > n_tr:
            ft = np.sqrt(np.mean((row[n_tr:] - y32[n_tr:]) ** 2))
            assert abs(Ft1[i] - ft) <= 1e-5 * ft, (run, i)
    if st1["elite_copied"]:
        assert st1["elite_src"] == best0
        assert F1[st1["elite_dst"]] == F0[best0]
        assert np.array_equal(_row(R, run, 0, st1["elite_dst"]), rows[(0, best0)])
    # a few more generations: elitism keeps the best train RMSE monotone
    R.generation(G_TEST - 1)
    best = R.stats(run, 0, G_TEST + 1)["best_train_rmse"]
    assert np.all(np.diff(best) <= 0)
    assert R.stats(run, 0, G_TEST + 1)["best_index"].min() >= 0


def _settings(wl, precision, seed):
    return gsgp.Settings(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                         n_generations_max=G_TEST, tournament_size=wl.tournament_size,
                         p_crossover=wl.p_crossover, mutation_step=wl.mutation_step,
                         precision=precision, seed=seed)


@pytest.mark.parametrize("name,make,seed_index,launch,n_off", [
    ("single_fp32_100k", synth.single_run, 1, (4, 4, 1, 0), 40),
    ("large_fp32_1m", synth.large_run, 2, (2, 2, 1, 0), 12),
])
def test_single_run_full_size(name, make, seed_index, launch, n_off):
    wl = synth.WORKLOADS[name]
    d = make(wl.n_train, wl.n_test, wl.n_features)
    s = _settings(wl, gsgp.FP32, synth.evolution_seed(seed_index))
    R = gsgp.Runner(s, [d])
    R.set_launch(*launch)
    R.eval_population()
    _check_run(R, 0, s, d, np.random.default_rng(seed_index), n_off)
    R.close()


def test_batched_full_size():
    wl = synth.WORKLOADS["batched_256"]
    datasets = synth.batched_runs(wl.runs)
    s = _settings(wl, gsgp.FP32_KAHAN, synth.evolution_seed(4))
    R = gsgp.Runner(s, datasets)
    R.set_launch(4, 8, 2, 0)
    sizes = np.array([dd.X_train.shape[0] for dd in datasets])
    order = np.argsort(sizes)
    picks = [int(order[-1]), int(order[0]), int(order[len(order) // 2])]
    for j in picks:
        # each check advances every run of the handle, so restart for each
        R.eval_population()
        _check_run(R, j, s, datasets[j], np.random.default_rng(100 + j), 16)
    R.close()


def test_paper_shape_full_size():
    wl = synth.WORKLOADS["paper_shape_k127"]
    d = synth.paper_shape(wl.n_train, wl.n_features)
    s = _settings(wl, gsgp.FP32, synth.evolution_seed(5))
    s.ms_random = 1
    R = gsgp.Runner(s, [d])
    R.set_launch(4, 4, 0, 0)
    R.eval_population()
    _check_run(R, 0, s, d, np.random.default_rng(5), 24)
    R.close()
