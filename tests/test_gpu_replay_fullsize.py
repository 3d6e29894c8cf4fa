"""Oracle replay parity at the benchmark's full sizes (Algorithm 1's loop
body, generation by generation).

The device runs freely, one generation at a time, in the launch shape the
benchmark uses.  The FP64 CPU oracle follows the device's lineage in replay
mode: it takes each generation's variation draws and survival decision from
the device, computes the offspring semantics and fitness itself from the
same seeded data, and checks every draw against its own (operator, pool rows
and step equal; tournament winners and survival decisions equal except at
near ties, whose relative fitness gap is bounded and reported).

  - single_fp32_100k data (100,000 / 25,000 cases, 20 features, m = r =
    1,024) at FP64: 10 generations, every semantic element of every
    individual within 1e-6 * max(|oracle|, RMS(t)) and every fitness within
    1e-6 relative;
  - the same data in FP32 and FP32-Kahan: 20 generations, every fitness
    within 1e-4 relative of the oracle's FP64 value along the device lineage
    (the drift bar of the FP32 forms);
  - large_fp32_1m (1,000,000 / 250,000 cases, 64 features, m = r = 2,048,
    FP32): 20 generations on the device at full size; the oracle (61 GB in
    FP64 for every case) follows the lineage on a fixed slice of the cases
    (the first 1/8 of the train and of the test cases): the slice RMSE of
    every individual within 1e-4 relative, and every element of the slice
    within 1e-4 * max(E, RMS(t)), E the running error scale of FP32 storage
    along the lineage (see _Envelope);
  - precision_1m (large_fp32_1m data, m = r = 1,024): the FP64 replay of an
    FP32-Kahan lineage, which the precision benchmark uses as its drift
    reference, against the oracle for the first 50 generations on a 1/16
    case slice: elements within 1e-6 * max(|oracle|, RMS(t)), slice RMSE
    within 1e-6 relative.

Each test prints the replay check's counts (near ties the device and the
oracle decided differently, and the largest gap behind one).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2106_04034_amd import gsgp, synth
from tests.gpu_helpers import elite_of, oracle_config, oracle_records

pytestmark = pytest.mark.gpu


class _Lineage:
    """The device's lineage as the oracle's replay input, produced lazily:
    asking for generation g's draws runs generation g on the device (its
    draws were made at the end of generation g - 1 under the device's own
    fitness), so that the oracle's per-generation hook sees the device at the
    same generation."""

    def __init__(self, R, run=0):
        self.R, self.run = R, run
        self.records = _Seq(self._records)
        self.elite = _Seq(self._elite)

    def _records(self, i):
        self.R.generation(1, stats=False)
        assert self.R.current_generation() == i + 1
        return oracle_records(self.R.records(self.run, i + 1, 1)[0])

    def _elite(self, i):
        return elite_of(self.R.stats(self.run, i + 1, 1))[0]

    def pair(self):
        return (self.records, self.elite)


class _Seq:
    def __init__(self, fn):
        self.fn = fn

    def __getitem__(self, i):
        return self.fn(i)


def _settings(wl, precision, seed, G):
    return gsgp.Settings(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                         n_generations_max=G, tournament_size=wl.tournament_size,
                         p_crossover=wl.p_crossover, mutation_step=wl.mutation_step,
                         precision=precision, seed=seed)


def _rel(a, b, floor):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


def _report(name, res):
    w = sum(c["winner_mismatch"] for c in res.replay)
    e = sum(c["elite_mismatch"] for c in res.replay)
    gap = max([c["winner_gap_max"] for c in res.replay] + [c["elite_gap"] for c in res.replay] + [0.0])
    print(f"{name}: {len(res.replay)} generations replayed, tournament near-tie disagreements {w}, "
          f"survival near-tie disagreements {e}, largest gap {gap:.3e}", flush=True)
    assert all(c["draw_mismatch"] == 0 for c in res.replay)
    return gap


@pytest.mark.timeout(900)
def test_single_fp32_100k_data_at_fp64_replays_on_the_oracle():
    wl = synth.WORKLOADS["single_fp32_100k"]
    d = synth.single_run(wl.n_train, wl.n_test, wl.n_features)
    G = 10
    s = _settings(wl, gsgp.FP64, synth.evolution_seed(1), G)
    R = gsgp.Runner(s, [d])
    R.set_launch(4, 4, 1, 0)
    R.eval_population()
    floor = float(np.sqrt(np.mean(d.y_train ** 2)))
    worst = {"sem": 0.0, "fit": 0.0}

    def check(g, S_tr, S_te, F, Ft):
        S = R.semantics(0, 0)
        n_tr = S_tr.shape[1]
        worst["sem"] = max(worst["sem"], _rel(S[:, :n_tr], S_tr, floor), _rel(S[:, n_tr:], S_te, floor))
        Fd, Ftd = R.fitness(0)
        worst["fit"] = max(worst["fit"], _rel(Fd, F, 1e-300), _rel(Ftd, Ft, 1e-300))
        assert worst["sem"] <= 1e-6 and worst["fit"] <= 1e-6, (g, worst)
        del S

    cfg = oracle_config(s)
    res = orc.run(cfg, d.X_train, d.y_train, d.X_test, d.y_test, G, drive=_Lineage(R).pair(), on_generation=check)
    gap = _report("single_fp32_100k FP64", res)
    # FP64 fitness agrees to ~1e-13: a disagreement can only be an exact-looking tie
    assert gap <= 1e-9
    print(f"single_fp32_100k FP64: worst semantic error {worst['sem']:.3e}, fitness {worst['fit']:.3e}")
    R.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [gsgp.FP32, gsgp.FP32_KAHAN])
def test_single_fp32_100k_fp32_forms_drift_against_the_oracle(precision):
    wl = synth.WORKLOADS["single_fp32_100k"]
    d = synth.single_run(wl.n_train, wl.n_test, wl.n_features)
    G = 20
    s = _settings(wl, precision, synth.evolution_seed(1), G)
    R = gsgp.Runner(s, [d])
    R.set_launch(4, 4, 1, 0)
    R.eval_population()
    floor = float(np.sqrt(np.mean(d.y_train ** 2)))
    drift = []

    def check(g, S_tr, S_te, F, Ft):
        Fd, Ftd = R.fitness(0)
        drift.append(max(_rel(Fd, F, 1e-300), _rel(Ftd, Ft, 1e-300)))
        assert drift[-1] <= 1e-4, (g, drift[-1])
        if g in (0, G // 2, G):
            S = R.semantics(0, 0)
            n_tr = S_tr.shape[1]
            assert _rel(S[:, :n_tr], S_tr, floor) <= 1e-4 and _rel(S[:, n_tr:], S_te, floor) <= 1e-4, g

    res = orc.run(oracle_config(s), d.X_train, d.y_train, d.X_test, d.y_test, G, drive=_Lineage(R).pair(),
                  on_generation=check)
    gap = _report(f"single_fp32_100k precision {precision}", res)
    assert gap <= 1e-5  # near ties only, at the FP32 forms' fitness resolution
    print(f"precision {precision}: fitness drift per generation {['%.1e' % x for x in drift]}")
    R.close()


def _slice(d, frac):
    ntr, nte = d.X_train.shape[0] // frac, d.X_test.shape[0] // frac
    return ntr, nte, (d.X_train[:ntr], d.y_train[:ntr], d.X_test[:nte], d.y_test[:nte])


class _Envelope:
    """Running error scale of FP32 storage along a lineage (the standard
    running error bound, Higham, Accuracy and Stability of Numerical
    Algorithms, ch. 3): every operator evaluated on magnitudes,
      generation 0:  E = |S|
      mutation:      E_O = E[p1] + ms * (sR[r1] + sR[r2])
      crossover:     E_O = E[p1] * sR[r1] + E[p2] * (1 - sR[r1])
                           + sR[r1] * (E[p1] + E[p2])
      elite copy:    E_O[dst] = E[src]
    (sR in (0, 1)).  The crossover's last term is the FP32 rounding of the
    stored sR itself, which moves the result by (S[p1] - S[p2]) times that
    rounding: with sR = 1 - 2e-8 stored as exactly 1.0, S[p2] (1 - sR) drops
    out whatever the size of S[p2].  A value formed in FP32 from
    FP32-stored operands, g generations deep, differs from the exact one by
    at most about 6 g u E (u = 2^-24: rounding of each stored operand, of
    the products and of the sums), however much the operands cancel; the
    parity bar is then tol * max(E, RMS(t)).  The oracle's own pool
    semantics on the case slice give sR; the lineage is the device's, as in
    the replay."""

    def __init__(self, R, sig_tr, sig_te):
        self.R, self.sig = R, (sig_tr.astype(np.float32), sig_te.astype(np.float32))
        self.E = None

    def step(self, g, S_tr, S_te):
        if g == 0:
            self.E = [np.abs(S_tr).astype(np.float32), np.abs(S_te).astype(np.float32)]
            return self.E
        rec = self.R.records(0, g, 1)[0]
        st = self.R.stats(0, g, 1)[0]
        xo = rec["op"] == 1
        ms = rec["ms"].astype(np.float32)[:, None]
        out = []
        for E, sig in zip(self.E, self.sig):
            s1 = sig[rec["r1"]]
            E1, E2 = E[rec["p1"]], E[np.where(xo, rec["p2"], 0)]
            O = np.where(xo[:, None], E1 * s1 + E2 * (1 - s1) + s1 * (E1 + E2),
                         E1 + ms * (s1 + sig[np.where(xo, 0, rec["r2"])]))
            if st["elite_copied"]:
                O[st["elite_dst"]] = E[st["elite_src"]]
            out.append(O)
        self.E = out
        return out


def _slice_check(R, d, ntr, nte, tol, worst, envelope=None):
    """Compares the device's population on the case slice with the oracle's.
    Element errors are relative to max(|oracle|, RMS(t)), or with an
    envelope (FP32 storage) to max(E, RMS(t)) with E the running error scale
    of _Envelope: a crossover of two large rows that nearly cancel at a case
    keeps the FP32 rounding of its operands, however small the result
    there."""
    n_train = d.X_train.shape[0]
    floor = float(np.sqrt(np.mean(d.y_train[:ntr] ** 2)))

    def check(g, S_tr, S_te, F, Ft):
        A = R.semantics_cases(0, 0, 0, ntr)
        B = R.semantics_cases(0, 0, n_train, nte)
        if envelope is not None:
            E_tr, E_te = envelope.step(g, S_tr, S_te)
            sc_tr, sc_te = np.maximum(E_tr, floor), np.maximum(E_te, floor)
        else:
            sc_tr, sc_te = np.maximum(np.abs(S_tr), floor), np.maximum(np.abs(S_te), floor)
        worst["sem"] = max(worst["sem"], float(np.max(np.abs(A - S_tr) / sc_tr)),
                           float(np.max(np.abs(B - S_te) / sc_te)))
        f_tr = np.sqrt(np.mean((A - d.y_train[:ntr]) ** 2, axis=1))
        f_te = np.sqrt(np.mean((B - d.y_test[:nte]) ** 2, axis=1))
        worst["fit"] = max(worst["fit"], _rel(f_tr, F, 1e-300), _rel(f_te, Ft, 1e-300))
        assert worst["sem"] <= tol and worst["fit"] <= tol, (g, worst)

    return check


@pytest.mark.timeout(900)
def test_large_fp32_1m_drift_on_a_case_slice():
    wl = synth.WORKLOADS["large_fp32_1m"]
    d = synth.large_run(wl.n_train, wl.n_test, wl.n_features)
    G = 20
    s = _settings(wl, gsgp.FP32, synth.evolution_seed(2), G)
    R = gsgp.Runner(s, [d])
    R.set_launch(2, 2, 1, 0)
    R.eval_population()
    ntr, nte, data = _slice(d, 8)
    worst = {"sem": 0.0, "fit": 0.0}
    cfg = oracle_config(s)
    cr, vr = orc.genomes(cfg, wl.n_features, orc.TAG_POOL, s.pool_size)
    env = _Envelope(R, orc.sigmoid(orc.interpret(cr, vr, data[0])), orc.sigmoid(orc.interpret(cr, vr, data[2])))
    res = orc.run(cfg, *data, G, drive=_Lineage(R).pair(),
                  on_generation=_slice_check(R, d, ntr, nte, 1e-4, worst, envelope=env))
    # the oracle's own decisions use the slice's fitness, so its replay check
    # is informative only: the draws themselves must still match
    assert all(c["draw_mismatch"] == 0 for c in res.replay)
    print(f"large_fp32_1m FP32 on cases 1/8: worst semantic error {worst['sem']:.3e}, slice RMSE {worst['fit']:.3e}")
    R.close()


@pytest.mark.timeout(900)
def test_precision_1m_fp64_replay_matches_the_oracle_for_50_generations():
    wl = synth.WORKLOADS["precision_1m"]
    d = synth.large_run()
    G = 50
    seed = synth.evolution_seed(3)
    K = gsgp.Runner(_settings(wl, gsgp.FP32_KAHAN, seed, G), [d])
    K.eval_population()
    K.generation(G, stats=False)
    rec, elite = K.records(0, 1, G), K.stats(0, 1, G)
    K.close()
    s64 = _settings(wl, gsgp.FP64, seed, G)
    R = gsgp.Runner(s64, [d])
    R.eval_population()

    class _Replay(_Lineage):
        def _records(self, i):
            self.R.replay(rec[i:i + 1], elite[i:i + 1], stats=False)
            return oracle_records(rec[i])

        def _elite(self, i):
            return elite_of(elite[i:i + 1])[0]

    ntr, nte, data = _slice(d, 16)
    worst = {"sem": 0.0, "fit": 0.0}
    res = orc.run(oracle_config(s64), *data, G, drive=_Replay(R).pair(),
                  on_generation=_slice_check(R, d, ntr, nte, 1e-6, worst))
    assert all(c["draw_mismatch"] == 0 for c in res.replay)
    print(f"precision_1m FP64 replay on cases 1/16: worst semantic error {worst['sem']:.3e}, "
          f"slice RMSE {worst['fit']:.3e}")
    R.close()


def _oracle_lineage(R, s, d, G):
    """An oracle Result holding the oracle's own genomes (drawn from the same
    Philox stream) and the device's lineage, for reconstruction."""
    cfg = oracle_config(s)
    l = d.X_train.shape[1]
    cp, vp = orc.genomes(cfg, l, orc.TAG_POPULATION, s.pop_size)
    cr, vr = orc.genomes(cfg, l, orc.TAG_POOL, s.pool_size)
    res = orc.Result(np.concatenate([cp, cr]), np.concatenate([vp, vr]), None, None, None, None, None, None,
                     oracle_records(R.records(0, 1, G)), elite_of(R.stats(0, 1, G)))
    res.scale = np.zeros((G + 1, s.pop_size, 2))
    res.scale[:, :, 1] = 1.0
    return cfg, res


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [gsgp.FP64, gsgp.FP32])
def test_reconstruct_the_best_of_200_generations_on_unseen_cases(precision):
    """Model export at scale (Algorithm 1, "Return: best individual"; the
    lineage structures of Section 2.1): after 200 generations of the
    single_fp32_100k workload the best individual is rebuilt from its
    ancestry record on 10,000 unseen cases and equals the oracle's
    reconstruction along the same lineage (reconstruction is FP64 in every
    form); rebuilt on the training cases it equals the stored semantics (FP64)
    or their FP32 storage within the drift bar."""
    import time
    wl = synth.WORKLOADS["single_fp32_100k"]
    d = synth.single_run(wl.n_train, wl.n_test, wl.n_features)
    G = 200
    s = _settings(wl, precision, synth.evolution_seed(1), G)
    R = gsgp.Runner(s, [d])
    R.set_launch(4, 4, 1, 0)
    R.eval_population()
    R.generation(G, stats=False)
    best = int(R.stats(0, G, 1)[0]["best_index"])
    Xnew = np.random.default_rng(200).uniform(-1.0, 1.0, size=(10_000, wl.n_features))
    t0 = time.perf_counter()
    got = R.reconstruct(0, G, best, Xnew)
    t_rec = time.perf_counter() - t0
    cfg, res = _oracle_lineage(R, s, d, G)
    t0 = time.perf_counter()
    want = orc.reconstruct(res, cfg, G, best, Xnew)
    t_orc = time.perf_counter() - t0
    err = _rel(got, want, 1.0)
    assert err <= 1e-12, err
    on_train = R.reconstruct(0, G, best, d.X_train)
    stored = R.semantics_rows(0, 0, best, 1)[0, :wl.n_train]
    floor = float(np.sqrt(np.mean(d.y_train ** 2)))
    assert _rel(on_train, stored, floor) <= (1e-12 if precision == gsgp.FP64 else 1e-4)
    import ctypes
    size = ctypes.c_size_t(0)
    gsgp.check(gsgp.lib().gsgp_reconstruct_scratch_size(R._h, 0, G, best, 10_000, ctypes.byref(size)), "size")
    print(f"reconstruct precision {precision}: best of {G} generations on 10,000 cases in {t_rec * 1e3:.1f} ms "
          f"(scratch {size.value / 2**20:.1f} MiB), oracle {t_orc:.1f} s, relative error {err:.2e}")
    R.close()


@pytest.mark.timeout(900)
def test_export_linear_of_the_paper_loop_at_scale():
    """The paper's own loop (every individual mutated once per generation,
    random step) on the single_fp32_100k data with m = r = 1,024 for 200
    generations: the compact model of sampled individuals equals the
    oracle's along the same lineage bit for bit, and evaluating it on unseen
    cases reproduces the device's lineage reconstruction."""
    wl = synth.WORKLOADS["single_fp32_100k"]
    d = synth.single_run(wl.n_train, wl.n_test, wl.n_features)
    G = 200
    s = _settings(wl, gsgp.FP32, synth.evolution_seed(1), G)
    s.tournament_size, s.p_crossover, s.ms_random = 0, 0.0, 1
    R = gsgp.Runner(s, [d])
    R.eval_population()
    R.generation(G, stats=False)
    cfg, res = _oracle_lineage(R, s, d, G)
    m = s.pop_size
    Xnew = np.random.default_rng(201).uniform(-1.0, 1.0, size=(2_000, wl.n_features))
    sig = orc.sigmoid(orc.interpret(res.code[m:], res.cval[m:], Xnew))
    best = int(R.stats(0, G, 1)[0]["best_index"])
    for i in sorted({best, 0, 517, m - 1}):
        tree, c, b, w = R.export_linear(0, G, i)
        otree, oc, ob, ow = orc.export_linear(res, cfg, G, i)
        assert tree == otree and np.array_equal(w, ow) and (c, b) == (oc, ob) == (0.0, 1.0), i
        val = orc.interpret(res.code[tree:tree + 1], res.cval[tree:tree + 1], Xnew)[0] + w @ sig
        rec = R.reconstruct(0, G, i, Xnew)
        assert np.allclose(val, rec, rtol=1e-12, atol=1e-12 * np.max(np.abs(rec))), i
    R.close()
