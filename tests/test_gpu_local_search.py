"""GSGP with local search on the GPU against the FP64 oracle.

Local search is named by the paper (Sections 3.2 and 5) without a
definition; the reading both sides implement is the least-squares scaling
alpha + beta * O of every variation offspring, fitted on the training cases
and applied to the offspring's test cases too (oracle: orc_ls_fit, two-pass
regression; device: closed form from FP64 chunk sums of o, o^2 and o * t,
with the parents' scaling applied as the variation kernel reads them).

Bars:
  - FP64 free runs: records, survival decisions and best index equal the
    oracle's in every generation; semantics within 1e-9 * max(|b|, RMS(t)),
    fitness within 1e-9 relative, scaling coefficients within 1e-9 (the two
    sides sum in different orders and the device's train RMSE comes from the
    closed form, whose cancellation costs a few digits of the FP64 rounding);
  - FP32 forms driven along their own lineage by the oracle in replay mode:
    fitness within 1e-4 relative in every generation;
  - batched runs byte-identical to the same run alone; graph, no graph and
    launch shapes change no bit; checkpoints resume bit for bit;
  - reconstruction and export of the device lineage equal the oracle's along
    the same lineage and scaling.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2106_04034_amd import gsgp, synth
from tests.gpu_helpers import dataset, elite_of, oracle_config, oracle_records, records_equal, rel_err

pytestmark = pytest.mark.gpu


def _ls_settings(**kw):
    base = dict(pop_size=32, pool_size=16, n_generations_max=8, seed=11, flags=gsgp.FLAG_LOCAL_SEARCH)
    base.update(kw)
    return gsgp.Settings(**base)


def _ocfg(s, run_id=0):
    c = oracle_config(s, run_id)
    c.local_search = True
    return c


def _free_run_ls(s, d, G, tol=1e-9):
    R = gsgp.Runner(s, [d])
    res = orc.run(_ocfg(s), d.X_train, d.y_train, d.X_test, d.y_test, G, keep_semantics=True)
    R.eval_population()
    floor = float(np.sqrt(np.mean(d.y_train ** 2)))
    n_tr = d.X_train.shape[0]
    for g in range(G + 1):
        if g > 0:
            st = R.generation(1)[0, 0]
            ost = res.stats[g]
            assert (st["elite_copied"], st["elite_src"], st["elite_dst"]) == (
                ost["elite_copied"], ost["elite_src"], ost["elite_dst"]), g
            assert st["best_index"] == ost["best_index"], g
            assert records_equal(R.records(0, g, 1)[0], res.records[g - 1]), g
        S = R.semantics(0, 0)
        assert rel_err(S[:, :n_tr], res.S_hist[g][0], floor) <= tol, g
        if d.X_test.shape[0]:
            assert rel_err(S[:, n_tr:], res.S_hist[g][1], floor) <= tol, g
        F, Ft = R.fitness(0)
        assert rel_err(F, res.F_hist[g], 1e-300) <= tol, (g, rel_err(F, res.F_hist[g], 1e-300))
        if d.X_test.shape[0]:
            assert rel_err(Ft, res.Ft_hist[g], 1e-300) <= tol, g
        sc = R.scaling(0, g, 1)[0]
        assert np.all(np.abs(sc - res.scale[g]) <= tol * np.maximum(1.0, np.abs(res.scale[g]))), g
    best = R.stats(0, 0, G + 1)["best_train_rmse"]
    assert np.all(np.diff(best) <= 0)
    R.close()
    return res


def test_local_search_plain_fp64_500x8_full_run():
    """The plain FP64 workload (500 / 200 cases, m = r = 128, 20
    generations) with local search: a free run in step with the oracle."""
    d = synth.plain_small()
    s = _ls_settings(pop_size=128, pool_size=128, n_generations_max=20, seed=synth.evolution_seed(0))
    res = _free_run_ls(s, d, 20)
    # the scaling is at work: most offspring are rescaled, and it helps
    assert np.mean(res.scale[1:, :, 1] != 1.0) > 0.5
    plain = orc.run(oracle_config(s), d.X_train, d.y_train, d.X_test, d.y_test, 20)
    assert res.stats[20]["best_train_rmse"] < plain.stats[20]["best_train_rmse"]


@pytest.mark.parametrize("variant", ["paper_mutate_all", "ragged_with_test", "ragged_no_test", "all_crossover"])
def test_local_search_variants(variant):
    """The paper's own loop (every individual mutated, random step), ragged
    sizes whose last chunk holds pads (the scaled parents must keep pads at
    zero), no test set, and crossover only."""
    G = 6
    if variant == "paper_mutate_all":
        d = dataset(300, 100, 4, seed=81)
        s = _ls_settings(tournament_size=0, p_crossover=0.0, ms_random=1, n_generations_max=G)
    elif variant == "ragged_with_test":
        d = dataset(1500, 77, 4, seed=82)
        s = _ls_settings(n_generations_max=G, seed=12)
    elif variant == "ragged_no_test":
        d = dataset(513, 0, 3, seed=83)
        s = _ls_settings(n_generations_max=G, seed=13)
    else:
        d = dataset(700, 150, 5, seed=84)
        s = _ls_settings(p_crossover=1.0, n_generations_max=G, seed=14)
    _free_run_ls(s, d, G)


class _Lineage:
    """Device lineage for the oracle's replay mode, one device generation per
    generation asked for."""

    def __init__(self, R):
        self.R = R

    def rec(self, i):
        self.R.generation(1, stats=False)
        return oracle_records(self.R.records(0, i + 1, 1)[0])

    def el(self, i):
        return elite_of(self.R.stats(0, i + 1, 1))[0]

    def pair(self):
        class Seq:
            def __init__(self, f):
                self.f = f

            def __getitem__(self, i):
                return self.f(i)
        return (Seq(self.rec), Seq(self.el))


@pytest.mark.parametrize("precision", [gsgp.FP32, gsgp.FP32_KAHAN])
def test_local_search_fp32_forms_against_the_oracle_replay(precision):
    d = dataset(4000, 1000, 6, seed=85)
    G = 30
    s = _ls_settings(pop_size=64, pool_size=64, n_generations_max=G, seed=21, precision=precision)
    R = gsgp.Runner(s, [d])
    R.eval_population()
    worst = []

    def check(g, S_tr, S_te, F, Ft):
        Fd, Ftd = R.fitness(0)
        worst.append(max(rel_err(Fd, F, 1e-300), rel_err(Ftd, Ft, 1e-300)))
        assert worst[-1] <= 1e-4, (g, worst[-1])

    res = orc.run(_ocfg(s), d.X_train, d.y_train, d.X_test, d.y_test, G, drive=_Lineage(R).pair(),
                  on_generation=check)
    assert all(c["draw_mismatch"] == 0 for c in res.replay)
    assert max(c["winner_gap_max"] for c in res.replay) <= 1e-5
    R.close()


def test_local_search_batched_graphs_and_shapes_keep_bits():
    ds = [dataset(n, n // 4, l, seed=n) for n, l in [(200, 4), (1700, 9), (4096, 5)]]
    for prec in (gsgp.FP64, gsgp.FP32_KAHAN):
        s = _ls_settings(n_generations_max=7, seed=99, precision=prec)
        B = gsgp.Runner(s, ds)
        B.set_launch(2, 6, 2, 0)
        B.eval_population()
        B.generation(7, stats=False)
        for flags, shape in ((gsgp.FLAG_LOCAL_SEARCH, (4, 4, 1, 0)),
                             (gsgp.FLAG_LOCAL_SEARCH | gsgp.FLAG_NO_GRAPH, (1, 1, 0, 37))):
            single = gsgp.Runner(dataclasses.replace(s, flags=flags), [ds[0]])
            single.set_launch(*shape)
            single.eval_population()
            single.generation(7, stats=False)
            assert np.array_equal(single.semantics(0, 0), B.semantics(0, 0))
            assert np.array_equal(single.fitness(0)[0], B.fitness(0)[0])
            assert np.array_equal(single.scaling(0, 0, 8), B.scaling(0, 0, 8))
            single.close()
        B.close()


def _lineage_result(R, s, G, codes, consts):
    res = orc.Result(codes, consts, None, None, None, None, None, None,
                     oracle_records(R.records(0, 1, G)), elite_of(R.stats(0, 1, G)))
    res.scale = R.scaling(0, 0, G + 1)
    return res


def test_local_search_reconstruct_and_export():
    """Reconstruction of device lineages with local search on new cases, and
    the compact model c + b T + sum_j w_j sigma(R_j) of the paper loop's
    lineages, equal the oracle's along the same lineage and scaling."""
    d = dataset(600, 200, 5, seed=86)
    G = 12
    s = _ls_settings(pop_size=40, pool_size=24, n_generations_max=G, seed=31)
    R = gsgp.Runner(s, [d])
    R.eval_population()
    R.generation(G, stats=False)
    codes, consts = R.genomes(0)
    res = _lineage_result(R, s, G, codes, consts)
    cfg = _ocfg(s)
    Xnew = np.random.default_rng(87).uniform(-1, 1, size=(333, 5))
    best = int(R.stats(0, G, 1)[0]["best_index"])
    for i in sorted({best, 0, 39}):
        assert rel_err(R.reconstruct(0, G, i, Xnew), orc.reconstruct(res, cfg, G, i, Xnew), 1.0) <= 1e-12, i
    # on the training cases the reconstruction is the individual's semantics
    S = R.semantics(0, 0)
    assert rel_err(R.reconstruct(0, G, best, d.X_train), S[best, :600], 1.0) <= 1e-12
    R.close()
    sp = _ls_settings(pop_size=24, pool_size=20, n_generations_max=G, seed=32, tournament_size=0, p_crossover=0.0,
                      ms_random=1)
    P = gsgp.Runner(sp, [d])
    P.eval_population()
    P.generation(G, stats=False)
    codes, consts = P.genomes(0)
    res = _lineage_result(P, sp, G, codes, consts)
    cfg = _ocfg(sp)
    sig = orc.sigmoid(orc.interpret(codes[24:], consts[24:], Xnew))
    for i in range(24):
        tree, c, b, w = P.export_linear(0, G, i)
        otree, oc, ob, ow = orc.export_linear(res, cfg, G, i)
        assert tree == otree and (c, b) == (oc, ob) and np.array_equal(w, ow), i
        val = c + b * orc.interpret(codes[tree:tree + 1], consts[tree:tree + 1], Xnew)[0] + w @ sig
        rec = P.reconstruct(0, G, i, Xnew)
        assert np.allclose(val, rec, rtol=1e-10, atol=1e-10 * np.max(np.abs(rec))), i
    P.close()


def test_local_search_checkpoint_resume():
    ds = [dataset(900, 150, 4, seed=88), dataset(130, 0, 3, seed=89)]
    s = _ls_settings(pop_size=36, pool_size=20, n_generations_max=12, seed=9, precision=gsgp.FP32_KAHAN)
    A = gsgp.Runner(s, ds)
    A.eval_population()
    A.generation(5)
    blob = A.checkpoint()
    A.generation(7)
    B = gsgp.Runner(s, ds)
    B.restore(blob)
    B.generation(7)
    for j in range(2):
        assert np.array_equal(A.semantics(j, 0), B.semantics(j, 0))
        assert np.array_equal(A.fitness(j)[0], B.fitness(j)[0])
        assert np.array_equal(A.scaling(j, 0, 13), B.scaling(j, 0, 13))
        assert np.array_equal(A.stats(j, 0, 13), B.stats(j, 0, 13))
    plain = gsgp.Runner(dataclasses.replace(s, flags=0), ds)
    with pytest.raises(gsgp.GSGPError) as e:
        plain.restore(blob)
    assert e.value.status == -1
    A.close()
    B.close()
    plain.close()
