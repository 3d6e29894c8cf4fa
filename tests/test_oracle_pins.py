"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: published
known answers, hand-worked values (tests/golden), closed forms, textbook
evaluation, brute force and distribution laws.  A plausible mistake (a wrong
sign, swapped operands, a dropped term, an off-by-one index) fails at least
one of them.  The paper is arXiv 2106.04034 (GSGP-CUDA); section references
are to it.
"""
import math
import os
import random

import numpy as np
import pytest

from tests import pyphilox
from tests.conftest import GOLDEN

FLT_MAX = 3.4028234663852886e38


# --------------------------------------------------------------------------
# Philox (counter-based generator that every random draw of the method uses)

def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[:4], v[4:6], tuple(v[6:10])))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, out in _kat():
        assert orc.philox(ctr, key) == out
        assert pyphilox.philox(ctr, key) == out


def test_philox_matches_python_twin(orc):
    rng = random.Random(7)
    for _ in range(2000):
        ctr = [rng.getrandbits(32) for _ in range(4)]
        key = [rng.getrandbits(32) for _ in range(2)]
        assert orc.philox(ctr, key) == pyphilox.philox(ctr, key)


def test_event_threshold(orc):
    assert orc.event_threshold(0.0) == 0
    assert orc.event_threshold(1.0) == 1 << 32
    assert orc.event_threshold(0.5) == 1 << 31
    assert orc.event_threshold(0.25) == 1 << 30
    assert orc.event_threshold(0.8) == 3435973836  # floor(0.8 * 2^32)


# --------------------------------------------------------------------------
# CreatePopulation (Section 2.2, "Initialization")

def test_genome_gene_types_and_values(orc):
    cfg = orc.Config(pop_size=64, genome_len=127, seed=11, run_id=3)
    l = 7
    code, cval = orc.genomes(cfg, l, orc.TAG_POPULATION, 64)
    key = (cfg.seed, cfg.run_id)
    tf = pyphilox.threshold(cfg.p_function)
    tfe = pyphilox.threshold(cfg.p_function + cfg.p_feature)
    for t in (0, 5, 63):
        for q in (0, 1, 50, 126):
            w = pyphilox.philox((q, t, 0, orc.TAG_POPULATION), key)
            if w[0] < tf:
                assert code[t, q] == -1 - (w[1] >> 30)
            elif w[0] < tfe:
                assert code[t, q] == pyphilox.below(w[1], l)
            else:
                assert code[t, q] == orc.GENE_CONST
                assert cval[t, q] == cfg.erc_lo + (cfg.erc_hi - cfg.erc_lo) * pyphilox.u53(w[2], w[3])


def test_genome_frequencies():
    """Gene-type, function and feature frequencies within 99.9 % binomial
    intervals over ~1e6 genes (probabilities 0.8 / 0.14 / remainder)."""
    from oracle import oracle as orc
    cfg = orc.Config(pop_size=8000, genome_len=127, seed=99)
    l = 10
    code, cval = orc.genomes(cfg, l, orc.TAG_POPULATION, 8000)
    n = code.size
    z = 3.29

    def within(count, p, total):
        sd = math.sqrt(total * p * (1 - p))
        return abs(count - total * p) <= z * sd

    func = code < 0
    func &= code != orc.GENE_CONST
    feat = code >= 0
    const = code == orc.GENE_CONST
    assert within(func.sum(), 0.80, n)
    assert within(feat.sum(), 0.14, n)
    assert within(const.sum(), 0.06, n)
    nf = int(func.sum())
    for f in (-1, -2, -3, -4):
        assert within(int((code == f).sum()), 0.25, nf)
    nfe = int(feat.sum())
    for f in range(l):
        assert within(int((code == f).sum()), 1.0 / l, nfe)
    v = cval[const]
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < z * math.sqrt(1 / 3.0 / v.size)
    assert np.all(cval[~const] == 0.0)


def test_genome_tags_and_runs_differ(orc):
    cfg = orc.Config(pop_size=16, seed=5, run_id=0)
    a, _ = orc.genomes(cfg, 4, orc.TAG_POPULATION, 16)
    b, _ = orc.genomes(cfg, 4, orc.TAG_POOL, 16)
    cfg.run_id = 1
    c, _ = orc.genomes(cfg, 4, orc.TAG_POPULATION, 16)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


# --------------------------------------------------------------------------
# Interpreter (Section 2.2, "Interpreter")

def _parse_program(tokens):
    code, cval = [], []
    for tok in tokens:
        if tok in "+-*/":
            code.append({"+": -1, "-": -2, "*": -3, "/": -4}[tok])
            cval.append(0.0)
        elif tok.startswith("x"):
            code.append(int(tok[1:]))
            cval.append(0.0)
        else:
            code.append(-5)
            cval.append(float(tok[2:]))
    return code, cval


def _golden_programs():
    out = []
    for line in open(os.path.join(GOLDEN, "interpreter_programs.txt")):
        if line.startswith("#") or not line.strip():
            continue
        exp, prog, what = (s.strip() for s in line.split("|", 2))
        out.append((float(exp), prog.split(), what))
    return out


def test_interpreter_hand_worked(orc):
    x = np.array([[0.5, -0.25, 2.0]])
    progs = _golden_programs()
    assert len(progs) >= 15
    k = max(len(p) for _, p, _ in progs)
    for exp, toks, what in progs:
        code, cval = _parse_program(toks)
        pad = k - len(code)
        # padding with skipped functions at the front keeps the value: a
        # function on an empty stack is skipped (also pins the skip rule)
        code = [-1] * pad + code
        cval = [0.0] * pad + cval
        got = orc.interpret(np.array([code], np.int32), np.array([cval]), x)[0, 0]
        assert got == exp, (what, got, exp)


def _pdiv(a, b):
    return 1.0 if abs(b) < 1e-6 else a / b


def _clamp(r):
    return FLT_MAX if r > FLT_MAX else (-FLT_MAX if r < -FLT_MAX else r)


def _infix(code, cval):
    """Textbook RPN-to-expression conversion (skips only when < 2 operands);
    returns a Python expression string of the last valid function."""
    stack, last = [], "0.0"
    for g, v in zip(code, cval):
        if g >= 0:
            stack.append(f"x[{g}]")
        elif g == -5:
            stack.append(repr(float(v)))
        elif len(stack) >= 2:
            b = stack.pop()
            a = stack.pop()
            expr = {-1: f"C({a} + {b})", -2: f"C({a} - {b})", -3: f"C({a} * {b})",
                    -4: f"C(D({a}, {b}))"}[g]
            stack.append(expr)
            last = expr
    return last


def test_interpreter_random_programs_vs_infix(orc):
    rng = random.Random(3)
    l = 5
    X = np.random.default_rng(1).uniform(-2, 2, size=(40, l))
    X[0, :] = 0.0  # exercises protected division
    for _ in range(60):
        k = rng.randint(1, 40)
        code, cval = [], []
        for _ in range(k):
            u = rng.random()
            if u < 0.5:
                code.append(-rng.randint(1, 4))
                cval.append(0.0)
            elif u < 0.85:
                code.append(rng.randrange(l))
                cval.append(0.0)
            else:
                code.append(-5)
                cval.append(rng.uniform(-3, 3))
        expr = _infix(code, cval)
        got = orc.interpret(np.array([code], np.int32), np.array([cval]), X)[0]
        for c in range(X.shape[0]):
            want = eval(expr, {"x": list(X[c]), "C": _clamp, "D": _pdiv})
            assert got[c] == want


def test_interpreter_rows_independent(orc):
    cfg = orc.Config(pop_size=6, seed=4)
    code, cval = orc.genomes(cfg, 3, orc.TAG_POPULATION, 6)
    X = np.random.default_rng(2).uniform(-1, 1, size=(9, 3))
    full = orc.interpret(code, cval, X)
    for t in range(6):
        assert np.array_equal(orc.interpret(code[t:t + 1], cval[t:t + 1], X)[0], full[t])
    for c in range(9):
        assert np.array_equal(orc.interpret(code, cval, X[c:c + 1])[:, 0], full[:, c])


def test_interpreter_finite_on_random_genomes(orc):
    cfg = orc.Config(pop_size=300, seed=8)
    code, cval = orc.genomes(cfg, 4, orc.TAG_POPULATION, 300)
    X = np.random.default_rng(5).uniform(-1, 1, size=(50, 4))
    S = orc.interpret(code, cval, X)
    assert np.all(np.isfinite(S)) and np.all(np.abs(S) <= FLT_MAX)


# --------------------------------------------------------------------------
# Logistic squashing of random trees and RMSE fitness (Section 2, 2.2)

def test_sigmoid_closed_forms(orc):
    x = np.array([0.0, -800.0, 800.0, 1.0, -1.0, 3.5, -20.0, 1e-9])
    s = orc.sigmoid(x)
    assert s[0] == 0.5 and s[1] == 0.0 and s[2] == 1.0
    with np.errstate(over="ignore"):
        ref = 1.0 / (1.0 + np.exp(-x))
    assert np.all(np.abs(s - ref) <= 2 * np.spacing(np.abs(ref)))
    assert abs(s[3] + s[4] - 1.0) <= 2 ** -52
    assert abs(s[3] - 1 / (1 + math.e ** -1)) <= 2 ** -52
    assert abs(orc.sigmoid(np.array([math.log(3.0)]))[0] - 0.75) <= 2 ** -53


def test_rmse_rows(orc):
    rng = np.random.default_rng(0)
    S = rng.normal(size=(5, 33))
    t = rng.normal(size=33)
    got = orc.rmse_rows(S, t)
    want = np.sqrt(np.mean((S - t) ** 2, axis=1))
    assert np.allclose(got, want, rtol=1e-14, atol=0)
    tt = np.arange(16) / 1024.0
    assert orc.rmse_rows(tt[None, :], tt)[0] == 0.0
    assert orc.rmse_rows((tt + 0.5)[None, :], tt)[0] == 0.5
    assert orc.rmse_rows(np.zeros((2, 0)), np.zeros(0))[1] == 0.0


# --------------------------------------------------------------------------
# Geometric semantic operators (Section 2; Algorithm 1 GSM)

def _worked_rows():
    out = []
    for line in open(os.path.join(GOLDEN, "variation_worked.txt")):
        if line.startswith("#") or not line.strip():
            continue
        head, o, r = (s.strip() for s in line.split("|"))
        f = head.split()
        out.append((f[0], [int(v) for v in f[1:5]], float(f[5]), [float(v) for v in o.split()],
                    float(r)))
    return out


def test_variation_hand_worked(orc):
    S_P = np.array([[1.0, 2.0], [0.0, 0.0]])
    sigR = orc.sigmoid(np.array([[0.0, 0.0], [math.log(3.0), -math.log(3.0)]]))
    t = np.array([1.0, 2.0])
    rows = _worked_rows()
    rec = np.zeros(len(rows), dtype=orc.RECORD_DTYPE)
    for i, (op, idx, ms, _, _) in enumerate(rows):
        rec[i] = (orc.OP_XO if op == "XO" else orc.OP_MUT, idx[0], idx[1], idx[2], idx[3], 0, ms)
    # vary() needs a square parent matrix only through its indices: embed
    S_big = np.zeros((len(rows), 2))
    S_big[:2] = S_P
    O = orc.vary(rec, S_big, sigR)
    F = orc.rmse_rows(O, t)
    for i, (_, _, _, o, r) in enumerate(rows):
        assert np.allclose(O[i], o, rtol=1e-15, atol=1e-15), (i, O[i], o)
        assert abs(F[i] - r) <= 1e-15 * max(1.0, r), (i, F[i], r)


def test_variation_identities_and_bounds(orc):
    rng = np.random.default_rng(4)
    m, r, n = 8, 5, 40
    S = rng.normal(scale=3.0, size=(m, n))
    R = orc.sigmoid(rng.normal(scale=2.0, size=(r, n)))
    rec = np.zeros(m, dtype=orc.RECORD_DTYPE)
    for i in range(m):
        rec[i] = (orc.OP_MUT, i, -1, i % r, i % r, 0, 0.3)      # R1 == R2
    assert np.array_equal(orc.vary(rec, S, R), S)
    for i in range(m):
        rec[i] = (orc.OP_MUT, i, -1, (i + 1) % r, i % r, 0, 0.0)  # ms == 0
    assert np.array_equal(orc.vary(rec, S, R), S)
    for i in range(m):
        rec[i] = (orc.OP_MUT, i, -1, (i + 1) % r, (i + 2) % r, 0, 0.1)
    O = orc.vary(rec, S, R)
    assert np.all(np.abs(O - S) <= 0.1 + 1e-15)
    for i in range(m):
        rec[i] = (orc.OP_XO, i, (i + 3) % m, i % r, -1, 0, 0.0)
    O = orc.vary(rec, S, R)
    lo = np.minimum(S, S[(np.arange(m) + 3) % m])
    hi = np.maximum(S, S[(np.arange(m) + 3) % m])
    assert np.all(O >= lo - 1e-12) and np.all(O <= hi + 1e-12)
    for i in range(m):
        rec[i] = (orc.OP_XO, i, i, i % r, -1, 0, 0.0)             # p1 == p2
    assert np.allclose(orc.vary(rec, S, R), S, rtol=2 ** -52, atol=0)
    half = orc.sigmoid(np.zeros((1, n)))
    for i in range(m):
        rec[i] = (orc.OP_XO, i, (i + 1) % m, 0, -1, 0, 0.0)       # pool tree == 0
    O = orc.vary(rec, S, half)
    assert np.allclose(O, 0.5 * (S + S[(np.arange(m) + 1) % m]), rtol=1e-15, atol=1e-15)


# --------------------------------------------------------------------------
# Variation draws: tournaments and the random-tree / step indices

def test_select_matches_brute_force(orc):
    cfg = orc.Config(pop_size=50, pool_size=17, tournament_size=4, p_crossover=0.5,
                     mutation_step=0.1, ms_random=1, seed=1234, run_id=2)
    F = np.random.default_rng(3).uniform(size=50)
    F[7] = F[9] = F[11] = F.min() - 1.0  # exact ties: the first drawn wins
    for gen in (1, 2, 77):
        rec = orc.select(cfg, gen, F)
        for i in range(cfg.pop_size):
            W = pyphilox.words(i, gen, 5 + 2 * 4, cfg.seed, cfg.run_id)
            cand1 = [pyphilox.below(w, 50) for w in W[5:9]]
            cand2 = [pyphilox.below(w, 50) for w in W[9:13]]

            def winner(c):
                best = c[0]
                for x in c[1:]:
                    if F[x] < F[best]:
                        best = x
                return best

            xo = W[0] < pyphilox.threshold(0.5)
            d = rec[i]
            assert d["op"] == (orc.OP_XO if xo else orc.OP_MUT)
            assert d["p1"] == winner(cand1)
            assert d["r1"] == pyphilox.below(W[1], 17)
            if xo:
                assert d["p2"] == winner(cand2) and d["r2"] == -1 and d["ms"] == 0.0
            else:
                assert d["p2"] == -1 and d["r2"] == pyphilox.below(W[2], 17)
                assert d["ms"] == 0.1 * pyphilox.u53(W[3], W[4])


def test_select_rank_frequencies():
    """Winner rank law of a size-s tournament with replacement:
    P(rank j) = ((m - j + 1)^s - (m - j)^s) / m^s (rank 1 = best)."""
    from oracle import oracle as orc
    from scipy import stats
    m, s = 32, 4
    cfg = orc.Config(pop_size=m, pool_size=8, tournament_size=s, p_crossover=0.0, seed=9)
    F = np.arange(m, dtype=float)[::-1].copy()  # individual m-1 is the best
    counts = np.zeros(m)
    for gen in range(1, 400):
        rec = orc.select(cfg, gen, F)
        ranks = (m - 1 - rec["p1"])  # rank 0 = best
        counts += np.bincount(ranks, minlength=m)
    j = np.arange(1, m + 1)
    p = ((m - j + 1.0) ** s - (m - j) ** s) / m ** s
    exp = p * counts.sum()
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    assert stats.chisquare(obs, ex).pvalue > 1e-3


def test_select_size_one_is_uniform_and_paper_mode(orc):
    from scipy import stats
    m = 16
    cfg = orc.Config(pop_size=m, pool_size=4, tournament_size=1, p_crossover=0.0, seed=2)
    F = np.arange(m, dtype=float)
    counts = np.zeros(m)
    for gen in range(1, 300):
        counts += np.bincount(orc.select(cfg, gen, F)["p1"], minlength=m)
    assert stats.chisquare(counts).pvalue > 1e-3
    cfg = orc.Config(pop_size=m, pool_size=4, tournament_size=0, p_crossover=0.0, seed=2)
    rec = orc.select(cfg, 1, F)
    assert np.array_equal(rec["p1"], np.arange(m)) and np.all(rec["op"] == orc.OP_MUT)


# --------------------------------------------------------------------------
# Survival with elitism (Section 2.2 "Survival")

def test_survival_rules(orc):
    m, n = 5, 3
    SP = np.arange(m * n, dtype=float).reshape(m, n)
    SO = -np.arange(m * n, dtype=float).reshape(m, n)
    SPt = SP[:, :2].copy()
    SOt = SO[:, :2].copy()
    F_P = np.array([3.0, 1.0, 2.0, 1.0, 5.0])
    Ft_P = F_P * 10
    F_O = np.array([4.0, 2.0, 7.0, 7.0, 1.5])
    Ft_O = F_O * 10
    copied, src, dst = orc.survive(F_P, Ft_P, F_O, Ft_O, SP, SO, SPt, SOt)
    assert (copied, src, dst) == (1, 1, 2)  # first argmin parent, first argmax offspring
    assert np.array_equal(SO[2], SP[1]) and np.array_equal(SOt[2], SPt[1])
    assert F_O[2] == 1.0 and Ft_O[2] == 10.0
    F_O2 = np.array([4.0, 1.0, 7.0, 7.0, 1.5])  # tie: parent not strictly better
    copied, _, _ = orc.survive(F_P, Ft_P, F_O2, F_O2 * 10, SP, SO, SPt, SOt)
    assert copied == 0


# --------------------------------------------------------------------------
# Whole runs (Algorithm 1)

def _small_data(n_tr=30, n_te=10, l=3, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n_tr + n_te, l))
    y = X[:, 0] * X[:, 1] + np.sin(X[:, 2])
    return X[:n_tr], y[:n_tr], X[n_tr:], y[n_tr:]


def test_run_elitism_monotone_and_consistent(orc):
    cfg = orc.Config(pop_size=24, pool_size=16, seed=21)
    Xtr, ytr, Xte, yte = _small_data()
    res = orc.run(cfg, Xtr, ytr, Xte, yte, 25, keep_semantics=True)
    best = [s["best_train_rmse"] for s in res.stats]
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    for g in range(26):
        Str, Ste = res.S_hist[g]
        assert np.allclose(res.F_hist[g], np.sqrt(np.mean((Str - ytr) ** 2, axis=1)), rtol=1e-13)
        assert np.allclose(res.Ft_hist[g], np.sqrt(np.mean((Ste - yte) ** 2, axis=1)), rtol=1e-13)
    for g in range(1, 26):
        copied, src, dst = res.elite[g - 1]
        if copied:
            assert np.array_equal(res.S_hist[g][0][dst], res.S_hist[g - 1][0][src])
    assert res.elite[:, 0].sum() > 0


def test_run_deterministic_and_thread_independent(orc):
    cfg = orc.Config(pop_size=20, pool_size=12, seed=5)
    Xtr, ytr, Xte, yte = _small_data(seed=1)
    orc.set_threads(1)
    a = orc.run(cfg, Xtr, ytr, Xte, yte, 8)
    orc.set_threads(4)
    b = orc.run(cfg, Xtr, ytr, Xte, yte, 8)
    assert np.array_equal(a.S_train, b.S_train) and np.array_equal(a.records, b.records)
    assert np.array_equal(a.F, b.F)


def test_run_drive_reproduces(orc):
    cfg = orc.Config(pop_size=16, pool_size=8, seed=6)
    Xtr, ytr, Xte, yte = _small_data(seed=2)
    a = orc.run(cfg, Xtr, ytr, Xte, yte, 6)
    b = orc.run(cfg, Xtr, ytr, Xte, yte, 6, drive=(a.records, a.elite))
    assert np.array_equal(a.S_train, b.S_train) and np.array_equal(a.F, b.F)


# --------------------------------------------------------------------------
# Lineage reconstruction (Section 2.1 stage 3; Algorithm 1 "Return")

def _brute(res, cfg, g, i, X, orc):
    """Recursive evaluation without memoisation, straight from the definitions."""
    m = cfg.pop_size
    if g == 0:
        return orc.interpret(res.code[i:i + 1], res.cval[i:i + 1], X)[0]
    copied, src, dst = res.elite[g - 1]
    if copied and i == dst:
        return _brute(res, cfg, g - 1, int(src), X, orc)
    d = res.records[g - 1][i]

    def R(j):
        return orc.sigmoid(orc.interpret(res.code[m + j:m + j + 1], res.cval[m + j:m + j + 1], X))[0]

    if d["op"] == orc.OP_XO:
        r = R(int(d["r1"]))
        return _brute(res, cfg, g - 1, int(d["p1"]), X, orc) * r + \
            _brute(res, cfg, g - 1, int(d["p2"]), X, orc) * (1.0 - r)
    return _brute(res, cfg, g - 1, int(d["p1"]), X, orc) + float(d["ms"]) * (
        R(int(d["r1"])) - R(int(d["r2"])))


def test_reconstruct_brute_force(orc):
    cfg = orc.Config(pop_size=4, pool_size=4, seed=17)
    Xtr, ytr, Xte, yte = _small_data(n_tr=5, n_te=3, seed=3)
    G = 5
    res = orc.run(cfg, Xtr, ytr, Xte, yte, G, keep_semantics=True)
    for i in range(4):
        bf = _brute(res, cfg, G, i, Xtr, orc)
        assert np.array_equal(bf, res.S_train[i])
        assert np.array_equal(orc.reconstruct(res, cfg, G, i, Xtr), res.S_train[i])
        assert np.array_equal(orc.reconstruct(res, cfg, G, i, Xte), res.S_test[i])
    Xnew = np.random.default_rng(9).uniform(-1, 1, size=(7, 3))
    for g in (0, 2, G):
        for i in range(4):
            assert np.array_equal(orc.reconstruct(res, cfg, g, i, Xnew), _brute(res, cfg, g, i, Xnew, orc))


def test_reconstruct_mutation_only_closed_form(orc):
    """Paper loop (mutate every individual, no selection): individual i after
    G generations is T0[i] + sum_g ms_g (sigma(R_u_g) - sigma(R_v_g)) unless an
    elite copy interrupts its line."""
    cfg = orc.Config(pop_size=6, pool_size=5, tournament_size=0, p_crossover=0.0,
                     ms_random=1, seed=23)
    Xtr, ytr, Xte, yte = _small_data(n_tr=12, n_te=4, seed=4)
    G = 10
    res = orc.run(cfg, Xtr, ytr, Xte, yte, G)
    m = cfg.pop_size
    sig = orc.sigmoid(orc.interpret(res.code[m:], res.cval[m:], Xtr))
    for i in range(m):
        if any(res.elite[g, 0] and res.elite[g, 2] == i for g in range(G)):
            continue
        val = orc.interpret(res.code[i:i + 1], res.cval[i:i + 1], Xtr)[0].copy()
        for g in range(G):
            d = res.records[g][i]
            assert d["p1"] == i and d["op"] == orc.OP_MUT
            val += float(d["ms"]) * (sig[int(d["r1"])] - sig[int(d["r2"])])
        assert np.allclose(val, res.S_train[i], rtol=1e-12, atol=1e-12)


def test_export_linear_evaluates_to_the_lineage(orc):
    """The compact model of a mutation-only lineage, evaluated as
    T(x) + sum_j w_j sigma(R_j(x)), equals the individual's semantics on the
    training cases and on new cases (through reconstruction), elite copies
    included; a lineage with a crossover has no such model."""
    cfg = orc.Config(pop_size=8, pool_size=6, tournament_size=0, p_crossover=0.0, ms_random=1, seed=31)
    Xtr, ytr, Xte, yte = _small_data(n_tr=20, n_te=6, seed=9)
    G = 14
    res = orc.run(cfg, Xtr, ytr, Xte, yte, G)
    assert res.elite[:, 0].sum() > 0  # the walk crosses elite copies
    m = cfg.pop_size
    Xnew = np.random.default_rng(5).uniform(-1, 1, size=(9, Xtr.shape[1]))
    for X, want_of in ((Xtr, lambda i: res.S_train[i]), (Xnew, lambda i: orc.reconstruct(res, cfg, G, i, Xnew))):
        sig = orc.sigmoid(orc.interpret(res.code[m:], res.cval[m:], X))
        for i in range(m):
            tree, c, b, w = orc.export_linear(res, cfg, G, i)
            assert c == 0.0 and b == 1.0
            val = orc.interpret(res.code[tree:tree + 1], res.cval[tree:tree + 1], X)[0] + w @ sig
            want = want_of(i)
            assert np.allclose(val, want, rtol=1e-12, atol=1e-12 * np.max(np.abs(want)))
    # generation 0: the tree itself, no weights
    tree, c, b, w = orc.export_linear(res, cfg, 0, 3)
    assert tree == 3 and not w.any() and (c, b) == (0.0, 1.0)
    cfg2 = orc.Config(pop_size=8, pool_size=6, seed=31)  # tournaments and crossover
    res2 = orc.run(cfg2, Xtr, ytr, Xte, yte, 6)
    with pytest.raises(ValueError):
        for i in range(8):
            orc.export_linear(res2, cfg2, 6, i)


def test_resume_from_a_saved_state_is_bit_exact(orc):
    """Checkpoint / resume: the state after generation g (population
    semantics and fitness; the pool and the data do not change) and the
    generation index determine the rest of the run, because every draw of
    generation g' comes from counter (offspring, word block, g', 3).  A run
    continued by hand from generation 6 equals the straight run bit for bit."""
    cfg = orc.Config(pop_size=20, pool_size=12, seed=41)
    Xtr, ytr, Xte, yte = _small_data(n_tr=30, n_te=10, seed=6)
    G, g0 = 12, 6
    full = orc.run(cfg, Xtr, ytr, Xte, yte, G, keep_semantics=True)
    S_tr, S_te = (a.copy() for a in full.S_hist[g0])
    F, Ft = full.F_hist[g0].copy(), full.Ft_hist[g0].copy()
    m = cfg.pop_size
    R_tr, R_te = full.sigR_train, full.sigR_test
    for g in range(g0 + 1, G + 1):
        rec = orc.select(cfg, g, F)
        assert np.array_equal(rec, full.records[g - 1]), g
        O_tr, O_te = orc.vary(rec, S_tr, R_tr), orc.vary(rec, S_te, R_te)
        F_O, Ft_O = orc.rmse_rows(O_tr, ytr), orc.rmse_rows(O_te, yte)
        elite = orc.survive(F, Ft, F_O, Ft_O, S_tr, O_tr, S_te, O_te)
        assert tuple(elite) == tuple(int(v) for v in full.elite[g - 1]), g
        S_tr, S_te, F, Ft = O_tr, O_te, F_O, Ft_O
    assert np.array_equal(S_tr, full.S_train) and np.array_equal(S_te, full.S_test)
    assert np.array_equal(F, full.F) and np.array_equal(Ft, full.Ft)


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The oracle's C code built with AddressSanitizer and UBSan runs a
    small GSGP loop (ragged sizes, tournaments, crossover, the mutate-all
    loop with random steps, a one-case test segment) without a report."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "oracle_sanitized")
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_sanitize_driver.c")
    osrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "gsgp_oracle.c")
    subprocess.check_call([gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", exe, src, osrc, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "sanitized oracle ok" in out.stdout


# --------------------------------------------------------------------------
# Local search: least-squares scaling of each offspring (Section 3.2 and
# Section 5 name GSGP with local search without defining it; the reading is
# the simple linear regression of the training target on the offspring).

def _ls_golden():
    rows = []
    for line in open(os.path.join(GOLDEN, "least_squares_worked.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = [part.split() for part in line.split("|")]
        rows.append(([float(v) for v in f[0]], [float(v) for v in f[1]], float(f[2][0]), float(f[2][1]),
                     float(f[3][0]), [float(v) for v in f[4]], [float(v) for v in f[5]], float(f[6][0])))
    return rows


def test_least_squares_hand_worked(orc):
    for O, t, a, b, rmse, Ote, tte, rmse_te in _ls_golden():
        ga, gb = orc.ls_fit(np.array([O]), np.array(t))
        assert abs(ga[0] - a) <= 1e-12 * max(1.0, abs(a)) and abs(gb[0] - b) <= 1e-12 * max(1.0, abs(b)), (O, t)
        Os = orc.ls_apply(np.array([O]), ga, gb)
        assert abs(orc.rmse_rows(Os, np.array(t))[0] - rmse) <= 1e-12 * max(1.0, rmse)
        Ot = orc.ls_apply(np.array([Ote]), ga, gb)
        assert abs(orc.rmse_rows(Ot, np.array(tte))[0] - rmse_te) <= 1e-12 * max(1.0, rmse_te)


def test_least_squares_matches_numpy_lstsq_and_is_optimal(orc):
    rng = np.random.default_rng(41)
    n = 300
    O = rng.normal(0.3, 2.0, size=(12, n))
    t = np.sin(rng.uniform(-2, 2, size=n)) + 0.1 * rng.normal(size=n)
    a, b = orc.ls_fit(O, t)
    Os = orc.ls_apply(O, a, b)
    for i in range(O.shape[0]):
        A = np.stack([np.ones(n), O[i]], axis=1)
        coef = np.linalg.lstsq(A, t, rcond=None)[0]
        assert np.allclose([a[i], b[i]], coef, rtol=1e-10, atol=1e-12)
        base = float(np.sqrt(np.mean((Os[i] - t) ** 2)))
        assert base <= float(np.sqrt(np.mean((O[i] - t) ** 2)))  # never worse than unscaled
        for da, db in ((1e-3, 0), (-1e-3, 0), (0, 1e-3), (0, -1e-3)):
            assert base <= float(np.sqrt(np.mean((a[i] + da + (b[i] + db) * O[i] - t) ** 2)))
        r = t - Os[i]  # normal equations: residual orthogonal to 1 and to O
        assert abs(r.sum()) <= 1e-10 * n and abs(r @ O[i]) <= 1e-10 * n * np.max(np.abs(O[i]))


def test_least_squares_exact_cases(orc):
    rng = np.random.default_rng(42)
    O = rng.uniform(-3, 3, size=(4, 50))
    # a target that already equals the offspring: nothing to scale
    a, b = orc.ls_fit(O[:1], O[0])
    assert a[0] == 0.0 and b[0] == 1.0
    # an exactly linear target: recovered, zero error
    t = -1.25 + 0.5 * O[1]
    a, b = orc.ls_fit(O[1:2], t)
    assert abs(a[0] + 1.25) <= 1e-12 and abs(b[0] - 0.5) <= 1e-12
    assert orc.rmse_rows(orc.ls_apply(O[1:2], a, b), t)[0] <= 1e-13
    # the scaled offspring does not depend on an affine change of O
    a1, b1 = orc.ls_fit(O[2:3], O[3])
    a2, b2 = orc.ls_fit(4.0 - 3.0 * O[2:3], O[3])
    assert np.allclose(orc.ls_apply(O[2:3], a1, b1), orc.ls_apply(4.0 - 3.0 * O[2:3], a2, b2), atol=1e-12)
    # a constant offspring is kept as it is
    a, b = orc.ls_fit(np.full((1, 50), 0.7), O[3])
    assert a[0] == 0.0 and b[0] == 1.0


def test_run_with_local_search_scales_every_variation_offspring(orc):
    """In a run with local search every offspring of a variation is the
    least-squares scaling of the plain operator's output (the residual of
    its training semantics sums to zero and is orthogonal to it), an elite
    copy carries its source's values and scaling, and elitism still keeps
    the best RMSE monotone."""
    Xtr, ytr, Xte, yte = _small_data(n_tr=80, n_te=30, seed=11)
    cfg = orc.Config(pop_size=24, pool_size=16, seed=7, local_search=True)
    G = 10
    res = orc.run(cfg, Xtr, ytr, Xte, yte, G, keep_semantics=True)
    best = [s["best_train_rmse"] for s in res.stats]
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    m = cfg.pop_size
    plain = orc.Config(pop_size=24, pool_size=16, seed=7)
    for g in range(1, G + 1):
        S_prev_tr, S_prev_te = res.S_hist[g - 1]
        O_tr = orc.vary(res.records[g - 1], S_prev_tr, res.sigR_train)
        O_te = orc.vary(res.records[g - 1], S_prev_te, res.sigR_test)
        copied, src, dst = res.elite[g - 1]
        S_tr, S_te = res.S_hist[g]
        for i in range(m):
            if copied and i == dst:
                assert np.array_equal(S_tr[i], S_prev_tr[src])
                assert np.array_equal(res.scale[g, i], res.scale[g - 1, src])
                continue
            a, b = res.scale[g, i]
            assert np.allclose(S_tr[i], a + b * O_tr[i], rtol=0, atol=1e-12 * max(1.0, np.abs(S_tr[i]).max()))
            assert np.allclose(S_te[i], a + b * O_te[i], rtol=0, atol=1e-12 * max(1.0, np.abs(S_te[i]).max()))
            r = ytr - S_tr[i]
            if b != 1.0 or a != 0.0:
                assert abs(r.sum()) <= 1e-9 * len(r) and abs(r @ S_tr[i]) <= 1e-9 * len(r) * np.abs(S_tr[i]).max()
        assert np.allclose(res.F_hist[g], np.sqrt(np.mean((S_tr - ytr) ** 2, axis=1)), rtol=1e-13)
    # local search never makes the run's best worse than the plain run's after the same draws
    assert res.scale[1:, :, 1].std() > 0
    del plain


def test_reconstruct_and_export_with_local_search(orc):
    """Lineages of a run with local search: brute-force recursion (each step
    followed by its offspring's recorded scaling) equals the stored
    semantics and the memoised reconstruction on new cases; the compact model
    c + b T + sum_j w_j sigma(R_j) of a mutation-only lineage evaluates to
    the same values."""
    Xtr, ytr, Xte, yte = _small_data(n_tr=9, n_te=4, seed=12)
    cfg = orc.Config(pop_size=5, pool_size=4, seed=19, local_search=True)
    G = 5
    res = orc.run(cfg, Xtr, ytr, Xte, yte, G, keep_semantics=True)
    m = cfg.pop_size

    def R(j, X):
        return orc.sigmoid(orc.interpret(res.code[m + j:m + j + 1], res.cval[m + j:m + j + 1], X))[0]

    def brute(g, i, X):
        if g == 0:
            return orc.interpret(res.code[i:i + 1], res.cval[i:i + 1], X)[0]
        copied, src, dst = res.elite[g - 1]
        if copied and i == dst:
            return brute(g - 1, int(src), X)
        d = res.records[g - 1][i]
        if d["op"] == orc.OP_XO:
            o = brute(g - 1, int(d["p1"]), X) * R(int(d["r1"]), X) + \
                brute(g - 1, int(d["p2"]), X) * (1.0 - R(int(d["r1"]), X))
        else:
            o = brute(g - 1, int(d["p1"]), X) + float(d["ms"]) * (R(int(d["r1"]), X) - R(int(d["r2"]), X))
        a, b = res.scale[g, i]
        return a + b * o

    Xnew = np.random.default_rng(13).uniform(-1, 1, size=(6, Xtr.shape[1]))
    for i in range(m):
        assert np.array_equal(brute(G, i, Xtr), res.S_train[i])
        assert np.array_equal(orc.reconstruct(res, cfg, G, i, Xnew), brute(G, i, Xnew))
    cfgm = orc.Config(pop_size=6, pool_size=5, tournament_size=0, p_crossover=0.0, ms_random=1, seed=23,
                      local_search=True)
    resm = orc.run(cfgm, Xtr, ytr, Xte, yte, 8)
    sig = orc.sigmoid(orc.interpret(resm.code[6:], resm.cval[6:], Xnew))
    for i in range(6):
        tree, c, b, w = orc.export_linear(resm, cfgm, 8, i)
        val = c + b * orc.interpret(resm.code[tree:tree + 1], resm.cval[tree:tree + 1], Xnew)[0] + w @ sig
        want = orc.reconstruct(resm, cfgm, 8, i, Xnew)
        assert np.allclose(val, want, rtol=1e-12, atol=1e-12 * np.max(np.abs(want)))


# --------------------------------------------------------------------------
# Replay mode's own check (the oracle follows a given lineage and confirms
# every recorded decision against its own draws and fitness)

def test_replay_check_counts_disagreements_and_near_ties(orc):
    Xtr, ytr, Xte, yte = _small_data(seed=14)
    cfg = orc.Config(pop_size=32, pool_size=16, seed=29)
    G = 8
    a = orc.run(cfg, Xtr, ytr, Xte, yte, G)
    b = orc.run(cfg, Xtr, ytr, Xte, yte, G, drive=(a.records, a.elite))
    assert len(b.replay) == G
    assert all(c["draw_mismatch"] == 0 and c["winner_mismatch"] == 0 and c["elite_mismatch"] == 0 for c in b.replay)
    # a planted wrong tournament winner (not a near tie) is counted with its gap
    rec = a.records.copy()
    g, i = 3, int(np.nonzero(rec[3]["op"] == orc.OP_MUT)[0][0])
    F2 = a.F_hist[g]
    worst = int(np.argmax(F2))
    assert rec[g][i]["p1"] != worst
    rec[g][i]["p1"] = worst
    c = orc.run(cfg, Xtr, ytr, Xte, yte, G, drive=(rec, a.elite))
    assert c.replay[g]["winner_mismatch"] == 1 and c.replay[g]["winner_gap_max"] > 1e-3
    assert sum(x["winner_mismatch"] for x in c.replay[:g]) == 0
    # a planted pool row is a draw mismatch; a planted elite decision is counted
    rec2 = a.records.copy()
    rec2[1][0]["r1"] = (rec2[1][0]["r1"] + 1) % cfg.pool_size
    el = a.elite.copy()
    el[5] = (0, -1, -1) if el[5][0] else (1, 0, 1)
    d = orc.run(cfg, Xtr, ytr, Xte, yte, G, drive=(rec2, el))
    assert d.replay[1]["draw_mismatch"] == 1 and d.replay[5]["elite_mismatch"] == 1
