"""Python driver of the plain FP64 CPU oracle (test infrastructure).

THIS IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  It never imports the HIP
package and the HIP package never imports it; both receive the same seeded
inputs from ``paper_2106_04034_amd.synth`` (which holds none of the method).

The arithmetic lives in ``gsgp_oracle.c`` (plain loops, FP64).  This module
only marshals numpy arrays and runs Algorithm 1 of the GSGP-CUDA paper
(arXiv 2106.04034, Section 2.2) generation by generation:

    CreatePopulation(m), CreatePopulation(r)       -> genomes
    ComputeSemantics(P), ComputeSemantics(R)       -> S_P, S_R (R squashed)
    ComputeFitness(S_P)                            -> F_P
    for generation 1..G: variation draws, GSM/GSC, ComputeFitness, survival

and the lineage reconstruction of an individual on new data (Section 2.1,
stage 3: lineage structures; Algorithm 1: "Return: best individual").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsgp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

RECORD_DTYPE = np.dtype(
    [("op", "<i4"), ("p1", "<i4"), ("p2", "<i4"), ("r1", "<i4"), ("r2", "<i4"),
     ("pad", "<i4"), ("ms", "<f8")]
)
OP_MUT, OP_XO = 0, 1
GENE_ADD, GENE_SUB, GENE_MUL, GENE_DIV, GENE_CONST = -1, -2, -3, -4, -5
TAG_POPULATION, TAG_POOL, TAG_SELECTION = 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP over rows)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("pop_size", ctypes.c_int32), ("pool_size", ctypes.c_int32),
        ("genome_len", ctypes.c_int32), ("tournament_size", ctypes.c_int32),
        ("p_crossover", ctypes.c_double), ("mutation_step", ctypes.c_double),
        ("ms_random", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("p_function", ctypes.c_double), ("p_feature", ctypes.c_double),
        ("erc_lo", ctypes.c_double), ("erc_hi", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("run_id", ctypes.c_uint32),
    ]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.orc_philox.argtypes = [P, P, P]
        L.orc_event_threshold.argtypes = [ctypes.c_double]
        L.orc_event_threshold.restype = ctypes.c_uint64
        L.orc_genomes.argtypes = [P, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32, P, P]
        L.orc_interpret.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64,
                                    ctypes.c_int32, P]
        L.orc_sigmoid.argtypes = [P, P, ctypes.c_int64]
        L.orc_rmse_rows.argtypes = [P, ctypes.c_int32, ctypes.c_int64, P, P]
        L.orc_select.argtypes = [P, ctypes.c_int32, P, P]
        L.orc_vary.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int64, P]
        L.orc_argmin.argtypes = [P, ctypes.c_int32]
        L.orc_argmin.restype = ctypes.c_int32
        L.orc_argmax.argtypes = [P, ctypes.c_int32]
        L.orc_argmax.restype = ctypes.c_int32
        L.orc_survive.argtypes = [ctypes.c_int32, P, P, P, P, P, P, ctypes.c_int64, P, P,
                                  ctypes.c_int64, P, P]
        L.orc_survive.restype = ctypes.c_int32
        L.orc_ls_fit.argtypes = [P, ctypes.c_int32, ctypes.c_int64, P, P, P]
        L.orc_ls_apply.argtypes = [P, ctypes.c_int32, ctypes.c_int64, P, P]
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_max_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Config:
    """Run parameters (Algorithm 1 inputs m, r, k, g plus operator settings)."""
    pop_size: int = 128
    pool_size: int = 128
    genome_len: int = 127
    tournament_size: int = 4
    p_crossover: float = 0.5
    mutation_step: float = 0.1
    ms_random: int = 0
    p_function: float = 0.80
    p_feature: float = 0.14
    erc_lo: float = -1.0
    erc_hi: float = 1.0
    seed: int = 1
    run_id: int = 0
    local_search: bool = False  # least-squares scaling of every offspring (see ls_fit)

    def c(self) -> _Cfg:
        return _Cfg(self.pop_size, self.pool_size, self.genome_len, self.tournament_size,
                    self.p_crossover, self.mutation_step, self.ms_random, 0,
                    self.p_function, self.p_feature, self.erc_lo, self.erc_hi,
                    self.seed & 0xFFFFFFFF, self.run_id & 0xFFFFFFFF)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def philox(ctr, key) -> tuple:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c), _p(k), _p(o))
    return tuple(int(v) for v in o)


def event_threshold(p: float) -> int:
    return int(lib().orc_event_threshold(float(p)))


def genomes(cfg: Config, n_features: int, tag: int, rows: int):
    code = np.zeros((rows, cfg.genome_len), dtype=np.int32)
    cval = np.zeros((rows, cfg.genome_len), dtype=np.float64)
    c = cfg.c()
    lib().orc_genomes(ctypes.byref(c), n_features, tag, rows, _p(code), _p(cval))
    return code, cval


def interpret(code: np.ndarray, cval: np.ndarray, X: np.ndarray) -> np.ndarray:
    code = np.ascontiguousarray(code, dtype=np.int32)
    cval = np.ascontiguousarray(cval, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    rows, k = code.shape
    n, l = X.shape if X.ndim == 2 else (0, 1)
    out = np.zeros((rows, n), dtype=np.float64)
    if rows and n:
        lib().orc_interpret(_p(code), _p(cval), rows, k, _p(X), n, l, _p(out))
    return out


def sigmoid(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    if x.size:
        lib().orc_sigmoid(_p(x), _p(out), x.size)
    return out


def rmse_rows(S: np.ndarray, t: np.ndarray) -> np.ndarray:
    S = np.ascontiguousarray(S, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    rows = S.shape[0]
    n = S.shape[1] if S.ndim == 2 else 0
    out = np.zeros(rows, dtype=np.float64)
    if rows:
        lib().orc_rmse_rows(_p(S), rows, n, _p(t) if n else None, _p(out))
    return out


def select(cfg: Config, gen: int, F: np.ndarray) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.float64)
    rec = np.zeros(cfg.pop_size, dtype=RECORD_DTYPE)
    c = cfg.c()
    lib().orc_select(ctypes.byref(c), gen, _p(F), _p(rec))
    return rec


def vary(rec: np.ndarray, S_P: np.ndarray, sigR: np.ndarray) -> np.ndarray:
    rec = np.ascontiguousarray(rec, dtype=RECORD_DTYPE)
    S_P = np.ascontiguousarray(S_P, dtype=np.float64)
    sigR = np.ascontiguousarray(sigR, dtype=np.float64)
    m = rec.shape[0]
    n = S_P.shape[1]
    out = np.zeros((m, n), dtype=np.float64)
    if m and n:
        lib().orc_vary(_p(rec), m, _p(S_P), _p(sigR), n, _p(out))
    return out


def ls_fit(O: np.ndarray, t: np.ndarray):
    """Least-squares scaling (alpha, beta) of each row of O against t
    (local search; see orc_ls_fit for the reading)."""
    O = np.ascontiguousarray(O, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    rows = O.shape[0]
    n = O.shape[1] if O.ndim == 2 else 0
    a = np.zeros(rows)
    b = np.ones(rows)
    if rows and n:
        lib().orc_ls_fit(_p(O), rows, n, _p(t), _p(a), _p(b))
    return a, b


def ls_apply(O: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """alpha + beta * O row by row (a new array)."""
    O = np.array(O, dtype=np.float64, order="C", copy=True)
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    if O.size:
        lib().orc_ls_apply(_p(O), O.shape[0], O.shape[1], _p(a), _p(b))
    return O


def argmin(F: np.ndarray) -> int:
    F = np.ascontiguousarray(F, dtype=np.float64)
    return int(lib().orc_argmin(_p(F), F.size))


def argmax(F: np.ndarray) -> int:
    F = np.ascontiguousarray(F, dtype=np.float64)
    return int(lib().orc_argmax(_p(F), F.size))


def survive(F_P, Ft_P, F_O, Ft_O, SP_tr, SO_tr, SP_te, SO_te):
    """Elitist survival in place on the offspring arrays; returns (copied, src, dst)."""
    m = F_P.size
    src = ctypes.c_int32(-1)
    dst = ctypes.c_int32(-1)
    n_tr = SP_tr.shape[1]
    n_te = SP_te.shape[1]
    copied = lib().orc_survive(
        m, _p(F_P), _p(Ft_P), _p(F_O), _p(Ft_O), _p(SP_tr), _p(SO_tr), n_tr,
        _p(SP_te) if n_te else None, _p(SO_te) if n_te else None, n_te,
        ctypes.byref(src), ctypes.byref(dst))
    return int(copied), int(src.value), int(dst.value)


@dataclass
class Result:
    code: np.ndarray            # (m + r) x k genome codes (population rows, then pool rows)
    cval: np.ndarray            # (m + r) x k constants
    sigR_train: np.ndarray      # r x n_train, logistic of the pool trees
    sigR_test: np.ndarray
    S_train: np.ndarray         # m x n_train, population after the last generation
    S_test: np.ndarray
    F: np.ndarray               # m, train RMSE of that population
    Ft: np.ndarray
    records: np.ndarray         # G x m raw variation draws
    elite: np.ndarray           # G x 3: (copied, src, dst)
    scale: np.ndarray = None    # (G + 1) x m x 2: (alpha, beta) of each individual (local search)
    stats: list = field(default_factory=list)   # per generation 0..G: dict
    F_hist: list = field(default_factory=list)  # per generation 0..G: F copy
    Ft_hist: list = field(default_factory=list)
    S_hist: list = field(default_factory=list)  # per generation (train, test) when kept
    replay: list = field(default_factory=list)  # per driven generation 1..G: replay check (see run)


def initial_state(cfg: Config, Xtr, ytr, Xte, yte):
    """Genomes, semantics, squashed pool semantics and generation-0 fitness."""
    l = Xtr.shape[1]
    cp, vp = genomes(cfg, l, TAG_POPULATION, cfg.pop_size)
    cr, vr = genomes(cfg, l, TAG_POOL, cfg.pool_size)
    S_tr = interpret(cp, vp, Xtr)
    S_te = interpret(cp, vp, Xte) if Xte.shape[0] else np.zeros((cfg.pop_size, 0))
    R_tr = sigmoid(interpret(cr, vr, Xtr))
    R_te = sigmoid(interpret(cr, vr, Xte)) if Xte.shape[0] else np.zeros((cfg.pool_size, 0))
    F = rmse_rows(S_tr, ytr)
    Ft = rmse_rows(S_te, yte) if Xte.shape[0] else np.zeros(cfg.pop_size)
    return (np.concatenate([cp, cr]), np.concatenate([vp, vr]), S_tr, S_te, R_tr, R_te, F, Ft)


def _stats(F, Ft, copied, src, dst):
    b = argmin(F)
    return {"best_train_rmse": float(F[b]), "best_test_rmse": float(Ft[b]), "best_index": b,
            "elite_copied": copied, "elite_src": src, "elite_dst": dst}


def _rel_gap(a: float, b: float) -> float:
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def replay_check(cfg: Config, gen: int, F: np.ndarray, rec: np.ndarray) -> dict:
    """Checks one generation's given variation draws against the oracle's
    own draws under its own fitness F (the fitness the tournaments of
    generation ``gen`` select on).  Operator, pool rows and step do not
    depend on fitness and must be equal; a tournament winner may differ only
    where the candidates' fitness values nearly tie, so each disagreement is
    counted with the relative fitness gap between the given winner and the
    oracle's winner (0 for an exact tie)."""
    own = select(cfg, gen, F)
    draws = int(np.sum((own["op"] != rec["op"]) | (own["r1"] != rec["r1"]) | (own["r2"] != rec["r2"])
                       | (own["ms"] != rec["ms"])))
    gaps = []
    for key in ("p1", "p2"):
        valid = (own[key] >= 0) & (rec[key] >= 0)
        diff = np.nonzero(valid & (own[key] != rec[key]))[0]
        gaps += [_rel_gap(float(F[rec[key][i]]), float(F[own[key][i]])) for i in diff]
    return {"draw_mismatch": draws, "winner_mismatch": len(gaps), "winner_gap_max": max(gaps, default=0.0)}


def _elite_check(F, F_O, given) -> dict:
    """The survival decision the oracle takes under its own fitness, against
    a given one: equal, or differing only at a near tie (relative gap of the
    comparison that decided it)."""
    bP, bO = argmin(F), argmin(F_O)
    copied = int(F[bP] < F_O[bO])
    w = argmax(F_O)
    own = (copied, bP if copied else -1, w if copied else -1)
    given = tuple(int(v) for v in given)
    if own == given:
        return {"elite_mismatch": 0, "elite_gap": 0.0}
    gaps = [_rel_gap(float(F[bP]), float(F_O[bO]))]
    if given[0] and copied:
        gaps += [_rel_gap(float(F[given[1]]), float(F[bP])), _rel_gap(float(F_O[given[2]]), float(F_O[w]))]
    return {"elite_mismatch": 1, "elite_gap": max(gaps)}


def run(cfg: Config, Xtr, ytr, Xte, yte, G: int, drive=None, keep_semantics=False,
        on_generation=None) -> Result:
    """Algorithm 1 for G generations.

    ``drive`` (optional) is a pair (records G x m, elite G x 3) that replaces
    the oracle's own draws and survival decisions, to follow a lineage made
    elsewhere (replay mode).  In replay mode every generation is also
    checked against what the oracle would have decided itself (its own
    Philox draws and tournaments under its own fitness, its own survival
    decision): ``Result.replay[g - 1]`` holds the counts of disagreements and
    the largest relative fitness gap behind one (see ``replay_check``).

    With ``cfg.local_search`` every offspring formed by a variation operator
    is replaced by its least-squares scaling before its fitness is taken
    (``ls_fit``); the scaling of each individual is kept in
    ``Result.scale``.

    ``on_generation(g, S_tr, S_te, F, Ft)`` (optional) is called with the
    population of generation g = 0..G after survival.
    """
    Xtr = np.ascontiguousarray(Xtr, dtype=np.float64)
    Xte = np.ascontiguousarray(Xte, dtype=np.float64).reshape(-1, Xtr.shape[1])
    ytr = np.ascontiguousarray(ytr, dtype=np.float64)
    yte = np.ascontiguousarray(yte, dtype=np.float64)
    code, cval, S_tr, S_te, R_tr, R_te, F, Ft = initial_state(cfg, Xtr, ytr, Xte, yte)
    m = cfg.pop_size
    records = np.zeros((G, m), dtype=RECORD_DTYPE)
    elite = np.zeros((G, 3), dtype=np.int32)
    scale = np.zeros((G + 1, m, 2))
    scale[0, :, 1] = 1.0
    res = Result(code, cval, R_tr, R_te, S_tr, S_te, F, Ft, records, elite, scale)
    res.stats.append(_stats(F, Ft, 0, -1, -1))
    res.F_hist.append(F.copy())
    res.Ft_hist.append(Ft.copy())
    if keep_semantics:
        res.S_hist.append((S_tr.copy(), S_te.copy()))
    if on_generation is not None:
        on_generation(0, S_tr, S_te, F, Ft)
    for g in range(1, G + 1):
        if drive is not None:
            rec = np.ascontiguousarray(drive[0][g - 1], dtype=RECORD_DTYPE)
            check = replay_check(cfg, g, F, rec)
        else:
            rec = select(cfg, g, F)
        O_tr = vary(rec, S_tr, R_tr)
        O_te = vary(rec, S_te, R_te) if Xte.shape[0] else np.zeros((m, 0))
        if cfg.local_search:
            a, b = ls_fit(O_tr, ytr)
            O_tr = ls_apply(O_tr, a, b)
            if Xte.shape[0]:
                O_te = ls_apply(O_te, a, b)
            scale[g, :, 0], scale[g, :, 1] = a, b
        else:
            scale[g, :, 1] = 1.0
        F_O = rmse_rows(O_tr, ytr)
        Ft_O = rmse_rows(O_te, yte) if Xte.shape[0] else np.zeros(m)
        if drive is not None:
            copied, src, dst = (int(v) for v in drive[1][g - 1])
            check.update(_elite_check(F, F_O, (copied, src, dst)))
            res.replay.append(check)
            if copied:
                O_tr[dst] = S_tr[src]
                if Xte.shape[0]:
                    O_te[dst] = S_te[src]
                F_O[dst] = F[src]
                Ft_O[dst] = Ft[src]
        else:
            copied, src, dst = survive(F, Ft, F_O, Ft_O, S_tr, O_tr, S_te, O_te)
        if copied:
            scale[g, dst] = scale[g - 1, src]
        records[g - 1] = rec
        elite[g - 1] = (copied, src, dst)
        S_tr, S_te, F, Ft = O_tr, O_te, F_O, Ft_O
        res.stats.append(_stats(F, Ft, copied, src, dst))
        res.F_hist.append(F.copy())
        res.Ft_hist.append(Ft.copy())
        if keep_semantics:
            res.S_hist.append((S_tr.copy(), S_te.copy()))
        if on_generation is not None:
            on_generation(g, S_tr, S_te, F, Ft)
    res.S_train, res.S_test, res.F, res.Ft = S_tr, S_te, F, Ft
    return res


def reconstruct(res: Result, cfg: Config, gen: int, individual: int, X: np.ndarray) -> np.ndarray:
    """Semantics of individual ``individual`` of generation ``gen`` on new cases X.

    Walks the lineage backwards to the generation-0 genomes and the pool trees
    it touches, interprets them on X, then replays the recorded combinations
    forward (memoised over the ancestor DAG)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m = cfg.pop_size
    need = [set() for _ in range(gen + 1)]
    need[gen].add(individual)
    pool_needed = set()
    for g in range(gen, 0, -1):
        rec = res.records[g - 1]
        copied, src, dst = (int(v) for v in res.elite[g - 1])
        for i in need[g]:
            if copied and i == dst:
                need[g - 1].add(src)
                continue
            d = rec[i]
            need[g - 1].add(int(d["p1"]))
            pool_needed.add(int(d["r1"]))
            if d["op"] == OP_XO:
                need[g - 1].add(int(d["p2"]))
            else:
                pool_needed.add(int(d["r2"]))
    pool_idx = sorted(pool_needed)
    pop_idx = sorted(need[0])
    vals = {}
    if pop_idx:
        S0 = interpret(res.code[pop_idx], res.cval[pop_idx], X)
        vals = {i: S0[j] for j, i in enumerate(pop_idx)}
    sig = {}
    if pool_idx:
        rows = [m + j for j in pool_idx]
        R = sigmoid(interpret(res.code[rows], res.cval[rows], X))
        sig = {j: R[q] for q, j in enumerate(pool_idx)}
    for g in range(1, gen + 1):
        rec = res.records[g - 1]
        copied, src, dst = (int(v) for v in res.elite[g - 1])
        nxt = {}
        for i in need[g]:
            if copied and i == dst:
                nxt[i] = vals[src].copy()
                continue
            d = rec[i]
            if d["op"] == OP_XO:
                nxt[i] = vals[int(d["p1"])] * sig[int(d["r1"])] + \
                    vals[int(d["p2"])] * (1.0 - sig[int(d["r1"])])
            else:
                nxt[i] = vals[int(d["p1"])] + float(d["ms"]) * (sig[int(d["r1"])] - sig[int(d["r2"])])
            if cfg.local_search:
                a, b = res.scale[g, i]
                nxt[i] = a + b * nxt[i]
        vals = nxt
    return vals[individual]


def export_linear(res: Result, cfg: Config, gen: int, individual: int):
    """Compact model of a mutation-only lineage (the paper's own loop).

    Along a lineage of mutations only, individual ``individual`` of
    generation ``gen`` is c + b T(x) + sum_j w_j sigma(R_j(x)): one
    generation-0 population tree T and a weight per pool tree R_j, since
    every GSM step adds ms (sigma(R_u) - sigma(R_v)) (Section 2, GSM;
    Section 2.1 stage 3, lineage structures).  Without local search c = 0 and
    b = 1; with it each step is followed by the offspring's scaling
    alpha + beta * (...), which scales c, b and w by beta and adds alpha to c.
    Returns (tree index, c, b, weights [r]), accumulated forward generation by
    generation: c = alpha + beta c, b = beta b, w = beta w, then
    w[u] += beta ms, w[v] -= beta ms.  Raises ValueError if the lineage
    contains a crossover."""
    r = cfg.pool_size
    steps = []
    i = individual
    for g in range(gen, 0, -1):
        copied, src, dst = (int(v) for v in res.elite[g - 1])
        if copied and i == dst:
            i = src
            continue
        d = res.records[g - 1][i]
        if d["op"] == OP_XO:
            raise ValueError(f"the lineage contains a crossover at generation {g}")
        steps.append((d, g, i))
        i = int(d["p1"])
    w = np.zeros(r)
    c, b = 0.0, 1.0
    for d, g, j in reversed(steps):
        alpha, beta = (float(res.scale[g, j, 0]), float(res.scale[g, j, 1])) if cfg.local_search else (0.0, 1.0)
        c = alpha + beta * c
        b = beta * b
        w = beta * w
        w[int(d["r1"])] += beta * float(d["ms"])
        w[int(d["r2"])] -= beta * float(d["ms"])
    return i, c, b, w
