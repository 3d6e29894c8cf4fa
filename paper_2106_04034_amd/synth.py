"""Seeded synthetic regression data for GSGP runs.

This module only draws input data (features, targets, per-run sizes).  It
holds none of the evolutionary method, so both the HIP library's callers and
the CPU oracle's tests may use it.  The paper's datasets are not available;
these workloads stand in for the "dummy datasets" of its speed-up study
(Section 3.1) and for real symbolic-regression problems (Section 3.2), with
the shapes listed in ``WORKLOADS``.

Every array is float64, row-major (cases x features), the layout of the
paper's train/test text files (Section 3.3): one row per instance.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 21060403


@dataclass
class Dataset:
    X_train: np.ndarray
    y_train: np.ndarray
    X_test: np.ndarray
    y_test: np.ndarray

    @property
    def n_features(self) -> int:
        return self.X_train.shape[1]


@dataclass
class Workload:
    name: str
    n_train: int
    n_test: int
    n_features: int
    pop_size: int
    pool_size: int
    generations: int
    precision: str
    runs: int = 1
    genome_len: int = 127
    tournament_size: int = 4
    p_crossover: float = 0.5
    mutation_step: float = 0.1
    notes: str = ""
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "plain_fp64_500x8": Workload("plain_fp64_500x8", 500, 200, 8, 128, 128, 20, "fp64",
                                 notes="x0*x1+sin(x2)+0.5*x3^2-x4/(1+|x5|)+N(0,0.01), U[-1,1]"),
    "single_fp32_100k": Workload("single_fp32_100k", 100_000, 25_000, 20, 1024, 1024, 1000, "fp32",
                                 notes="sparse cubic polynomial of 6 features + N(0,0.05), U[-1,1]"),
    "large_fp32_1m": Workload("large_fp32_1m", 1_000_000, 250_000, 64, 2048, 2048, 500, "fp32",
                              notes="sum of 10 feature-pair products + tanh(w.x), N(0,1) features"),
    "precision_1m": Workload("precision_1m", 1_000_000, 250_000, 64, 1024, 1024, 2000, "fp32_kahan",
                             notes="large_fp32_1m data; FP32 vs FP32-Kahan vs FP64 drift"),
    "batched_256": Workload("batched_256", 0, 0, 0, 256, 256, 300, "fp32_kahan", runs=256,
                            notes="n per run log-uniform in [200, 50000], test n/4, 4..32 features"),
}
# The speed-up study's shape (Section 3.1): 102,400 cases, 1,024 features,
# 10,240 individuals, 50 generations, program sizes 127 / 1,023 / 2,047, the
# paper's own loop (every individual mutated once, random step), FP32.
for _k in (127, 1023, 2047):
    WORKLOADS[f"paper_shape_k{_k}"] = Workload(
        f"paper_shape_k{_k}", 102_400, 0, 1024, 10_240, 10_240, 50, "fp32", genome_len=_k,
        tournament_size=0, p_crossover=0.0, mutation_step=0.1,
        notes="U[-1,1] features, sparse cubic target; mutate-all loop, random mutation step")



def _split(X, y, n_train):
    return Dataset(np.ascontiguousarray(X[:n_train]), np.ascontiguousarray(y[:n_train]),
                   np.ascontiguousarray(X[n_train:]), np.ascontiguousarray(y[n_train:]))


def plain_small(n_train=500, n_test=200, n_features=8, seed_offset=0) -> Dataset:
    """x0*x1 + sin(x2) + 0.5*x3^2 - x4/(1+|x5|) + N(0, 0.01), features U[-1, 1]."""
    rng = np.random.default_rng(BASE_SEED + 10 * 0 + seed_offset)
    n = n_train + n_test
    X = rng.uniform(-1.0, 1.0, size=(n, n_features))
    y = (X[:, 0] * X[:, 1] + np.sin(X[:, 2]) + 0.5 * X[:, 3] ** 2
         - X[:, 4] / (1.0 + np.abs(X[:, 5])) + rng.normal(0.0, 0.01, size=n))
    return _split(X, y, n_train)


def sparse_cubic(rng, X, n_vars=6, noise=0.05):
    """Random sparse polynomial of degree 3 over n_vars distinct features:
    2 cubic, 3 quadratic and 3 linear monomials, coefficients U[-1, 1] with
    |a| >= 0.1, variables drawn with replacement from the chosen features."""
    l = X.shape[1]
    feats = rng.choice(l, size=min(n_vars, l), replace=False)
    y = np.zeros(X.shape[0])
    for degree, count in ((3, 2), (2, 3), (1, 3)):
        for _ in range(count):
            a = 0.0
            while abs(a) < 0.1:
                a = rng.uniform(-1.0, 1.0)
            vars_ = rng.choice(feats, size=degree, replace=True)
            term = np.full(X.shape[0], a)
            for v in vars_:
                term = term * X[:, v]
            y = y + term
    return y + rng.normal(0.0, noise, size=X.shape[0])


def single_run(n_train=100_000, n_test=25_000, n_features=20, seed_offset=0) -> Dataset:
    rng = np.random.default_rng(BASE_SEED + 10 * 1 + seed_offset)
    n = n_train + n_test
    X = rng.uniform(-1.0, 1.0, size=(n, n_features))
    y = sparse_cubic(rng, X)
    return _split(X, y, n_train)


def large_run(n_train=1_000_000, n_test=250_000, n_features=64, seed_offset=0) -> Dataset:
    """Sum of 10 products of distinct feature pairs plus tanh(w . x),
    w ~ N(0, 1/64) (standard deviation 1/8), features N(0, 1)."""
    rng = np.random.default_rng(BASE_SEED + 10 * 2 + seed_offset)
    n = n_train + n_test
    X = rng.standard_normal(size=(n, n_features))
    y = np.zeros(n)
    for _ in range(10):
        a, b = rng.choice(n_features, size=2, replace=False)
        y = y + X[:, a] * X[:, b]
    w = rng.normal(0.0, 1.0 / 8.0, size=n_features)
    y = y + np.tanh(X @ w)
    return _split(X, y, n_train)


def batched_runs(runs=256, n_lo=200, n_hi=50_000, seed_offset=0, max_total=None) -> list:
    """Independent runs with uneven sizes: n log-uniform in [n_lo, n_hi],
    test = floor(n / 4), 4..32 features U[-1, 1], sparse cubic target."""
    rng = np.random.default_rng(BASE_SEED + 10 * 4 + seed_offset)
    out = []
    for _ in range(runs):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        n_test = n // 4
        l = int(rng.integers(4, 33))
        X = rng.uniform(-1.0, 1.0, size=(n + n_test, l))
        y = sparse_cubic(rng, X)
        out.append(_split(X, y, n))
    return out


def paper_shape(n_train=102_400, n_features=1024, seed_offset=0) -> Dataset:
    """Stand-in for the speed-up study's dummy data: U[-1, 1] features and a
    sparse cubic target (the paper does not state its distribution)."""
    rng = np.random.default_rng(BASE_SEED + 10 * 5 + seed_offset)
    X = rng.uniform(-1.0, 1.0, size=(n_train, n_features))
    y = sparse_cubic(rng, X)
    return Dataset(X, y, np.zeros((0, n_features)), np.zeros(0))


def evolution_seed(workload_index: int) -> int:
    """Philox key word 0 for a workload; key word 1 is the run index."""
    return (BASE_SEED + 100 * workload_index) & 0xFFFFFFFF
