"""The paper's file formats (Section 3.3): fitness cases as text, one
instance per row, the feature values in columns and the target in the last
column; and, per run, two text files with the train fitness of the best
individual of every generation and the test fitness of the same individual.
"""
from __future__ import annotations

import numpy as np

from . import synth


def read_cases(path: str) -> tuple[np.ndarray, np.ndarray]:
    """(X [n][l], y [n]) from a text file: whitespace- or comma-separated
    numbers, one instance per row, the target last.  Blank lines and lines
    starting with '#' are skipped."""
    rows = []
    with open(path) as f:
        for line in f:
            text = line.strip()
            if not text or text.startswith("#"):
                continue
            rows.append([float(v) for v in text.replace(",", " ").split()])
    if not rows:
        raise ValueError(f"{path}: no instances")
    width = len(rows[0])
    if width < 2 or any(len(r) != width for r in rows):
        raise ValueError(f"{path}: every row needs the same number (>= 2) of columns")
    a = np.asarray(rows, dtype=np.float64)
    return np.ascontiguousarray(a[:, :-1]), np.ascontiguousarray(a[:, -1])


def read_dataset(train_path: str, test_path: str | None = None) -> synth.Dataset:
    Xtr, ytr = read_cases(train_path)
    if test_path:
        Xte, yte = read_cases(test_path)
        if Xte.shape[1] != Xtr.shape[1]:
            raise ValueError("train and test files have different numbers of features")
    else:
        Xte, yte = np.zeros((0, Xtr.shape[1])), np.zeros(0)
    return synth.Dataset(Xtr, ytr, Xte, yte)


def write_fitness_files(stats: np.ndarray, train_path: str, test_path: str) -> None:
    """One line per generation (0 .. G): the best train RMSE, and the test
    RMSE of that same individual, from the per-generation summaries."""
    with open(train_path, "w") as f:
        for v in stats["best_train_rmse"]:
            f.write(f"{float(v):.17g}\n")
    with open(test_path, "w") as f:
        for v in stats["best_test_rmse"]:
            f.write(f"{float(v):.17g}\n")
