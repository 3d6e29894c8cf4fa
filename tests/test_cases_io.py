"""The paper's text formats (Section 3.3): fitness cases with the target in
the last column; per-generation fitness files.  CPU tests of the reader and
writer; a GPU test of the command line end to end."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2106_04034_amd import cases, gsgp
from tests.conftest import ROOT


def test_read_cases_formats(tmp_path):
    p = tmp_path / "train.txt"
    p.write_text("# x0 x1 y\n1 2 3\n\n4,5,6\n-1.5e-3\t2 0.25\n")
    X, y = cases.read_cases(str(p))
    assert X.shape == (3, 2) and X.flags["C_CONTIGUOUS"]
    assert np.array_equal(X, [[1, 2], [4, 5], [-1.5e-3, 2]]) and np.array_equal(y, [3, 6, 0.25])


@pytest.mark.parametrize("text", ["", "1\n2\n", "1 2 3\n4 5\n"])
def test_read_cases_rejects_bad_files(tmp_path, text):
    p = tmp_path / "bad.txt"
    p.write_text(text)
    with pytest.raises(ValueError):
        cases.read_cases(str(p))


def test_read_dataset_checks_feature_counts(tmp_path):
    (tmp_path / "a.txt").write_text("1 2 3\n4 5 6\n")
    (tmp_path / "b.txt").write_text("1 2\n")
    d = cases.read_dataset(str(tmp_path / "a.txt"))
    assert d.X_test.shape == (0, 2) and d.y_test.shape == (0,)
    with pytest.raises(ValueError):
        cases.read_dataset(str(tmp_path / "a.txt"), str(tmp_path / "b.txt"))


def test_write_fitness_files_round_trip(tmp_path):
    st = np.zeros(4, dtype=gsgp.STATS_DTYPE)
    st["best_train_rmse"] = [0.5, 0.25, 0.25, 1 / 3]
    st["best_test_rmse"] = [0.75, 0.5, 0.125, 0.1]
    cases.write_fitness_files(st, str(tmp_path / "tr.txt"), str(tmp_path / "te.txt"))
    assert np.array_equal(np.loadtxt(tmp_path / "tr.txt"), st["best_train_rmse"])
    assert np.array_equal(np.loadtxt(tmp_path / "te.txt"), st["best_test_rmse"])


@pytest.mark.gpu
def test_command_line_end_to_end(tmp_path):
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, size=(700, 3))
    y = X[:, 0] * X[:, 1] + 0.5 * X[:, 2]
    np.savetxt(tmp_path / "train.txt", np.column_stack([X[:500], y[:500]]))
    np.savetxt(tmp_path / "test.txt", np.column_stack([X[500:], y[500:]]))
    out_tr, out_te = tmp_path / "fit_train.txt", tmp_path / "fit_test.txt"
    args = ["-train_file", str(tmp_path / "train.txt"), "-test_file", str(tmp_path / "test.txt"),
            "--population", "64", "--pool", "32", "--generations", "12", "--precision", "fp64", "--seed", "5",
            "--out-train", str(out_tr), "--out-test", str(out_te)]
    res = subprocess.run([sys.executable, "-m", "paper_2106_04034_amd", *args], cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    tr, te = np.loadtxt(out_tr), np.loadtxt(out_te)
    assert tr.shape == (13,) and te.shape == (13,)
    assert np.all(np.diff(tr) <= 0)
    # the same run through the binding gives the same summaries
    d = cases.read_dataset(str(tmp_path / "train.txt"), str(tmp_path / "test.txt"))
    s = gsgp.Settings(pop_size=64, pool_size=32, n_generations_max=12, seed=5, precision=gsgp.FP64)
    R = gsgp.Runner(s, [d])
    R.eval_population()
    R.generation(12)
    st = R.stats(0, 0, 13)
    R.close()
    assert np.array_equal(tr, st["best_train_rmse"]) and np.array_equal(te, st["best_test_rmse"])
