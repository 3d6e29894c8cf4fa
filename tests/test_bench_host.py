"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte count of the variation kernel, the interpreter's gene-step count and
the use of the committed counter summary.  Each count is checked against a
plain per-item loop."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from paper_2106_04034_amd import gsgp  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def _records(rng, m, r, p_xo):
    rec = np.zeros(m, dtype=gsgp.RECORD_DTYPE)
    xo = rng.random(m) < p_xo
    rec["op"] = xo.astype(np.int32)
    rec["p1"] = rng.integers(0, m, m)
    rec["p2"] = np.where(xo, rng.integers(0, m, m), -1)
    rec["r1"] = rng.integers(0, r, m)
    rec["r2"] = np.where(xo, -1, rng.integers(0, r, m))
    return rec


@pytest.mark.parametrize("p_xo", [0.0, 0.5, 1.0])
def test_variation_bytes_count_each_distinct_row_once(p_xo):
    rng = np.random.default_rng(3)
    m, r, n_all, s = 200, 150, 1000, 4
    rec = _records(rng, m, r, p_xo)
    parents, pool = set(), set()
    for x in rec:
        parents.add(int(x["p1"]))
        if x["op"] == 1:
            parents.add(int(x["p2"]))
            pool.add(int(x["r1"]))
        else:
            pool.add(int(x["r1"]))
            pool.add(int(x["r2"]))
    assert bench.distinct_rows(rec) == (len(parents), len(pool))
    want = s * n_all * (m + len(parents) + len(pool) + 1) + 32 * m
    assert bench.vary_bytes(rec, n_all, s, m) == want


def _steps_one(genome):
    depth = ops = last = 0
    for c in genome:
        if c >= 0 or c == -5:
            depth += 1
            ops += 1
        elif depth >= 2:
            depth -= 1
            ops += 1
            last = ops
    return last


@pytest.mark.parametrize("k", [1, 7, 127])
def test_gene_steps_count_pushes_and_valid_functions_up_to_the_last_function(k):
    cfg = orc.Config(pop_size=40, pool_size=8, genome_len=k, seed=11)
    codes, _ = orc.genomes(cfg, 5, orc.TAG_POPULATION, 40)
    assert bench.gene_steps(codes) == sum(_steps_one(g) for g in codes)
    # hand-made: "x0 x1 + c -" is 5 steps; a lone push and "x0" followed by
    # functions on a one-value stack count nothing (no function runs)
    hand = np.array([[0, 1, -1, -5, -2], [-1, -1, -1, -1, 0], [-1, 0, -1, -1, -1]], np.int32)
    assert bench.gene_steps(hand) == 5


def test_interpreter_feature_bytes_count_feature_pushes_up_to_the_last_function():
    # "x0 x1 + c - x2": the trailing x2 never runs; x0 and x1 are read per case
    hand = np.array([[0, 1, -1, -5, -2, 2], [3, -1, -1, -1, 0, 1], [-5, 4, -3, 0, -4, -4]], np.int32)
    steps, feats = bench.gene_work_rows(hand)
    assert list(steps) == [5, 0, 5] and list(feats) == [2, 0, 2]
    rate = bench.interpreter_rate(hand, 10, 1.0)
    assert rate["feature_bytes"] == 4 * 10 * 8
    assert abs(rate["feature_GBps"] - 320 / 1e-3 / 1e9) < 1e-12


def test_traffic_comes_from_the_counter_summary_only_for_the_same_kernel_sources(monkeypatch, tmp_path):
    path = tmp_path / "k_vary_x_pmc.md"
    path.write_text("# summary\n\nhbm_bytes_per_launch: 1234567890\nkernel_source_sha256_16: 0123456789abcdef\n")
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0123456789abcdef")
    assert bench.traffic_from_profile(str(path)) == 1234567890.0
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 16)
    assert bench.traffic_from_profile(str(path)) is None
    assert bench.traffic_from_profile(str(tmp_path / "missing.md")) is None
    for w, p in bench.PMC_SUMMARIES.items():  # committed summaries carry both fields
        if os.path.exists(p):
            text = open(p).read()
            assert re.search(r"kernel_source_sha256_16:\s*[0-9a-f]{16}", text), w
            assert re.search(r"hbm_bytes_per_launch:\s*[0-9.eE+]+", text), w


def test_interpreter_rate_weights_each_genome_by_its_run_cases():
    rng = np.random.default_rng(3)
    codes = rng.integers(-5, 4, size=(6, 40)).astype(np.int32)
    n = np.array([10, 10, 200, 200, 7, 7])
    rate = bench.interpreter_rate_rows(codes, n, 1.0)
    assert rate["gene_steps"] == sum(bench.gene_steps(codes[j:j + 1]) * int(n[j]) for j in range(6))
    assert bench.interpreter_rate(codes, 50, 1.0)["gene_steps"] == bench.gene_steps(codes) * 50


def test_kernel_digest_covers_the_kernels_and_their_shared_headers(tmp_path, monkeypatch):
    for name in ("kernels.hip", "common.hpp", "device.hpp"):
        (tmp_path / name).write_bytes(open(os.path.join(os.path.dirname(bench.KERNEL_SRC), name), "rb").read())
    monkeypatch.setattr(bench, "KERNEL_SRC", str(tmp_path / "kernels.hip"))
    for name in ("common.hpp", "device.hpp"):
        d0 = bench.kernel_digest()
        with open(tmp_path / name, "ab") as f:
            f.write(b"\n")
        assert bench.kernel_digest() != d0, name
