"""Shared set-up for the GPU parity tests: one seeded dataset feeds both the
HIP library (through its C ABI) and the CPU oracle."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc
from paper_2106_04034_amd import gsgp, synth


def oracle_config(s: gsgp.Settings, run_id: int = 0) -> orc.Config:
    return orc.Config(pop_size=s.pop_size, pool_size=s.pool_size, genome_len=s.genome_len,
                      tournament_size=s.tournament_size, p_crossover=s.p_crossover,
                      mutation_step=s.mutation_step, ms_random=s.ms_random,
                      p_function=s.p_function, p_feature=s.p_feature, erc_lo=s.erc_lo,
                      erc_hi=s.erc_hi, seed=s.seed, run_id=run_id)


def dataset(n_train: int, n_test: int, l: int, seed: int = 0) -> synth.Dataset:
    rng = np.random.default_rng(1000 + seed)
    X = rng.uniform(-1.0, 1.0, size=(n_train + n_test, l))
    y = synth.sparse_cubic(rng, X, n_vars=min(6, l), noise=0.05)
    return synth.Dataset(X[:n_train].copy(), y[:n_train].copy(), X[n_train:].copy(), y[n_train:].copy())


def rel_err(a, b, floor):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))) if a.size else 0.0


def concat_sem(S_tr, S_te):
    return np.concatenate([S_tr, S_te], axis=1)


def records_equal(gpu_rec, orc_rec) -> bool:
    for f in ("op", "p1", "p2", "r1", "r2", "ms"):
        if not np.array_equal(gpu_rec[f], orc_rec[f]):
            return False
    return True


def oracle_records(rec):
    """A device record array as the oracle's record dtype (same layout)."""
    out = np.zeros(rec.shape, dtype=orc.RECORD_DTYPE)
    for f in ("op", "p1", "p2", "r1", "r2", "ms"):
        out[f] = rec[f]
    return out


def elite_of(stats):
    """(copied, src, dst) rows from device summaries."""
    return np.stack([stats["elite_copied"], stats["elite_src"], stats["elite_dst"]], axis=-1).astype(np.int32)
