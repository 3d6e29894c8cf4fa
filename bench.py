"""Benchmark of the GSGP hot path on one MI355X.

A step is one whole GSGP run of the workload (Algorithm 1 of the GSGP-CUDA
paper, arXiv 2106.04034): genome generation, interpretation of population and
random-tree pool, initial fitness, then G generations of selection, GSM/GSC,
fitness and survival.  Inputs are resident in HBM before timing starts.

Default workload (single_fp32_100k): 100,000 train / 25,000 test cases,
20 features U[-1, 1], sparse cubic target + N(0, 0.05), population 1,024,
pool 1,024, 1,000 generations, FP32 semantics.

Prints one JSON line: offspring semantic elements/s (m * n_all * G per step),
the roofline of the dominant kernel (variation + fitness partials) from HIP
events on the library stream, and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_vary_single_fp32_100k_pmc.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2106_04034_amd", "csrc", "kernels.hip")


def kernel_digest() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def distinct_rows(rec: np.ndarray):
    """Distinct parent and pool rows one generation's records read."""
    xo = rec["op"] == 1
    parents = np.union1d(rec["p1"], rec["p2"][xo])
    pool = np.union1d(rec["r1"], rec["r2"][~xo])
    return parents.size, pool.size


def vary_bytes(rec: np.ndarray, n_all: int, s: int, m: int, n_chunks: int) -> int:
    """Algorithmic bytes of one variation launch: each offspring row written
    once, each distinct parent and pool row and the target read once, the
    chunk partial sums written and the records read."""
    u_p, u_r = distinct_rows(rec)
    return s * n_all * (m + u_p + u_r + 1) + 8 * m * n_chunks + 32 * m


def traffic_from_profile(per_launch_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; None otherwise."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_digest():
        return None
    return float(t.group(1))


def cpu_baseline(workload, data, G: int, seed: int, frac: int = 4, g_sample: int = 30):
    """The FP64 CPU oracle on a case slice of the same workload (all of m, r,
    k; 1/frac of the train and test cases), timed for initialisation and
    g_sample generations on every host core, then scaled linearly in the
    number of cases to a full step."""
    from oracle import oracle as orc
    cores = len(os.sched_getaffinity(0))
    orc.set_threads(cores)
    ntr = data.X_train.shape[0] // frac
    nte = data.X_test.shape[0] // frac
    Xtr, ytr = data.X_train[:ntr], data.y_train[:ntr]
    Xte, yte = data.X_test[:nte], data.y_test[:nte]
    cfg = orc.Config(pop_size=workload.pop_size, pool_size=workload.pool_size,
                     genome_len=workload.genome_len, seed=seed)
    t0 = time.perf_counter()
    state = orc.initial_state(cfg, Xtr, ytr, Xte, yte)
    t1 = time.perf_counter()
    _, _, S_tr, S_te, R_tr, R_te, F, Ft = state
    for g in range(1, g_sample + 1):
        rec = orc.select(cfg, g, F)
        O_tr, O_te = orc.vary(rec, S_tr, R_tr), orc.vary(rec, S_te, R_te)
        F_O, Ft_O = orc.rmse_rows(O_tr, ytr), orc.rmse_rows(O_te, yte)
        orc.survive(F, Ft, F_O, Ft_O, S_tr, O_tr, S_te, O_te)
        S_tr, S_te, F, Ft = O_tr, O_te, F_O, Ft_O
    t2 = time.perf_counter()
    scale = (data.X_train.shape[0] + data.X_test.shape[0]) / (ntr + nte)
    t_step = scale * ((t1 - t0) + (t2 - t1) / g_sample * G)
    n_all = data.X_train.shape[0] + data.X_test.shape[0]
    value = workload.pop_size * n_all * G / t_step
    sample = (f"FP64 oracle, {cores} threads: case slice 1/{frac} ({ntr} train + {nte} test), "
              f"m=r={workload.pop_size}, init {t1 - t0:.2f} s + {g_sample} generations "
              f"{t2 - t1:.2f} s, scaled linearly in cases to init + {G} generations")
    return {"value": value, "unit": "offspring elements/s", "cores": cores, "kind": "oracle",
            "sample": sample, "gen_elements_per_s": workload.pop_size * (ntr + nte) * g_sample / (t2 - t1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single_fp32_100k")
    ap.add_argument("--stage-gens", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--generations", type=int, default=0,
                    help="override the workload's generation count (profiling runs only)")
    ap.add_argument("--launch", default="",
                    help="variation launch shape waves,offspring_per_block,xcd_remap,max_blocks "
                         "(skips autotuning)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(a single run shards over fitness cases only in design, see the design notes)",
              file=sys.stderr)
        return 2

    import torch
    from paper_2106_04034_amd import gsgp, synth

    wl = synth.WORKLOADS[args.workload]
    if wl.name != "single_fp32_100k":
        print(f"bench.py: workload {wl.name} has no bench line; use the default", file=sys.stderr)
        return 2
    data = synth.single_run(wl.n_train, wl.n_test, wl.n_features)
    G = args.generations or wl.generations
    seed = synth.evolution_seed(1)
    prec = gsgp.PRECISIONS[wl.precision]
    settings = gsgp.Settings(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                             n_generations_max=G, tournament_size=wl.tournament_size,
                             p_crossover=wl.p_crossover, mutation_step=wl.mutation_step,
                             precision=prec, seed=seed)
    stream = torch.cuda.Stream()
    R = gsgp.Runner(settings, [data], stream=stream)
    n_all = wl.n_train + wl.n_test
    m = wl.pop_size
    s_bytes = 8 if prec == gsgp.FP64 else 4

    R.eval_population()
    if args.launch:
        w, o, x, g = (int(v) for v in args.launch.split(","))
        R.set_launch(w, o, x, g)
        tuned = {"waves": w, "offspring_per_block": o, "xcd_remap": x, "max_blocks": g}
    else:
        tuned = None if args.no_autotune else R.autotune()

    def step():
        R.eval_population()
        R.generation(G, stats=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = m * n_all * G * args.steps / elapsed
    final = R.stats(0, G, 1)[0]

    # initialisation alone (genomes, interpreter, sigmoid, initial fitness)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    R.eval_population()
    torch.cuda.synchronize()
    eval_ms = (time.perf_counter() - e0) * 1e3

    # per-stage HIP-event timing of the generation's kernels on the library stream
    ng = min(args.stage_gens, G)
    stages = R.time_stages(ng)
    rec = R.records(0, 1, ng)
    chunk = 4096 // s_bytes  # canonical chunk: 4 KiB of a semantic row
    n_chunks = -(-(-(-wl.n_train // 64) * 64) // chunk) + -(-(-(-wl.n_test // 64) * 64) // chunk)
    per_launch = float(np.mean([vary_bytes(rec[g], n_all, s_bytes, m, n_chunks) for g in range(ng)]))
    u = np.array([distinct_rows(rec[g]) for g in range(ng)])
    achieved = per_launch / (stages["vary_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profile(per_launch)
    gen_rate = m * n_all / (stages["generation_ms"] * 1e-3)

    out = {
        "metric": "offspring semantic elements/s (whole GSGP run incl. initialisation)",
        "value": value,
        "unit": "offspring elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_train": wl.n_train, "n_test": wl.n_test,
                   "n_features": wl.n_features, "pop_size": m, "pool_size": wl.pool_size,
                   "genome_len": wl.genome_len, "generations": G, "tournament_size": wl.tournament_size,
                   "p_crossover": wl.p_crossover, "mutation_step": wl.mutation_step,
                   "precision": wl.precision, "launch": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_vary (GSM/GSC + chunk partial sums)",
                     "alg_bytes_per_launch": per_launch, "launch_ms": stages["vary_ms"],
                     "distinct_parent_rows": float(u[:, 0].mean()),
                     "distinct_pool_rows": float(u[:, 1].mean())},
        "stages_ms": {k: round(v, 5) for k, v in stages.items()},
        "eval_population_ms": eval_ms,
        "generation_elements_per_s": gen_rate,
        "final_best_train_rmse": float(final["best_train_rmse"]),
        "final_best_test_rmse": float(final["best_test_rmse"]),
    }
    R.close()
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, data, G, seed)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["gen_elements_per_s"] = cb["gen_elements_per_s"]
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
