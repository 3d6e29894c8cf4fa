"""Benchmark of the GSGP hot path on one MI355X.

A step is one whole GSGP run of the workload (Algorithm 1 of the GSGP-CUDA
paper, arXiv 2106.04034): genome generation, interpretation of population and
random-tree pool, initial fitness, then G generations of selection, GSM/GSC,
fitness and survival.  Inputs are resident in HBM before timing starts.

Default workload (batched_256): 256 independent runs of uneven size in one
handle (n per run log-uniform in [200, 50,000], test n/4, 4..32 features
U[-1, 1], sparse cubic target + N(0, 0.05); population 256, pool 256, 300
generations, FP32 semantics with compensated fitness sums, 16 generations
per HIP graph).  A step is one whole batched run of all 256.  It prints one
JSON line: offspring semantic elements/s over all runs, the roofline of the
variation kernel (one launch over all runs) from HIP events on the library
stream, runs/hour against the plain per-run form (FP64, one handle per run,
no graph) and a per-run FP32-Kahan form, the best-fitness error against an
FP64 replay of every lineage and against the CPU oracle on four runs, and
the CPU oracle's rate on a bounded sample of the runs.

Other workloads (--workload) print their own line:
  single_fp32_100k one run of 100,000 / 25,000 cases, m = r = 1,024, 1,000
                   generations, FP32;
  large_fp32_1m    the same measurement on 1,000,000 / 250,000 cases, m = 2,048;
  plain_fp64_500x8 the same measurement on the small FP64 workload;
  precision_1m     FP32 and FP32-Kahan runs against an FP64 replay of the same
                   lineage: relative fitness drift per generation;
  paper_shape_k127 / _k1023 / _k2047
                   the shape of the paper's speed-up study (Section 3.1): stage
                   times in its categories next to the single-thread oracle.
--local-search turns on GSGP with local search (least-squares scaling of
every offspring) for the single-run and batched workloads.
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
BASELINE_METRIC = "offspring semantic elements/s + % HBM roofline; batched FP32 vs plain, 1e-4 fitness"
# rocprofv3 counter summaries of the variation kernel, per workload
PMC_SUMMARIES = {w: os.path.join(ROOT, "profiles", f"k_vary_{w}_pmc.md")
                 for w in ("single_fp32_100k", "large_fp32_1m", "batched_256")}
KERNEL_SRC = os.path.join(ROOT, "paper_2106_04034_amd", "csrc", "kernels.hip")


def kernel_digest() -> str:
    """Digest of the variation kernel's sources: the translation unit that
    holds it and the headers of shared constants, layouts and device helpers
    it includes (the interpreter's own unit is not part of it)."""
    h = hashlib.sha256()
    d = os.path.dirname(KERNEL_SRC)
    for path in (KERNEL_SRC, os.path.join(d, "common.hpp"), os.path.join(d, "device.hpp")):
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def distinct_rows(rec: np.ndarray):
    """Distinct parent and pool rows one generation's records read."""
    xo = rec["op"] == 1
    parents = np.union1d(rec["p1"], rec["p2"][xo])
    pool = np.union1d(rec["r1"], rec["r2"][~xo])
    return parents.size, pool.size


def vary_bytes(rec: np.ndarray, n_all: int, s: int, m: int) -> int:
    """Algorithmic bytes of one variation launch: each offspring row written
    once, each distinct parent and pool row and the target read once, and
    the variation records read (the chunk partial sums the kernel also
    writes are not the method's bytes and are not counted)."""
    u_p, u_r = distinct_rows(rec)
    return s * n_all * (m + u_p + u_r + 1) + 32 * m


FP64_VALU_OPS = 78.6e12 / 2  # FP64 vector operations/s (the vendor FLOP/s counts an FMA as two)
# L2 read bandwidth into the CUs: 8 XCDs x 16 L2 channels x 128 bytes per
# clock at 2.4 GHz (the path that feeds the interpreter its feature rows)
L2_READ_GBPS = 8 * 16 * 128 * 2.4
PROBE = os.path.join(ROOT, "paper_2106_04034_amd", "copy_probe")


def streaming_probe(mode: str):
    """GB/s of the streaming probe (1 GiB per array, 10 launches) on this
    device, run as a child process; None when the probe is not built."""
    if not os.path.exists(PROBE):
        return None
    import subprocess
    res = subprocess.run([PROBE, str(1 << 30), "10", mode], capture_output=True, text=True, timeout=120)
    m = re.search(r"GBps=([0-9.]+)", res.stdout)
    return float(m.group(1)) if res.returncode == 0 and m else None


def gene_steps(codes: np.ndarray) -> int:
    """Algorithmic interpreter work of a set of genomes: per genome, the
    pushes and valid functions up to its last valid function (the genes
    that shape its output; skipped functions and trailing pushes cost
    nothing once compiled).  Counted per case."""
    return int(gene_steps_rows(codes).sum())


def gene_steps_rows(codes: np.ndarray) -> np.ndarray:
    """gene_steps of each genome row."""
    return gene_work_rows(codes)[0]


def gene_work_rows(codes: np.ndarray):
    """Per genome row: its gene-steps and the feature pushes among them (each
    reads one feature value per case)."""
    depth = np.zeros(codes.shape[0], np.int64)
    ops = np.zeros(codes.shape[0], np.int64)
    feats = np.zeros(codes.shape[0], np.int64)
    last = np.zeros(codes.shape[0], np.int64)
    last_feats = np.zeros(codes.shape[0], np.int64)
    for q in range(codes.shape[1]):
        c = codes[:, q]
        push = (c >= 0) | (c == -5)
        fn = ~push & (depth >= 2)
        ops += push | fn
        feats += c >= 0
        depth += push.astype(np.int64) - fn.astype(np.int64)
        last = np.where(fn, ops, last)
        last_feats = np.where(fn, feats, last_feats)
    return last, last_feats


def interpreter_rate(codes: np.ndarray, n_cases: int, ms: float) -> dict:
    return interpreter_rate_rows(codes, np.full(codes.shape[0], n_cases), ms)


def interpreter_rate_rows(codes: np.ndarray, n_cases: np.ndarray, ms: float) -> dict:
    """Gene-steps/s of ComputeSemantics when genome row j runs on n_cases[j]
    cases (runs of uneven size in one handle)."""
    rows, feats = gene_work_rows(codes)
    n = np.asarray(n_cases, np.int64)
    steps = int(np.sum(rows * n))
    feature_bytes = int(np.sum(feats * n)) * 8
    rate = steps / (ms * 1e-3)
    feature_gbps = feature_bytes / (ms * 1e-3) / 1e9
    return {"bound": "l2", "gene_steps": steps, "gene_steps_per_s": rate,
            "feature_bytes": feature_bytes, "feature_GBps": feature_gbps, "peak_l2_read_GBps": L2_READ_GBPS,
            "frac": feature_gbps / L2_READ_GBPS, "peak_fp64_ops_per_s": FP64_VALU_OPS,
            "frac_fp64_ops": rate / FP64_VALU_OPS, "compute_semantics_ms": ms,
            "note": "one gene-step is one push or one valid function on one case; feature_bytes are the FP64 "
                    "feature values those steps read (8 bytes per feature push per case), which come from L2 "
                    "through each CU's vector memory path, the unit the interpreter's counters show saturated"}


def traffic_from_profile(path: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; None otherwise."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_digest():
        return None
    return float(t.group(1))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, data, G: int, seed: int, frac: int = 4, g_sample: int = 30, threads: int = 0,
                 local_search: bool = False):
    """The FP64 CPU oracle on a case slice of the same workload (all of m, r,
    k; 1/frac of the train and test cases), timed for initialisation and
    g_sample generations on `threads` host cores (0: every core), then
    scaled linearly in the number of cases to a full step."""
    from oracle import oracle as orc
    all_cores = len(os.sched_getaffinity(0))
    cores = threads or all_cores
    orc.set_threads(cores)
    ntr = data.X_train.shape[0] // frac
    nte = data.X_test.shape[0] // frac
    Xtr, ytr = data.X_train[:ntr], data.y_train[:ntr]
    Xte, yte = data.X_test[:nte], data.y_test[:nte]
    cfg = orc.Config(pop_size=workload.pop_size, pool_size=workload.pool_size,
                     genome_len=workload.genome_len, seed=seed, local_search=local_search)
    t0 = time.perf_counter()
    state = orc.initial_state(cfg, Xtr, ytr, Xte, yte)
    t1 = time.perf_counter()
    _, _, S_tr, S_te, R_tr, R_te, F, Ft = state
    for g in range(1, g_sample + 1):
        rec = orc.select(cfg, g, F)
        O_tr, O_te = orc.vary(rec, S_tr, R_tr), orc.vary(rec, S_te, R_te)
        if local_search:
            a, b = orc.ls_fit(O_tr, ytr)
            O_tr, O_te = orc.ls_apply(O_tr, a, b), orc.ls_apply(O_te, a, b)
        F_O, Ft_O = orc.rmse_rows(O_tr, ytr), orc.rmse_rows(O_te, yte)
        orc.survive(F, Ft, F_O, Ft_O, S_tr, O_tr, S_te, O_te)
        S_tr, S_te, F, Ft = O_tr, O_te, F_O, Ft_O
    t2 = time.perf_counter()
    scale = (data.X_train.shape[0] + data.X_test.shape[0]) / (ntr + nte)
    t_step = scale * ((t1 - t0) + (t2 - t1) / g_sample * G)
    n_all = data.X_train.shape[0] + data.X_test.shape[0]
    value = workload.pop_size * n_all * G / t_step
    orc.set_threads(all_cores)
    sample = (f"FP64 oracle, {cores} threads: case slice 1/{frac} ({ntr} train + {nte} test), "
              f"m=r={workload.pop_size}, init {t1 - t0:.2f} s + {g_sample} generations "
              f"{t2 - t1:.2f} s, scaled linearly in cases to init + {G} generations")
    return {"value": value, "unit": "offspring elements/s", "cores": cores, "kind": "oracle",
            "sample": sample, "gen_elements_per_s": workload.pop_size * (ntr + nte) * g_sample / (t2 - t1)}


def settings_for(gsgp, wl, G, precision, seed, flags=0):
    return gsgp.Settings(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                         n_generations_max=G, tournament_size=wl.tournament_size,
                         p_crossover=wl.p_crossover, mutation_step=wl.mutation_step,
                         precision=precision, seed=seed, flags=flags)


def bench_single(args, wl, data, seed) -> dict:
    """Whole runs of one workload; elements/s, roofline and CPU baseline."""
    import torch
    from paper_2106_04034_amd import gsgp

    G = args.generations or wl.generations
    prec = gsgp.PRECISIONS[wl.precision]
    flags = gsgp.FLAG_LOCAL_SEARCH if args.local_search else 0
    R = gsgp.Runner(settings_for(gsgp, wl, G, prec, seed, flags), [data], stream=torch.cuda.Stream())
    n_all = data.X_train.shape[0] + data.X_test.shape[0]
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
    eval_stages = R.time_eval()

    # per-stage HIP-event timing of the generation's kernels on the library stream
    ng = min(args.stage_gens, G)
    stages = R.time_stages(ng)
    rec = R.records(0, 1, ng)
    n_tr, n_te = data.X_train.shape[0], data.X_test.shape[0]
    per_launch = float(np.mean([vary_bytes(rec[g], n_all, s_bytes, m) for g in range(ng)]))
    u = np.array([distinct_rows(rec[g]) for g in range(ng)])
    achieved = per_launch / (stages["vary_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profile(PMC_SUMMARIES[wl.name]) if wl.name in PMC_SUMMARIES and not args.local_search \
        else None
    # the 3 : 1 read / write streaming rate the same device reaches, as a
    # practical ceiling next to the vendor peak
    probes = {mode: streaming_probe(mode) for mode in ("mix31", "mix31nt")}
    codes, _ = R.genomes(0)
    interp = interpreter_rate(codes, n_all, eval_stages["compute_semantics_ms"])
    gen_rate = m * n_all / (stages["generation_ms"] * 1e-3)
    # per-generation distribution: one graph launch per generation, HIP
    # events on the library stream around each
    per_gen = []
    n_single = max(1, min(50, G - R.current_generation()))
    if R.current_generation() + n_single > G:  # no generation left: restart the run
        R.eval_population()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_single)]
    for a, b in ev:
        a.record(R.stream)
        R.generation(1, stats=False)
        b.record(R.stream)
    torch.cuda.synchronize()
    per_gen = np.array([a.elapsed_time(b) for a, b in ev])
    R.close()

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
        "dtype": "f64" if prec == gsgp.FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_train": n_tr, "n_test": n_te,
                   "n_features": data.X_train.shape[1], "pop_size": m, "pool_size": wl.pool_size,
                   "genome_len": wl.genome_len, "generations": G, "tournament_size": wl.tournament_size,
                   "p_crossover": wl.p_crossover, "mutation_step": wl.mutation_step,
                   "precision": wl.precision, "local_search": bool(args.local_search), "launch": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_vary (GSM/GSC + chunk partial sums)",
                     "alg_bytes_per_launch": per_launch, "launch_ms": stages["vary_ms"],
                     "distinct_parent_rows": float(u[:, 0].mean()),
                     "distinct_pool_rows": float(u[:, 1].mean()),
                     # what a kernel without cross-offspring reuse would move:
                     # three operand rows read and one written per offspring
                     "operand_stream_GBps": 4 * s_bytes * m * n_all / (stages["vary_ms"] * 1e-3) / 1e9,
                     "probe_3to1_GBps": probes,
                     "frac_of_probe": {k: achieved / v for k, v in probes.items() if v}},
        "interpreter": interp,
        "stages_ms": {k: round(v, 5) for k, v in stages.items()},
        "eval_population_ms": eval_ms,
        "eval_stages_ms": {k: round(v, 5) for k, v in eval_stages.items()},
        "generation_elements_per_s": gen_rate,
        "generation_ms_single_launches": {"mean": float(per_gen.mean()), "p50": float(np.median(per_gen)),
                                          "max": float(per_gen.max()), "n": int(per_gen.size)},
        "final_best_train_rmse": float(final["best_train_rmse"]),
        "final_best_test_rmse": float(final["best_test_rmse"]),
    }
    if not args.no_cpu_baseline:
        frac = 4 if n_all <= 200_000 else 32
        if n_all < 10_000:
            frac = 1
        cb = cpu_baseline(wl, data, G, seed, frac=frac, local_search=args.local_search)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["gen_elements_per_s"] = cb["gen_elements_per_s"]
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        # the sequential reference point (the paper compares with a sequential
        # CPU implementation): one thread on a smaller slice
        c1 = cpu_baseline(wl, data, G, seed, frac=frac * 4 if frac > 1 else 1, g_sample=10, threads=1,
                          local_search=args.local_search)
        out["cpu_baseline"]["one_thread"] = {k: c1[k] for k in ("value", "gen_elements_per_s", "sample")}
    return out


def bench_precision(args) -> dict:
    """FP32 and FP32-Kahan runs, each followed by an FP64 replay of the same
    lineage (records and survival decisions) on the GPU; relative fitness
    drift per generation for the best individual and over the population.
    The GPU FP64 form is parity-checked against the CPU oracle in the tests."""
    import torch
    from paper_2106_04034_amd import gsgp, synth

    wl = synth.WORKLOADS["precision_1m"]
    G = args.generations or wl.generations
    data = synth.large_run()
    seed = synth.evolution_seed(3)
    m = wl.pop_size
    report = {}
    for name, prec in (("fp32", gsgp.FP32), ("fp32_kahan", gsgp.FP32_KAHAN)):
        R = gsgp.Runner(settings_for(gsgp, wl, G, prec, seed), [data], stream=torch.cuda.Stream())
        R.eval_population()
        F32 = [R.fitness(0)[0]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(G):
            R.generation(1, stats=False)
            F32.append(R.fitness(0)[0])
        t32 = time.perf_counter() - t0
        rec = R.records(0, 1, G)
        elite = R.stats(0, 1, G)
        best = R.stats(0, 0, G + 1)["best_index"]
        R.close()
        R64 = gsgp.Runner(settings_for(gsgp, wl, G, gsgp.FP64, seed), [data], stream=torch.cuda.Stream())
        R64.eval_population()
        F64 = [R64.fitness(0)[0]]
        for g in range(G):
            R64.replay(rec[g:g + 1], elite[g:g + 1], stats=False)
            F64.append(R64.fitness(0)[0])
        R64.close()
        F32, F64 = np.array(F32), np.array(F64)
        drift = np.abs(F32 - F64) / F64
        best_drift = drift[np.arange(G + 1), best]
        report[name] = {
            "best_drift_max": float(best_drift.max()),
            "best_drift_final": float(best_drift[-1]),
            "median_drift_max": float(np.median(drift, axis=1).max()),
            "population_drift_max": float(drift.max()),
            "final_best_rmse_fp32": float(F32[-1][best[-1]]),
            "final_best_rmse_fp64_replay": float(F64[-1][best[-1]]),
            "best_drift_every_100": [float(best_drift[g]) for g in range(0, G + 1, 100)],
            "generation_loop_s_with_readback": t32,
        }
    ok = all(v["best_drift_final"] <= 1e-4 for v in report.values())
    return {"metric": "relative fitness drift vs FP64 replay of the same lineage",
            "value": report["fp32_kahan"]["best_drift_final"], "unit": "relative",
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": wl.name, "n_train": data.X_train.shape[0],
                       "n_test": data.X_test.shape[0], "n_features": data.X_train.shape[1],
                       "pop_size": m, "pool_size": wl.pool_size, "generations": G},
            "forms": report, "end_of_run_within_1e-4": ok}


def cpu_baseline_runs(wl, datasets, G: int, seed: int, pick, g_sample: int, threads: int = 0,
                      local_search: bool = False):
    """The FP64 CPU oracle on a fixed subset of the independent runs (every
    case of each picked run; initialisation and g_sample generations), on
    `threads` host cores (0: every core), scaled to all runs and G
    generations by the runs' offspring elements per generation."""
    from oracle import oracle as orc
    all_cores = len(os.sched_getaffinity(0))
    cores = threads or all_cores
    orc.set_threads(cores)
    t_init = t_gen = 0.0
    elems_pick = 0
    for j in pick:
        d = datasets[j]
        cfg = orc.Config(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                         seed=seed, run_id=j, local_search=local_search)
        t0 = time.perf_counter()
        _, _, S_tr, S_te, R_tr, R_te, F, Ft = orc.initial_state(cfg, d.X_train, d.y_train, d.X_test, d.y_test)
        t1 = time.perf_counter()
        for g in range(1, g_sample + 1):
            rec = orc.select(cfg, g, F)
            O_tr, O_te = orc.vary(rec, S_tr, R_tr), orc.vary(rec, S_te, R_te)
            if local_search:
                a, b = orc.ls_fit(O_tr, d.y_train)
                O_tr, O_te = orc.ls_apply(O_tr, a, b), orc.ls_apply(O_te, a, b)
            F_O, Ft_O = orc.rmse_rows(O_tr, d.y_train), orc.rmse_rows(O_te, d.y_test)
            orc.survive(F, Ft, F_O, Ft_O, S_tr, O_tr, S_te, O_te)
            S_tr, S_te, F, Ft = O_tr, O_te, F_O, Ft_O
        t2 = time.perf_counter()
        t_init += t1 - t0
        t_gen += (t2 - t1) / g_sample
        elems_pick += wl.pop_size * (d.X_train.shape[0] + d.X_test.shape[0])
    orc.set_threads(all_cores)
    elems_all = sum(wl.pop_size * (d.X_train.shape[0] + d.X_test.shape[0]) for d in datasets)
    scale = elems_all / elems_pick
    t_step = scale * (t_init + t_gen * G)
    sample = (f"FP64 oracle, {cores} threads: {len(pick)} of the {len(datasets)} runs (every case), "
              f"m=r={wl.pop_size}, init {t_init:.2f} s + {g_sample} generations {t_gen * g_sample:.2f} s, "
              f"scaled by offspring elements to all runs and init + {G} generations")
    return {"value": elems_all * G / t_step, "unit": "offspring elements/s", "cores": cores, "kind": "oracle",
            "sample": sample, "runs_per_hour": len(datasets) * 3600 / t_step,
            "gen_elements_per_s": elems_pick / t_gen}


def oracle_fitness_check(wl, datasets, G, seed, rec, elite, F_dev, picks, local_search=False):
    """The oracle follows the device lineage of the picked runs (replay mode,
    every case, FP64) for G generations; returns the relative error of the
    device's final fitness at the oracle's best index, the largest over the
    population, and the replay check's near-tie counts."""
    from oracle import oracle as orc
    worst_best = worst_all = 0.0
    ties = 0
    for j in picks:
        d = datasets[j]
        cfg = orc.Config(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                         seed=seed, run_id=j, local_search=local_search)
        orec = np.zeros(rec[j].shape, dtype=orc.RECORD_DTYPE)
        for f in ("op", "p1", "p2", "r1", "r2", "ms"):
            orec[f] = rec[j][f]
        el = np.stack([elite[j]["elite_copied"], elite[j]["elite_src"], elite[j]["elite_dst"]], axis=1)
        res = orc.run(cfg, d.X_train, d.y_train, d.X_test, d.y_test, G, drive=(orec, el))
        b = int(np.argmin(res.F))
        worst_best = max(worst_best, abs(F_dev[j][b] - res.F[b]) / res.F[b])
        worst_all = max(worst_all, float(np.max(np.abs(F_dev[j] - res.F) / res.F)))
        ties += sum(c["winner_mismatch"] + c["elite_mismatch"] for c in res.replay)
    return {"runs": [int(j) for j in picks], "best_rel_err_max": worst_best, "population_rel_err_max": worst_all,
            "near_tie_disagreements": ties}


def bench_batched(args) -> dict:
    """The metric's own comparison: 256 uneven runs in one batched
    FP32-Kahan handle (every stage one launch over all runs, 16 generations
    per HIP graph) against the plain per-run form (one FP64 handle per run,
    launches one by one, no graph) and a per-run FP32-Kahan form.  A step is
    one whole batched run: initialisation of every run and G generations.
    The fitness error of the batched runs is measured against an FP64 replay
    of their own lineages on the GPU (every run) and against the CPU oracle
    following the same lineages (four runs)."""
    import torch
    from paper_2106_04034_amd import gsgp, synth

    wl = synth.WORKLOADS["batched_256"]
    G = args.generations or wl.generations
    n_runs = args.runs or wl.runs
    datasets = synth.batched_runs(n_runs)
    seed = synth.evolution_seed(4)
    stream = torch.cuda.Stream()
    flags = gsgp.FLAG_LOCAL_SEARCH if args.local_search else 0
    n_all = sum(d.X_train.shape[0] + d.X_test.shape[0] for d in datasets)

    B = gsgp.Runner(settings_for(gsgp, wl, G, gsgp.FP32_KAHAN, seed, flags), datasets, stream=stream)
    B.eval_population()
    if args.launch:
        w, o, x, g = (int(v) for v in args.launch.split(","))
        B.set_launch(w, o, x, g)
        tuned = {"waves": w, "offspring_per_block": o, "xcd_remap": x, "max_blocks": g}
    else:
        tuned = None if args.no_autotune else B.autotune()

    def step():
        B.eval_population()
        B.generation(G, stats=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    value = wl.pop_size * n_all * G / t_step
    rec = [B.records(j, 1, G) for j in range(n_runs)]
    elite = [B.stats(j, 1, G) for j in range(n_runs)]
    final = np.stack([B.stats(j, G, 1)[0] for j in range(n_runs)])
    F_b = np.stack([B.fitness(j)[0] for j in range(n_runs)])
    # roofline of the batched variation launch: algorithmic bytes of every
    # run (distinct parent / pool rows from its records) over its launch
    # time from HIP events on the library stream
    B.eval_population()
    ng = min(G, args.stage_gens)
    stg = B.time_stages(ng)
    alg = 0.0
    for j, d in enumerate(datasets):
        n_tr, n_te = d.X_train.shape[0], d.X_test.shape[0]
        rj = B.records(j, 1, ng)
        alg += float(np.mean([vary_bytes(rj[g], n_tr + n_te, 4, wl.pop_size) for g in range(ng)]))
    eval_stages = B.time_eval()
    codes = np.concatenate([B.genomes(j)[0] for j in range(n_runs)])
    n_cases = np.repeat([d.X_train.shape[0] + d.X_test.shape[0] for d in datasets], wl.pop_size + wl.pool_size)
    B.close()
    achieved = alg / (stg["vary_ms"] * 1e-3) / 1e9
    probes = {mode: streaming_probe(mode) for mode in ("mix31", "mix31nt")}

    # FP64 replay of every run's lineage on the GPU
    R64 = gsgp.Runner(settings_for(gsgp, wl, G, gsgp.FP64, seed, flags), datasets, stream=stream)
    R64.eval_population()
    R64.replay(np.stack(rec), np.stack(elite), stats=False)
    F_64 = np.stack([R64.fitness(j)[0] for j in range(n_runs)])
    R64.close()
    idx = final["best_index"]
    err = np.abs(F_b[np.arange(n_runs), idx] - F_64[np.arange(n_runs), idx]) / F_64[np.arange(n_runs), idx]

    def per_run(precision, run_flags):
        total = 0.0
        for j, d in enumerate(datasets):
            # run j of the batch: the same key word 1 (run index) as inside the batch
            R = gsgp.Runner(settings_for(gsgp, wl, G, precision, seed, run_flags | flags), [d], stream=stream)
            torch.cuda.synchronize()
            t = time.perf_counter()
            R.eval_population()
            R.generation(G, stats=False)
            torch.cuda.synchronize()
            total += time.perf_counter() - t
            R.close()
        return total

    if args.skip_per_run:  # profiling runs: the batched handle's kernels only
        t_plain = t_single32 = float("nan")
    else:
        t_plain = per_run(gsgp.FP64, gsgp.FLAG_NO_GRAPH)
        t_single32 = per_run(gsgp.FP32_KAHAN, 0)
    per_launch_traffic = traffic_from_profile(PMC_SUMMARIES["batched_256"]) if not args.local_search else None
    out = {
        "metric": BASELINE_METRIC,
        "value": value,
        "unit": "offspring elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "runs": n_runs, "total_cases": n_all, "pop_size": wl.pop_size,
                   "pool_size": wl.pool_size, "genome_len": wl.genome_len, "generations": G,
                   "tournament_size": wl.tournament_size, "p_crossover": wl.p_crossover,
                   "mutation_step": wl.mutation_step, "precision": "fp32_kahan", "graph_generations": 16,
                   "local_search": bool(args.local_search), "launch": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": per_launch_traffic,
                     "kernel": "k_vary over all 256 runs (one launch)",
                     "alg_bytes_per_launch": alg, "launch_ms": stg["vary_ms"],
                     "probe_3to1_GBps": probes,
                     "frac_of_probe": {k: achieved / v for k, v in probes.items() if v}},
        "stages_ms": {k: round(v, 5) for k, v in stg.items()},
        "eval_stages_ms": {k: round(v, 5) for k, v in eval_stages.items()},
        "interpreter": interpreter_rate_rows(codes, n_cases, eval_stages["compute_semantics_ms"]),
        "runs_per_hour": {"batched_fp32_kahan_graph": n_runs * 3600 / t_step,
                          "plain_per_run_fp64_no_graph": n_runs * 3600 / t_plain,
                          "per_run_fp32_kahan_graph": n_runs * 3600 / t_single32},
        "seconds_for_all_runs": {"batched_fp32_kahan_graph": t_step, "plain_per_run_fp64_no_graph": t_plain,
                                 "per_run_fp32_kahan_graph": t_single32},
        "speedup_vs_plain": t_plain / t_step,
        "best_fitness_rel_err_vs_fp64_replay": {"max": float(err.max()), "median": float(np.median(err))},
        "within_1e-4": bool(err.max() <= 1e-4),
    }
    if not args.no_cpu_baseline:
        sizes = np.array([d.X_train.shape[0] for d in datasets])
        order = np.argsort(sizes)
        picks = [int(order[0]), int(order[len(order) // 3]), int(order[2 * len(order) // 3]), int(order[-1])]
        out["oracle_fitness_check"] = oracle_fitness_check(wl, datasets, G, seed, rec, elite, F_b, picks,
                                                           args.local_search)
        cb = cpu_baseline_runs(wl, datasets, G, seed, list(range(0, n_runs, 4)), 50,
                               local_search=args.local_search)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["runs_per_hour"] = cb["runs_per_hour"]
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        c1 = cpu_baseline_runs(wl, datasets, G, seed, list(range(0, n_runs, 32)), 10, threads=1,
                               local_search=args.local_search)
        out["cpu_baseline"]["one_thread"] = {k: c1[k] for k in ("value", "runs_per_hour", "sample")}
    return out


def bench_paper_shape(args, wl) -> dict:
    """The speed-up study's shape (Section 3.1): CreatePopulation,
    ComputeSemantics, one generation and total run time on the GPU, each next
    to the single-thread FP64 oracle timed on a slice (all programs, 1/64 of
    the cases at k = 127, fewer for longer programs; genome generation in
    full) and scaled linearly in cases."""
    import torch
    from oracle import oracle as orc
    from paper_2106_04034_amd import gsgp, synth

    G = args.generations or wl.generations
    data = synth.paper_shape(wl.n_train, wl.n_features)
    seed = synth.evolution_seed(5)
    s = settings_for(gsgp, wl, G, gsgp.FP32, seed)
    s.ms_random = 1
    stream = torch.cuda.Stream()
    # the variation launch shape, picked by the autotuner on a handle of its own
    if args.launch:
        w, o, x, g = (int(v) for v in args.launch.split(","))
        tuned = {"waves": w, "offspring_per_block": o, "xcd_remap": x, "max_blocks": g}
    elif args.no_autotune:
        tuned = None
    else:
        T = gsgp.Runner(s, [data], stream=stream)
        T.eval_population()
        tuned = T.autotune()
        T.close()
    torch.cuda.synchronize()
    # Total run time as the paper takes it: host data in, whole run, the
    # final fitness back on the host.
    t0 = time.perf_counter()
    R = gsgp.Runner(s, [data], stream=stream)
    if tuned:
        R.set_launch(tuned["waves"], tuned["offspring_per_block"], tuned["xcd_remap"], tuned["max_blocks"])
    R.eval_population()
    R.generation(G, stats=False)
    F_final, _ = R.fitness(0)
    total_s = time.perf_counter() - t0
    ev = R.time_eval()
    ng = min(G, 20)
    stages = R.time_stages(ng)
    rec = R.records(0, 1, ng)
    per_launch = float(np.mean([vary_bytes(rec[g], wl.n_train, 4, wl.pop_size) for g in range(ng)]))
    achieved = per_launch / (stages["vary_ms"] * 1e-3) / 1e9
    codes, _ = R.genomes(0)
    interp = interpreter_rate(codes, wl.n_train, ev["compute_semantics_ms"])
    R.close()

    gpu = {"create_population_ms": ev["create_population_ms"], "compute_semantics_ms": ev["compute_semantics_ms"],
           "generation_ms": stages["generation_ms"], "total_run_ms": total_s * 1e3}
    out = {"metric": "stage speed-up over the single-thread FP64 oracle (paper's categories)",
           "value": None, "unit": "x (one generation)",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": wl.name, "n_train": wl.n_train, "n_features": wl.n_features,
                      "pop_size": wl.pop_size, "pool_size": wl.pool_size, "genome_len": wl.genome_len,
                      "generations": G, "loop": "mutate every individual, random step", "precision": "fp32",
                      "launch": tuned},
           "gpu": gpu, "best_train_rmse": float(np.min(F_final)),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "kernel": "k_vary (GSM + chunk partial sums)",
                        "alg_bytes_per_launch": per_launch, "launch_ms": stages["vary_ms"]},
           "interpreter": interp,
           "stages_ms": {k: round(v, 5) for k, v in stages.items()}}
    if args.no_cpu_baseline:
        return out

    orc.set_threads(1)
    cfg = orc.Config(pop_size=wl.pop_size, pool_size=wl.pool_size, genome_len=wl.genome_len,
                     tournament_size=0, p_crossover=0.0, ms_random=1, seed=seed)
    t = time.perf_counter()
    cp, vp = orc.genomes(cfg, wl.n_features, orc.TAG_POPULATION, wl.pop_size)
    cr, vr = orc.genomes(cfg, wl.n_features, orc.TAG_POOL, wl.pool_size)
    c_create = time.perf_counter() - t
    frac = 64 * max(1, (wl.genome_len + 1) // 128)       # ~15 s of oracle work at every size
    ncs = wl.n_train // frac
    Xs, ys = data.X_train[:ncs], data.y_train[:ncs]
    t = time.perf_counter()
    S = orc.interpret(cp, vp, Xs)
    sig = orc.sigmoid(orc.interpret(cr, vr, Xs))
    c_sem = (time.perf_counter() - t) * frac
    F = orc.rmse_rows(S, ys)
    t = time.perf_counter()
    gens = 3
    for g in range(1, gens + 1):
        rec = orc.select(cfg, g, F)
        O = orc.vary(rec, S, sig)
        F_O = orc.rmse_rows(O, ys)
        no_test = np.zeros((wl.pop_size, 0))
        orc.survive(F, F.copy(), F_O, F_O.copy(), S, O, no_test, no_test.copy())
        S, F = O, F_O
    c_gen = (time.perf_counter() - t) / gens * frac
    orc.set_threads(len(os.sched_getaffinity(0)))
    c_total = c_create + c_sem + G * c_gen                  # resident data: no load time
    cpu = {"create_population_ms": c_create * 1e3, "compute_semantics_ms": c_sem * 1e3,
           "generation_ms": c_gen * 1e3, "total_run_ms": c_total * 1e3}
    out.update({"value": cpu["generation_ms"] / gpu["generation_ms"], "cpu_oracle_1_thread": cpu,
                "speedup": {k: cpu[k] / gpu[k] for k in gpu},
                "cpu_sample": f"genomes in full; semantics and {gens} generations on 1/{frac} of the cases, "
                              "scaled linearly in cases"})
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched_256")
    ap.add_argument("--local-search", action="store_true",
                    help="GSGP with local search (single-run and batched workloads)")
    ap.add_argument("--stage-gens", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--generations", type=int, default=0,
                    help="override the workload's generation count (profiling runs only)")
    ap.add_argument("--runs", type=int, default=0, help="batched_256: number of runs (default 256)")
    ap.add_argument("--skip-per-run", action="store_true",
                    help="batched_256: skip the per-run comparison forms (profiling runs only)")
    ap.add_argument("--launch", default="",
                    help="variation launch shape waves,offspring_per_block,xcd_remap,max_blocks "
                         "(skips autotuning)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported (independent runs "
              "would shard over GPUs with no communication and a single run over its fitness cases, "
              "neither of which is built here)", file=sys.stderr)
        return 2

    from paper_2106_04034_amd import synth

    wl = synth.WORKLOADS[args.workload]
    if wl.name == "single_fp32_100k":
        out = bench_single(args, wl, synth.single_run(wl.n_train, wl.n_test, wl.n_features),
                           synth.evolution_seed(1))
    elif wl.name == "large_fp32_1m":
        out = bench_single(args, wl, synth.large_run(wl.n_train, wl.n_test, wl.n_features),
                           synth.evolution_seed(2))
    elif wl.name == "plain_fp64_500x8":
        out = bench_single(args, wl, synth.plain_small(wl.n_train, wl.n_test, wl.n_features),
                           synth.evolution_seed(0))
    elif wl.name == "precision_1m":
        out = bench_precision(args)
    elif wl.name.startswith("paper_shape"):
        out = bench_paper_shape(args, wl)
    else:
        out = bench_batched(args)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
