"""Python binding of libgsgp.so (the C ABI in include/gsgp.h).

Argument marshalling only: every step of the GSGP hot path runs in the HIP
kernels of the library.  PyTorch provides device memory (the workspace and
the input tensors) and the HIP stream; nothing here computes the method.
There is no CPU fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GSGP_LIBRARY selects another build of the same library (e.g. one with
# host-side sanitizers); by default the in-tree libgsgp.so.
LIB_PATH = os.environ.get("GSGP_LIBRARY") or os.path.join(_HERE, "libgsgp.so")

FP64, FP32, FP32_KAHAN = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp32_kahan": FP32_KAHAN}
FLAG_NO_GRAPH = 1
FLAG_GUARDS = 2
FLAG_LOCAL_SEARCH = 4

STATUS = {0: "GSGP_OK", -1: "GSGP_ERR_ARG", -2: "GSGP_ERR_STATE", -3: "GSGP_ERR_WORKSPACE",
          -4: "GSGP_ERR_NONFINITE", -5: "GSGP_ERR_HIP", -6: "GSGP_ERR_UNSUPPORTED"}

RECORD_DTYPE = np.dtype([("op", "<i4"), ("p1", "<i4"), ("p2", "<i4"), ("r1", "<i4"),
                         ("r2", "<i4"), ("reserved", "<i4"), ("ms", "<f8")])
STATS_DTYPE = np.dtype([("best_train_rmse", "<f8"), ("best_test_rmse", "<f8"),
                        ("best_index", "<i4"), ("elite_copied", "<i4"), ("elite_src", "<i4"),
                        ("elite_dst", "<i4")])

# Every entry point declared in include/gsgp.h.
EXPORTS = [
    "gsgp_workspace_size", "gsgp_init", "gsgp_eval_population", "gsgp_generation",
    "gsgp_generation_replay", "gsgp_reconstruct_scratch_size", "gsgp_reconstruct", "gsgp_reconstruct_static",
    "gsgp_export_linear",
    "gsgp_current_generation", "gsgp_get_fitness", "gsgp_get_semantics", "gsgp_get_semantics_rows",
    "gsgp_get_semantics_cases",
    "gsgp_get_records",
    "gsgp_get_stats", "gsgp_get_scaling", "gsgp_get_genomes", "gsgp_time_stages", "gsgp_time_eval", "gsgp_set_launch",
    "gsgp_autotune", "gsgp_checkpoint_size", "gsgp_checkpoint_save", "gsgp_checkpoint_load",
    "gsgp_guard_offsets", "gsgp_destroy", "gsgp_status_string", "gsgp_last_error",
]


class CConfig(ctypes.Structure):
    _fields_ = [
        ("pop_size", ctypes.c_int32), ("pool_size", ctypes.c_int32),
        ("genome_len", ctypes.c_int32), ("n_generations_max", ctypes.c_int32),
        ("tournament_size", ctypes.c_int32), ("ms_random", ctypes.c_int32),
        ("p_crossover", ctypes.c_double), ("mutation_step", ctypes.c_double),
        ("p_function", ctypes.c_double), ("p_feature", ctypes.c_double),
        ("erc_lo", ctypes.c_double), ("erc_hi", ctypes.c_double),
        ("precision", ctypes.c_int32), ("seed", ctypes.c_uint32), ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
    ]


class CRun(ctypes.Structure):
    _fields_ = [
        ("n_train", ctypes.c_int64), ("n_test", ctypes.c_int64),
        ("n_features", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("X_train", ctypes.c_void_p), ("y_train", ctypes.c_void_p),
        ("X_test", ctypes.c_void_p), ("y_test", ctypes.c_void_p),
    ]


class GSGPError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Loads libgsgp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2106_04034_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "gsgp_workspace_size": [P, P, I32, P],
            "gsgp_init": [P, P, I32, P, ctypes.c_size_t, P, P],
            "gsgp_eval_population": [P, P, P],
            "gsgp_generation": [P, I32, P],
            "gsgp_generation_replay": [P, I32, P, P, P],
            "gsgp_reconstruct_scratch_size": [P, I32, I32, I32, I64, P],
            "gsgp_reconstruct": [P, I32, I32, I32, P, I64, P, P, ctypes.c_size_t],
            "gsgp_reconstruct_static": [P, I32, I32, I32, P, I64, P],
            "gsgp_export_linear": [P, I32, I32, I32, P, P, P],
            "gsgp_current_generation": [P, P],
            "gsgp_get_fitness": [P, I32, P, P],
            "gsgp_get_semantics": [P, I32, I32, P],
            "gsgp_get_semantics_rows": [P, I32, I32, I32, I32, P],
            "gsgp_get_semantics_cases": [P, I32, I32, I64, I64, P],
            "gsgp_get_records": [P, I32, I32, I32, I32, P],
            "gsgp_get_stats": [P, I32, I32, I32, P],
            "gsgp_get_scaling": [P, I32, I32, I32, P],
            "gsgp_get_genomes": [P, I32, P, P],
            "gsgp_time_stages": [P, I32, P],
            "gsgp_time_eval": [P, P],
            "gsgp_set_launch": [P, I32, I32, I32, I32],
            "gsgp_autotune": [P, P],
            "gsgp_guard_offsets": [P, P, I32, P],
            "gsgp_checkpoint_size": [P, P],
            "gsgp_checkpoint_save": [P, P, ctypes.c_size_t],
            "gsgp_checkpoint_load": [P, P, ctypes.c_size_t],
            "gsgp_destroy": [P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.gsgp_status_string.argtypes = [ctypes.c_int]
        L.gsgp_status_string.restype = ctypes.c_char_p
        L.gsgp_last_error.argtypes = []
        L.gsgp_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != 0:
        raise GSGPError(status, where, lib().gsgp_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Settings:
    """Run parameters (mirror of gsgp_config)."""
    pop_size: int = 128
    pool_size: int = 128
    genome_len: int = 127
    n_generations_max: int = 20
    tournament_size: int = 4
    ms_random: int = 0
    p_crossover: float = 0.5
    mutation_step: float = 0.1
    p_function: float = 0.80
    p_feature: float = 0.14
    erc_lo: float = -1.0
    erc_hi: float = 1.0
    precision: int = FP64
    seed: int = 1
    flags: int = 0

    def c(self) -> CConfig:
        return CConfig(self.pop_size, self.pool_size, self.genome_len, self.n_generations_max,
                       self.tournament_size, self.ms_random, self.p_crossover, self.mutation_step,
                       self.p_function, self.p_feature, self.erc_lo, self.erc_hi, self.precision,
                       self.seed & 0xFFFFFFFF, self.flags, 0)


def run_descs(shapes) -> ctypes.Array:
    """Run descriptors from (n_train, n_test, n_features[, pointers]) tuples;
    used for host-only size queries."""
    arr = (CRun * len(shapes))()
    for i, s in enumerate(shapes):
        n_tr, n_te, l = s[:3]
        ptrs = s[3] if len(s) > 3 else (1, 1, 1 if n_te else None, 1 if n_te else None)
        arr[i] = CRun(n_tr, n_te, l, 0, *ptrs)
    return arr


def workspace_size(settings: Settings, shapes) -> int:
    runs = run_descs(shapes)
    out = ctypes.c_size_t(0)
    cfg = settings.c()
    check(lib().gsgp_workspace_size(ctypes.byref(cfg), runs, len(shapes), ctypes.byref(out)),
          "gsgp_workspace_size")
    return int(out.value)


class Runner:
    """One handle: n_runs independent runs (one dataset each) on cuda:`device`.

    ``datasets`` is a list of objects with X_train, y_train, X_test, y_test
    (numpy float64, rows = fitness cases).  The workspace is a torch uint8
    tensor; all work goes to ``stream`` (a torch.cuda.Stream, default: the
    current stream).
    """

    def __init__(self, settings: Settings, datasets, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.settings = settings
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n_runs = len(datasets)
        self.shapes = []
        inputs = []
        runs = (CRun * self.n_runs)()
        with torch.cuda.device(self.device):
            for i, d in enumerate(datasets):
                Xtr = torch.as_tensor(np.ascontiguousarray(d.X_train, np.float64), device=self.device)
                ytr = torch.as_tensor(np.ascontiguousarray(d.y_train, np.float64), device=self.device)
                n_te = int(d.X_test.shape[0])
                if n_te:
                    Xte = torch.as_tensor(np.ascontiguousarray(d.X_test, np.float64), device=self.device)
                    yte = torch.as_tensor(np.ascontiguousarray(d.y_test, np.float64), device=self.device)
                    pte = (Xte.data_ptr(), yte.data_ptr())
                    inputs += [Xte, yte]
                else:
                    pte = (None, None)
                inputs += [Xtr, ytr]
                l = int(d.X_train.shape[1])
                runs[i] = CRun(int(d.X_train.shape[0]), n_te, l, 0, Xtr.data_ptr(), ytr.data_ptr(), *pte)
                self.shapes.append((int(d.X_train.shape[0]), n_te, l))
            self._cfg = settings.c()
            size = ctypes.c_size_t(0)
            check(lib().gsgp_workspace_size(ctypes.byref(self._cfg), runs, self.n_runs,
                                            ctypes.byref(size)), "gsgp_workspace_size")
            self.ws_bytes = int(size.value)
            self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            self._h = ctypes.c_void_p(0)
            torch.cuda.synchronize(self.device)  # input tensors are written
            check(lib().gsgp_init(ctypes.byref(self._cfg), runs, self.n_runs,
                                  ctypes.c_void_p(self._ws_ptr), self.ws_bytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)),
                  "gsgp_init")
        del inputs  # gsgp_init copied them into the workspace

    # -- lifecycle -------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            check(lib().gsgp_destroy(self._h), "gsgp_destroy")
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def m(self) -> int:
        return self.settings.pop_size

    @property
    def r(self) -> int:
        return self.settings.pool_size

    # -- Algorithm 1 -----------------------------------------------------
    def eval_population(self, codes: np.ndarray | None = None, consts: np.ndarray | None = None):
        if codes is not None:
            codes = np.ascontiguousarray(codes, np.int32)
            consts = np.ascontiguousarray(consts, np.float64)
            check(lib().gsgp_eval_population(self._h, _ptr(codes), _ptr(consts)), "gsgp_eval_population")
        else:
            check(lib().gsgp_eval_population(self._h, None, None), "gsgp_eval_population")

    def generation(self, n: int = 1, stats: bool = True):
        out = np.zeros((self.n_runs, n), dtype=STATS_DTYPE) if stats else None
        check(lib().gsgp_generation(self._h, n, _ptr(out) if stats else None), "gsgp_generation")
        return out

    def replay(self, records: np.ndarray, elite: np.ndarray | None = None, stats: bool = True):
        """records: [n_runs][n][m] RECORD_DTYPE (or [n][m] for one run);
        elite: matching [n_runs][n] STATS_DTYPE-like array or None."""
        rec = np.ascontiguousarray(records, dtype=RECORD_DTYPE)
        if rec.ndim == 2:
            rec = rec[None]
        n = rec.shape[1]
        el = None
        if elite is not None:
            el = np.ascontiguousarray(elite, dtype=STATS_DTYPE)
            if el.ndim == 1:
                el = el[None]
        out = np.zeros((self.n_runs, n), dtype=STATS_DTYPE) if stats else None
        check(lib().gsgp_generation_replay(self._h, n, _ptr(rec), _ptr(el) if el is not None else None,
                                           _ptr(out) if stats else None), "gsgp_generation_replay")
        return out

    # -- inspection --------------------------------------------------------
    def current_generation(self) -> int:
        g = ctypes.c_int32(0)
        check(lib().gsgp_current_generation(self._h, ctypes.byref(g)), "gsgp_current_generation")
        return int(g.value)

    def fitness(self, run: int = 0):
        tr = np.zeros(self.m)
        te = np.zeros(self.m)
        check(lib().gsgp_get_fitness(self._h, run, _ptr(tr), _ptr(te)), "gsgp_get_fitness")
        return tr, te

    def semantics_rows(self, run: int, which: int, row0: int, n_rows: int) -> np.ndarray:
        n_tr, n_te, _ = self.shapes[run]
        out = np.zeros((n_rows, n_tr + n_te))
        check(lib().gsgp_get_semantics_rows(self._h, run, which, row0, n_rows, _ptr(out)),
              "gsgp_get_semantics_rows")
        return out

    def semantics_cases(self, run: int, which: int, case0: int, n_cases: int) -> np.ndarray:
        """Cases case0 .. case0 + n_cases - 1 (train then test numbering) of
        every population (which 0) or pool (which 1) row, FP64."""
        rows = self.m if which == 0 else self.r
        out = np.zeros((rows, n_cases))
        check(lib().gsgp_get_semantics_cases(self._h, run, which, int(case0), int(n_cases), _ptr(out)),
              "gsgp_get_semantics_cases")
        return out

    def semantics(self, run: int = 0, which: int = 0) -> np.ndarray:
        n_tr, n_te, _ = self.shapes[run]
        rows = self.m if which == 0 else self.r
        out = np.zeros((rows, n_tr + n_te))
        check(lib().gsgp_get_semantics(self._h, run, which, _ptr(out)), "gsgp_get_semantics")
        return out

    def records(self, run: int, gen0: int, n: int, raw: bool = True) -> np.ndarray:
        out = np.zeros((n, self.m), dtype=RECORD_DTYPE)
        check(lib().gsgp_get_records(self._h, run, gen0, n, 1 if raw else 0, _ptr(out)), "gsgp_get_records")
        return out

    def stats(self, run: int, gen0: int, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=STATS_DTYPE)
        check(lib().gsgp_get_stats(self._h, run, gen0, n, _ptr(out)), "gsgp_get_stats")
        return out

    def scaling(self, run: int, gen0: int, n: int) -> np.ndarray:
        """(alpha, beta) of every individual of generations gen0 .. gen0 + n - 1,
        [n][m][2] (local search; (0, 1) without it)."""
        out = np.zeros((n, self.m, 2))
        check(lib().gsgp_get_scaling(self._h, run, gen0, n, _ptr(out)), "gsgp_get_scaling")
        return out

    def genomes(self, run: int = 0):
        rows = self.m + self.r
        k = self.settings.genome_len
        codes = np.zeros((rows, k), np.int32)
        consts = np.zeros((rows, k))
        check(lib().gsgp_get_genomes(self._h, run, _ptr(codes), _ptr(consts)), "gsgp_get_genomes")
        return codes, consts

    def export_linear(self, run: int, gen: int, individual: int):
        """(tree, c, b, weights): individual = c + b tree(x) + weights . sigmoid(pool(x))
        for a mutation-only lineage; raises GSGPError (unsupported) otherwise."""
        tree = ctypes.c_int32(0)
        cb = np.zeros(2)
        w = np.zeros(self.r)
        check(lib().gsgp_export_linear(self._h, run, gen, individual, ctypes.byref(tree), _ptr(cb), _ptr(w)),
              "gsgp_export_linear")
        return int(tree.value), float(cb[0]), float(cb[1]), w

    def reconstruct(self, run: int, gen: int, individual: int, X: np.ndarray) -> np.ndarray:
        torch = self.torch
        X = np.ascontiguousarray(X, np.float64)
        n = X.shape[0]
        size = ctypes.c_size_t(0)
        check(lib().gsgp_reconstruct_scratch_size(self._h, run, gen, individual, n, ctypes.byref(size)),
              "gsgp_reconstruct_scratch_size")
        with torch.cuda.device(self.device):
            dX = torch.as_tensor(X, device=self.device)
            out = torch.empty(n, dtype=torch.float64, device=self.device)
            scratch = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=self.device)
            sp = (scratch.data_ptr() + 255) // 256 * 256
            torch.cuda.synchronize(self.device)
            check(lib().gsgp_reconstruct(self._h, run, gen, individual, ctypes.c_void_p(dX.data_ptr()), n,
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sp),
                                         int(size.value)), "gsgp_reconstruct")
            return out.cpu().numpy()

    def reconstruct_static(self, run: int, gen: int, individual: int, X: np.ndarray) -> np.ndarray:
        """reconstruct() through the entry point that uses the library's own
        device scratch array (no scratch allocation)."""
        torch = self.torch
        X = np.ascontiguousarray(X, np.float64)
        n = X.shape[0]
        with torch.cuda.device(self.device):
            dX = torch.as_tensor(X, device=self.device)
            out = torch.empty(n, dtype=torch.float64, device=self.device)
            torch.cuda.synchronize(self.device)
            check(lib().gsgp_reconstruct_static(self._h, run, gen, individual, ctypes.c_void_p(dX.data_ptr()), n,
                                                ctypes.c_void_p(out.data_ptr())), "gsgp_reconstruct_static")
            return out.cpu().numpy()

    # -- measurement -------------------------------------------------------
    def time_stages(self, n: int) -> dict:
        ms = np.zeros(4)
        check(lib().gsgp_time_stages(self._h, n, _ptr(ms)), "gsgp_time_stages")
        return {"survive_ms": ms[0], "vary_ms": ms[1], "fitness_ms": ms[2], "generation_ms": ms[3]}

    def time_eval(self) -> dict:
        """Initialisation with per-stage HIP-event timing (restarts the runs)."""
        ms = np.zeros(4)
        check(lib().gsgp_time_eval(self._h, _ptr(ms)), "gsgp_time_eval")
        return {"create_population_ms": ms[0], "compute_semantics_ms": ms[1],
                "initial_fitness_ms": ms[2], "eval_total_ms": ms[3]}

    def set_launch(self, waves: int = 0, offspring_per_block: int = 0, xcd_remap: int = 1,
                   max_blocks: int = 0) -> None:
        check(lib().gsgp_set_launch(self._h, waves, offspring_per_block, xcd_remap, max_blocks),
              "gsgp_set_launch")

    def checkpoint(self) -> bytes:
        """Every run's state at the current generation (see include/gsgp.h)."""
        size = ctypes.c_size_t(0)
        check(lib().gsgp_checkpoint_size(self._h, ctypes.byref(size)), "gsgp_checkpoint_size")
        buf = ctypes.create_string_buffer(size.value)
        check(lib().gsgp_checkpoint_save(self._h, buf, size.value), "gsgp_checkpoint_save")
        return buf.raw

    def restore(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().gsgp_checkpoint_load(self._h, buf, len(blob)), "gsgp_checkpoint_load")

    def guard_offsets(self) -> np.ndarray:
        """Workspace offsets of the guards (FLAG_GUARDS), relative to the
        workspace start."""
        n = ctypes.c_int32(0)
        check(lib().gsgp_guard_offsets(self._h, None, 0, ctypes.byref(n)), "gsgp_guard_offsets")
        out = np.zeros(n.value, dtype=np.int64)
        if n.value:
            check(lib().gsgp_guard_offsets(self._h, _ptr(out), n.value, ctypes.byref(n)), "gsgp_guard_offsets")
        return out

    def autotune(self):
        best = np.zeros(4, np.int32)
        check(lib().gsgp_autotune(self._h, _ptr(best)), "gsgp_autotune")
        return {"waves": int(best[0]), "offspring_per_block": int(best[1]), "xcd_remap": int(best[2]),
                "max_blocks": int(best[3])}
