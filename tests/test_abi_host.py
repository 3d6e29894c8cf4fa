"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/gsgp.h declares, sizes workspaces, and rejects
invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2106_04034_amd import gsgp
from tests.conftest import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "gsgp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:gsgp_status|const char\*)\s+(gsgp_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 19
    assert sorted(gsgp.EXPORTS) == names
    L = gsgp.lib()
    for n in names:
        assert getattr(L, n) is not None


def test_status_strings():
    L = gsgp.lib()
    for code in gsgp.STATUS:
        assert L.gsgp_status_string(code)
    assert L.gsgp_status_string(0) == b"ok"


def test_workspace_size_tracks_memory_complexity():
    """Section 2.3: memory O(mk + rk + 2mn + rn + nl); the workspace holds
    exactly those arrays (padded) plus the ancestry record and small tables."""
    for prec, s_bytes in ((gsgp.FP64, 8), (gsgp.FP32, 4)):
        st = gsgp.Settings(pop_size=1024, pool_size=512, genome_len=127, n_generations_max=100,
                           precision=prec)
        n_tr, n_te, l = 100_000, 25_000, 20
        size = gsgp.workspace_size(st, [(n_tr, n_te, l)])
        ld = -(-n_tr // 64) * 64 + -(-n_te // 64) * 64
        semantic = (2 * 1024 + 512) * ld * s_bytes
        data = l * ld * 8 + ld * s_bytes
        record = 100 * 1024 * 32
        genomes = (1024 + 512) * 127 * (4 + 8) * 2
        lower = semantic + data + record + genomes
        assert lower <= size <= lower * 1.02 + (1 << 20)
    # per-run buffers scale with the runs; with genomes of at most 66 genes
    # every stack fits an LDS column and no spill stacks are reserved
    short = gsgp.Settings(genome_len=66)
    one = gsgp.workspace_size(short, [(500, 200, 8)])
    two = gsgp.workspace_size(short, [(500, 200, 8), (500, 200, 8)])
    assert 1.9 * one < two < 2.1 * one


def test_spill_stacks_are_sized_for_the_deepest_possible_genome():
    """Genomes of k genes can need k - 3 stack values below the top two; past
    63 they run in the spill pass, whose 128 wavefront columns of (k - 3) x
    2 cases x 64 lanes doubles the workspace reserves once for all runs."""
    runs = [(500, 200, 8)]
    base = gsgp.workspace_size(gsgp.Settings(genome_len=66), runs)
    for k in (67, 127, 2047):
        extra = gsgp.workspace_size(gsgp.Settings(genome_len=k), runs) - base
        # codes and constants, compiled ops and constants, reciprocals
        genomes = (128 + 128) * (k - 66) * ((4 + 8) * 2 + 8)
        spill = 128 * (k - 3) * 2 * 64 * 8
        assert spill + genomes <= extra <= spill + genomes + 4096, k
    two = gsgp.workspace_size(gsgp.Settings(genome_len=127), runs * 2) - gsgp.workspace_size(
        gsgp.Settings(genome_len=127), runs)
    assert two < 128 * 124 * 1024  # shared, not per run


def test_guard_flag_adds_one_guard_per_buffer():
    """GSGP_FLAG_GUARDS: 4 shared buffers plus 23 per run, each followed by
    a 256-byte guard (rounded up to the 256-byte buffer alignment)."""
    for runs in ([(500, 200, 8)], [(500, 200, 8), (900, 0, 3)]):
        plain = gsgp.workspace_size(gsgp.Settings(), runs)
        guarded = gsgp.workspace_size(gsgp.Settings(flags=gsgp.FLAG_GUARDS), runs)
        n_guards = 4 + 23 * len(runs)
        assert plain + 256 * n_guards <= guarded <= plain + 512 * n_guards


BAD_SETTINGS = [
    dict(pop_size=0), dict(pool_size=0), dict(genome_len=0), dict(genome_len=5000),
    dict(n_generations_max=0), dict(tournament_size=-1), dict(tournament_size=65),
    dict(ms_random=2), dict(p_crossover=1.5), dict(p_crossover=-0.1),
    dict(tournament_size=0, p_crossover=0.5), dict(mutation_step=-1.0),
    dict(mutation_step=float("nan")), dict(p_function=0.9, p_feature=0.2),
    dict(erc_lo=1.0, erc_hi=-1.0), dict(erc_hi=float("inf")), dict(precision=3), dict(flags=8),
    dict(flags=16),
]


@pytest.mark.parametrize("bad", BAD_SETTINGS)
def test_invalid_settings_rejected(bad):
    st = gsgp.Settings(**bad)
    with pytest.raises(gsgp.GSGPError) as e:
        gsgp.workspace_size(st, [(100, 10, 3)])
    assert e.value.status == -1
    assert gsgp.lib().gsgp_last_error()


@pytest.mark.parametrize("shape", [(0, 10, 3), (10, -1, 3), (10, 5, 0), (10, 5, 70000)])
def test_invalid_runs_rejected(shape):
    with pytest.raises(gsgp.GSGPError) as e:
        gsgp.workspace_size(gsgp.Settings(), [shape])
    assert e.value.status == -1


def test_test_pointers_must_match_n_test():
    runs = gsgp.run_descs([(10, 0, 2, (1, 1, 1, 1))])
    out = ctypes.c_size_t(0)
    cfg = gsgp.Settings().c()
    assert gsgp.lib().gsgp_workspace_size(ctypes.byref(cfg), runs, 1, ctypes.byref(out)) == -1


def test_init_rejects_workspace_before_device_work():
    L = gsgp.lib()
    st = gsgp.Settings()
    runs = gsgp.run_descs([(100, 10, 3)])
    cfg = st.c()
    need = gsgp.workspace_size(st, [(100, 10, 3)])
    h = ctypes.c_void_p(0)
    assert L.gsgp_init(ctypes.byref(cfg), runs, 1, None, need, None, ctypes.byref(h)) == -3
    assert L.gsgp_init(ctypes.byref(cfg), runs, 1, ctypes.c_void_p(4096 + 8), need, None,
                       ctypes.byref(h)) == -3
    assert L.gsgp_init(ctypes.byref(cfg), runs, 1, ctypes.c_void_p(4096), need - 1, None,
                       ctypes.byref(h)) == -3
    assert b"needs" in L.gsgp_last_error()
    assert h.value is None
    assert L.gsgp_init(ctypes.byref(cfg), runs, 0, ctypes.c_void_p(4096), need, None,
                       ctypes.byref(h)) == -1


def test_null_handle_calls_fail_cleanly():
    L = gsgp.lib()
    g = ctypes.c_int32(0)
    assert L.gsgp_current_generation(None, ctypes.byref(g)) == -1
    assert L.gsgp_generation(None, 1, None) == -1
    assert L.gsgp_eval_population(None, None, None) == -1
    assert L.gsgp_destroy(None) == 0


def test_host_code_under_address_sanitizer(tmp_path):
    """The library's host code (argument validation, workspace planning,
    handle set-up up to the first device call) built with AddressSanitizer
    on the host side only: the checks above run clean against it."""
    import shutil
    import subprocess
    import sys
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rt = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"
    if not os.path.exists(hipcc) or not os.path.exists(rt):
        pytest.skip("hipcc or the clang AddressSanitizer runtime is not available")
    lib = str(tmp_path / "libgsgp_asan.so")
    csrc = os.path.join(ROOT, "paper_2106_04034_amd", "csrc")
    # the sanitizer applies to the host pass only (-Xarch_host before it)
    host_only = "-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -shared-libasan".split()
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           *host_only, "-o", lib, os.path.join(csrc, "kernels.hip"),
                           os.path.join(csrc, "interp.hip"), os.path.join(csrc, "runtime.hip")],
                          stderr=subprocess.DEVNULL)
    env = dict(os.environ, LD_PRELOAD=rt, GSGP_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0:detect_odr_violation=0")
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi_host.py"), "-k", "not sanitizer"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, (out.stdout[-3000:], out.stderr[-3000:])
    assert "AddressSanitizer" not in out.stderr
