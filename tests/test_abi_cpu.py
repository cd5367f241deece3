"""The C-ABI library loads and exports every symbol include/nsr.h declares;
host-side argument checks work without a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_2008_11480_amd import nsr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nsr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"^\s*#.*$", "", text, flags=re.M)       # preprocessor lines
    names = re.findall(r"\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;", text)
    return sorted(set(n for n in names if n not in ("sizeof",)))


def test_header_declares_the_binding_exports():
    decl = declared_functions()
    assert decl, "no declarations parsed"
    assert sorted(decl) == sorted(nsr.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = nsr.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.ns_version().startswith(b"nsr")


def test_workspace_bytes():
    plain = nsr.workspace_bytes(4096)
    comp = nsr.workspace_bytes(4096, composite=True)
    assert plain >= 7 * 4096 * 4096 * 8
    assert comp >= 11 * 4096 * 4096 * 8
    assert nsr.workspace_bytes(0) == 0
    assert nsr.workspace_bytes(64, precision=99) == 0
    # ragged sizes are padded to a 32-element leading dimension
    assert nsr.workspace_bytes(33) >= 7 * 33 * 64 * 8


def test_status_strings():
    L = nsr.lib()
    for st in range(0, -10, -1):
        assert L.ns_status_string(st)
    assert L.ns_status_string(-3) == b"iteration diverged"


def test_host_argument_checks_without_gpu():
    L = nsr.lib()
    h = ctypes.c_void_p()
    assert L.ns_create(0, None, 0, 0, 256, 1 << 20, ctypes.byref(h)) == nsr.NS_EINVAL
    assert L.ns_create(0, None, 64, 0, None, 1 << 20, ctypes.byref(h)) == nsr.NS_EINVAL
    assert L.ns_create(0, None, 64, 0, 257, 1 << 20, ctypes.byref(h)) == nsr.NS_EINVAL
    assert L.ns_create(0, None, 64, 0, 256, 16, ctypes.byref(h)) == nsr.NS_ENOMEM
    assert L.ns_create(0, None, 64, 7, 256, 1 << 20, ctypes.byref(h)) == nsr.NS_EINVAL
    assert b"precision" in L.ns_last_error()
    # GEMM argument checks
    assert L.ns_gemm_f64(None, -1, 1, 1, None, 1, None, 1, None, 1, None, 0, None, 0, 0.0, 1.0,
                         0, None) == nsr.NS_EINVAL
    assert L.ns_gemm_f64(None, 4, 4, 4, 256, 2, 512, 4, 768, 4, None, 0, None, 0, 0.0, 1.0,
                         0, None) == nsr.NS_EINVAL       # ldx < k
    assert L.ns_gemm_f64(None, 4, 4, 4, 256, 4, 512, 4, 256, 4, None, 0, None, 0, 0.0, 1.0,
                         0, None) == nsr.NS_EINVAL       # D aliases X
    assert L.ns_gemm_f64(None, 4, 5, 4, 256, 4, 512, 5, 768, 5, None, 0, None, 0, 0.0, 1.0,
                         nsr.GEMM_SYMMETRIC, None) == nsr.NS_EINVAL   # symmetric needs m == n
    assert L.ns_gemm_f64(None, 4, 4, 4, 256, 4, 512, 4, 768, 4, None, 0, None, 0, 0.0, 1.0,
                         8, None) == nsr.NS_EINVAL       # unknown flag
    assert L.ns_gemm_f64(None, 0, 4, 4, None, 4, None, 4, None, 4, None, 0, None, 0, 0.0, 1.0,
                         0, None) == nsr.NS_OK           # empty output: nothing to do
    # the symmetric-output bf16 flag is switched off (rejected before any
    # device work); the split product checks its scratch before launching
    assert L.ns_gemm_bf16_scratch_bytes(4096, 4096, 4096, nsr.GEMM_SYMMETRIC) == 0
    assert L.ns_gemm_bf16_nt_ws(None, 4096, 4096, 4096, 256, 4096, 512, 4096, 768, 4096, None,
                                0, None, 0, None, 0, 0.0, 1.0, nsr.GEMM_SYMMETRIC, None, None,
                                0) == nsr.NS_EINVAL
    assert b"disabled" in L.ns_last_error()
    need = L.ns_gemm_f32_split_scratch_bytes(64, 64, 64)
    assert need > 0
    assert L.ns_gemm_f32_split(None, 64, 64, 64, 256, 64, 512, 64, 768, 64, None, 0, None, 0,
                               None, 0, 0.0, 1.0, None, 1024, need - 1) == nsr.NS_ENOMEM
    assert L.ns_gemm_f32_split(None, 64, 64, 64, 256, 64, 512, 64, 768, 64, None, 0, None, 0,
                               None, 0, 0.0, 1.0, None, 1024 + 8, need) == nsr.NS_EINVAL
    # null handles
    assert L.ns_bind(None, 256, 64) == nsr.NS_EINVAL
    assert L.ns_step(None, 8, 1, 0, 0, None) == nsr.NS_EINVAL
    assert L.ns_destroy(None) == nsr.NS_OK


def test_gemm_partials_count():
    L = nsr.lib()
    assert L.ns_gemm_f64_partials(64, 64, 0) == 1
    assert L.ns_gemm_f64_partials(65, 64, 0) == 2
    assert L.ns_gemm_f64_partials(0, 5, 0) == 0
    # symmetric output: tiles on or above the diagonal only
    t = L.ns_gemm_f64_partials(1000, 1000, 0)
    ts = L.ns_gemm_f64_partials(1000, 1000, nsr.GEMM_SYMMETRIC)
    side = int(round(t ** 0.5))
    assert side * side == t and ts == side * (side + 1) // 2


def test_report_columns_match_the_c_struct():
    """The numpy view used by Batch.poll_arrays reads the same fields as the
    ctypes struct (offsets, types), for every report of an array."""
    reps = (nsr.SolveReportC * 4)()
    for i in range(4):
        reps[i].status = -i
        reps[i].precision = i % 2
        reps[i].ns_steps = 10 + i
        reps[i].refine_steps = 20 + i
        reps[i].ns_stop = i
        reps[i].refine_stop = 5 - i
        reps[i].alpha = 1.5 * i
        reps[i].rel_resid = 1e-11 * (i + 1)
        reps[i].mmm = 1000 + i
        reps[i].gemm_flop = 1e9 * i
        reps[i].fnorm_hist[3] = 7.0      # not a column: must not leak into one
    cols = nsr._report_arrays(reps, 3)
    assert set(cols) == set(nsr._REPORT_COLUMNS)
    for f in nsr._REPORT_COLUMNS:
        assert cols[f].tolist() == [getattr(reps[i], f) for i in range(3)], f
