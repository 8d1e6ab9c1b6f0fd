"""Host-side checks of the C ABI: no GPU compute is launched here.

* the library loads and exports every function include/psdproj.h declares;
* its coefficient tables (its own transcription of Tables 1-2 with the
  stage rescale folded in) equal the oracle's independent transcription;
* GEMM counts (Section 3.3: 22 half, 31 single) and argument validation that
  returns before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2507_09165_amd import psdproj as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "psdproj.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(psdproj_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "psdproj_project" in names and "psdproj_project_batched" in names
    L = P.lib()
    for nm in names:
        assert hasattr(L, nm), nm


@pytest.mark.parametrize("mode", ["fp32", "fp16", "bf16", "fp16_split", "fp32_emu", "fp8_fp16_split",
                                  "ns_fp16", "ns_fp32", "fp8_bf16_split"])
def test_library_coefficients_match_oracle(mode):
    lib_rows = P.coefficients(mode)
    ora_rows = oracle.stage_rows(mode)
    np.testing.assert_array_equal(lib_rows, ora_rows)


def test_gemm_counts():
    assert P.gemm_count("fp16") == 22 == oracle.gemm_count("fp16")
    # BF16: stages 1-4 split by default (X enters split from stage 1): 4 x 9 + 3 x 3 + 1
    assert P.gemm_count("bf16") == 46
    assert P.gemm_count("bf16", split_mask=0) == 22  # explicit: no split stage
    assert P.gemm_count("fp32") == 31 == oracle.gemm_count("fp32")
    assert P.gemm_count("ns_fp16") == 21 == oracle.gemm_count("ns_fp16")  # Section 4.1's count
    assert P.gemm_count("ns_fp32") == 31 == oracle.gemm_count("ns_fp32")
    assert P.gemm_count("fp32_emu") == 93  # 10 stages x 3 split products x 3 + 3
    # split products cost 2-3 GEMMs each: no split stages, split final only
    assert P.gemm_count("fp16_split", split_mask=0, split_final=1) == 24  # X0 and X_T as pairs
    assert P.gemm_count("fp16_split") == P.gemm_count("fp16_split", split_mask=0x6)  # default mask
    # a split product: 3 FP16 products with FP16 lo halves, 2 with FP8 pairs
    assert P.gemm_count("fp16_split", split_mask=0x6, split_final=0) == 22 + 6 * 2
    assert P.gemm_count("fp8_fp16_split", split_mask=0x6, split_final=0) == 22 + 6
    # default: stage 3 in full (2 extra), stages 1-2 B-only (0.5 extra each)
    sh = P.SPLIT_B_SHIFT
    assert P.gemm_count("fp8_fp16_split") == P.gemm_count("fp8_fp16_split", split_mask=0x4 | (0x3 << sh)) == 26
    assert P.gemm_count("fp8_fp16_split", split_mask=0x4 | (0xB << sh)) == 22 + 3 + 3 * 0.5
    # a stage set in both masks splits in full
    assert P.gemm_count("fp8_fp16_split", split_mask=0x6 | (0x6 << sh)) == 28
    assert P.gemm_count("fp16_split", split_mask=0x4 | (0x3 << sh)) == 22 + 6 + 2 * 1
    assert P.gemm_count("fp8_fp16_split", split_mask=0x7F, split_final=1) == 44
    # B-only split stages: X X and A A plain, B X one-sided (2 FP16 products
    # with FP16 lo halves, 1.5 with FP8 pairs)
    bo = P.SPLIT_B_ONLY
    assert P.gemm_count("fp8_fp16_split", split_mask=0xF | bo, split_final=0) == 22 + 4 * 0.5
    assert P.gemm_count("fp16_split", split_mask=0xF | bo, split_final=0) == 22 + 4
    assert P.gemm_count("fp8_fp16_split", split_mask=0xF | bo, split_final=1) == 22 + 2 + 1
    # BF16 with FP8 pairs: stages 1-4 split by default like BF16, 2 per split product
    assert P.gemm_count("fp8_bf16_split") == 4 * 3 * 2 + 3 * 3 + 1 == 34
    assert P.gemm_count("fp8_bf16_split", split_mask=0x6, split_final=0) == 22 + 6
    # the flag alone (no stage bits) is no split stage
    assert P.gemm_count("fp8_fp16_split", split_mask=0x80000000 | bo, split_final=0) == 22


def test_workspace_bytes_grow_with_n():
    a, b = P.workspace_bytes(1000, "fp16"), P.workspace_bytes(4000, "fp16")
    assert 0 < a < b
    assert P.workspace_bytes(0, "fp16") == 0
    assert P.workspace_bytes(100, "fp32") > P.workspace_bytes(100, "fp16")


def test_invalid_arguments_rejected_before_device_work():
    L = P.lib()
    vp = ctypes.c_void_p
    assert L.psdproj_project(0, 1, None, None, 1, None) == 0      # n = 0: no-op
    assert L.psdproj_project(5, 4, vp(16), vp(16), 1, None) == 1  # ld < n
    assert L.psdproj_project(-1, 1, vp(16), vp(16), 1, None) == 1
    assert L.psdproj_project(5, 5, None, vp(16), 1, None) == 1    # null X
    assert L.psdproj_project(5, 5, vp(16), vp(16), 99, None) == 1  # bad mode
    o = P.make_opts(mode="fp16", lanczos_steps=33)
    assert L.psdproj_project_ex(ctypes.byref(o), 5, 5, vp(16), vp(16), None, None) == 1
    assert L.psdproj_sym_gemm(1, 100, 100, vp(16), None, vp(16), None, None, None,
                              0.0, 1.0, 0.0, vp(16), None, None) == 1  # n_p % 128
    assert L.psdproj_sym_gemm_pair8(100, 100, vp(16), None, vp(16), None, None, None,
                                    0.0, 1.0, 0.0, vp(16), None, 0, 0, 0, 0, None) == 1  # n_p % 128
    assert L.psdproj_sym_gemm_pair8(128, 128, vp(16), None, vp(16), vp(16), None, None,
                                    0.0, 1.0, 0.0, vp(16), None, 0, 0, 0, 0, None) == 2  # only R split
    assert L.psdproj_sym_gemm_pair8(128, 128, vp(16), None, vp(16), None, None, None,
                                    0.0, 1.0, 0.0, vp(16), None, 0, 0, 0, 99, None) == 1  # exponent range


def test_status_strings():
    L = P.lib()
    assert L.psdproj_status_string(0) == b"ok"
    assert L.psdproj_status_string(3) == b"out of device memory"


def test_tuning_keys_validate_their_values():
    """psdproj_tune: unknown keys and out-of-range values are rejected; the
    host-only keys accept their documented values (defaults restored)."""
    L = P.lib()
    t = lambda k, v: L.psdproj_tune(k.encode(), ctypes.c_int64(v))
    assert t("no_such_key", 1) != 0
    for key, bad in (("gemm_tile", 64), ("gemm_big_min", -1), ("gemm_tail_cus", -1), ("gemm_split_big", 4),
                     ("gemm_ksplit", 0), ("gemm_block", 0), ("work_ld_pad", 100), ("work_ld_pad", -64),
                     ("small_max", -1), ("small_max", 129), ("batch_streams", 0), ("batch_streams", 5)):
        assert t(key, bad) == 1, (key, bad)
    try:
        for key, ok in (("gemm_tile", 256), ("gemm_tile", 128), ("gemm_big_min", 512), ("gemm_tail_cus", 64),
                        ("gemm_split_big", 0), ("gemm_ksplit", 1), ("gemm_block", (4 << 8) | 4),
                        ("small_max", 0), ("small_max", 64), ("batch_streams", 1), ("batch_streams", 4)):
            assert t(key, ok) == 0, (key, ok)
    finally:
        for key, v in (("gemm_tile", 0), ("gemm_big_min", 0), ("gemm_tail_cus", 0), ("gemm_split_big", 3),
                       ("gemm_ksplit", 8), ("gemm_block", (4 << 8) | 4), ("small_max", 128),
                       ("batch_streams", 2)):
            assert t(key, v) == 0


def test_noalloc_scratch_holds_n2048_in_every_mode():
    """The allocation-free entry point's fixed array (its size as the header
    defines it) holds the workspace of every n <= 2048 in every mode."""
    txt = open(os.path.join(ROOT, "include", "psdproj.h")).read()
    m = re.search(r"#define PSDPROJ_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m, "scratch size define"
    limit = int(m.group(1)) << int(m.group(2))
    assert limit == P.NOALLOC_SCRATCH_BYTES
    for mode in P.MODES:
        assert P.workspace_bytes(2048, mode) <= limit, mode
    assert P.workspace_bytes(4096, "fp16") > limit


def test_noalloc_argument_errors_before_device_work():
    L = P.lib()
    o = P.make_opts(mode="fp16")
    assert L.psdproj_project_noalloc(None, 4, 4, None, None, None, None) == 1
    assert L.psdproj_project_noalloc(ctypes.byref(o), -1, 4, None, None, None, None) == 1
    assert L.psdproj_project_noalloc(ctypes.byref(o), 4, 3, None, None, None, None) == 1
    assert L.psdproj_project_noalloc(ctypes.byref(o), 0, 1, None, None, None, None) == 0
    assert L.psdproj_status_string(11)
