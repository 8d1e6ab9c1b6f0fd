"""Every precision form at ragged orders around the tile and K-unit edges
(1, 2, 33, 65, 129, 257, 511, 1025): each projection against the FP64 oracle
evaluated with the device's bound, bitwise-symmetric output. The orders put
the last 32-K unit, the last 64-K tile and the last 128 tile one element past
a boundary, and n = 1 and 2 exercise the degenerate Lanczos runs."""
import numpy as np
import pytest

import oracle
from paper_2507_09165_amd import inputs
from paper_2507_09165_amd import psdproj as P
from gpu_util import rel_fro, say, to_dev

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 33, 65, 129, 257, 511, 1025]
FORMS = [("fp16", {}), ("bf16", {}), ("fp16_split", {}), ("fp8_fp16_split", {}), ("fp8_bf16_split", {}),
         ("fp32", {}), ("fp32_emu", {}), ("ns_fp16", {}),
         ("fp8_fp16_split", dict(split_mask=0x7F, split_final=1)),
         ("fp8_fp16_split", dict(split_mask=0xF | P.SPLIT_B_ONLY, split_final=0))]
TOL = {"fp32": 1e-5, "fp32_emu": 1e-5}


@pytest.mark.parametrize("n", SIZES)
def test_forms_at_ragged_orders(n):
    import torch
    X32 = inputs.goe(n, 1000 + n)
    X = to_dev(X32)
    say("sweep", n)
    runs = []
    for mode, opts in FORMS:
        out, info_t = P.project_ex(X, mode=mode, **opts)
        runs.append((mode, opts, out, info_t))
    torch.cuda.synchronize()
    for mode, opts, out, info_t in runs:
        info = P.read_info(info_t)
        ref, _ = oracle.project_poly(X32.astype(np.float64), mode, lam=info["lambda"])
        got = out.cpu().numpy().astype(np.float64)
        e = rel_fro(got, ref)
        np.testing.assert_array_equal(got, got.T)
        assert info["nonfinite"] == 0
        assert e <= TOL.get(mode, 5e-3), (n, mode, opts, e)
