"""The autotuner (psdproj_autotune / psdproj_tune_load): it writes one cache
line per size class for this device, the lines load back, and projections
under the tuned policies keep parity with the oracle and single/batched
bitwise agreement. Every test restores the default policies."""
import os

import numpy as np
import pytest

import oracle
from paper_2507_09165_amd import inputs
from paper_2507_09165_amd import psdproj as P
from gpu_util import rel_fro, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_autotune_writes_cache_and_keeps_parity(tmp_path):
    import torch
    cache = tmp_path / "tune.txt"
    cache.write_text("psdproj-tune 1 gfx000 7 1 40 256 8 1.0 1000\n")  # another device's line is kept
    sizes = [700, 2300, 6100]
    try:
        say("autotune fp16", sizes)
        P.autotune("fp16", sizes, str(cache))
        lines = [l.split() for l in cache.read_text().splitlines()]
        mine = [l for l in lines if l[2] != "gfx000"]
        say("  cache:", mine)
        assert len(lines) == 4 and len(mine) == 3
        assert all(l[2].startswith("gfx") and l[4] == "1" and l[6] in ("128", "256") for l in mine)
        assert sorted(int(l[9]) for l in mine) == sizes
        P.tune("class_choices_clear", 0)
        assert P.tune_load(str(cache)) == 3
        for n in (2300, 6100):
            X32 = inputs.goe(n, 50 + n)
            X = to_dev(X32)
            out, info_t = P.project_ex(X, mode="fp16")
            batched = P.project_batched([X, to_dev(inputs.goe(300, 9))], mode="fp16")[0]
            torch.cuda.synchronize()
            info = P.read_info(info_t)
            assert torch.equal(out, batched)
            ref, _ = oracle.project_poly(X32.astype(np.float64), "fp16", lam=info["lambda"])
            e = rel_fro(out.cpu().numpy(), ref)
            say(f"  n={n} tuned fp16 vs oracle {e:.3e}")
            assert e <= 5e-3
    finally:
        P.tune("class_choices_clear", 0)


def test_tune_load_ignores_other_devices_and_garbage(tmp_path):
    cache = tmp_path / "t.txt"
    cache.write_text("garbage\npsdproj-tune 1 gfx000 7 1 40 256 8 1.0 1000\npsdproj-tune 2 gfx950 256 1 40 256 8 1 9\n")
    try:
        assert P.tune_load(str(cache)) == 0
        assert P.tune_load(str(tmp_path / "missing.txt")) == 0
    finally:
        P.tune("class_choices_clear", 0)
