"""Batched and served forms on the GPU.

* Batched: one call covers every block (each launch spans all of them). Each
  block's result must equal, bitwise, the single-matrix projection of that
  block, and match the FP64 oracle evaluated with the device's bound.
* Served: requests of mixed sizes and accuracy targets submitted to the
  continuous-batching loop; each result must equal, bitwise, the same
  request computed alone.
"""
import numpy as np
import pytest

import oracle
from paper_2507_09165_amd import inputs
from paper_2507_09165_amd import psdproj as P
from gpu_util import dev, rel_fro, say, to_dev

pytestmark = pytest.mark.gpu


def _single(X, mode):
    out, info_t = P.project_ex(X, mode=mode)
    return out, info_t


@pytest.mark.parametrize("mode", ["bf16", "fp16", "fp32", "fp16_split", "fp8_fp16_split", "fp8_bf16_split"])
def test_batched_mixed_sizes_equal_single(mode):
    import torch
    sizes = [1, 32, 33, 100, 128, 257, 640, 1024, 1600]
    say("batched", mode, sizes)
    Xs = [to_dev(inputs.goe(n, 300 + n) if n > 1 else np.array([[0.7]], np.float32)) for n in sizes]
    outs = P.project_batched(Xs, mode=mode)
    singles = [P.project(X, mode=mode) for X in Xs]
    torch.cuda.synchronize()
    for n, a, b in zip(sizes, outs, singles):
        assert torch.equal(a, b), n


@pytest.mark.parametrize("mode", ["bf16", "fp8_bf16_split"])
def test_batched_blocks_match_oracle(mode):
    """The batched workload (256 GOE blocks, n log-uniform in [32, 1024],
    seed 7, BF16 with its default split: BF16 hi+lo pairs, or a BF16 hi part
    with FP8 lo codes): every block against the FP64 oracle with the bound the
    batch computed for it, at the half-precision target."""
    import torch
    sizes = inputs.batch_sizes(256, 7)
    blocks = inputs.batch_blocks(sizes, 7)
    say("batched C4, 256 blocks", mode)
    Xs = [to_dev(B) for B in blocks]
    outs, info_t = P.project_batched_ex(Xs, mode=mode)
    torch.cuda.synchronize()
    infos = P.read_infos(info_t)
    worst = 0.0
    for k, (B, o, info) in enumerate(zip(blocks, outs, infos)):
        assert info["nonfinite"] == 0 and info["fallback"] == 0
        ref, _ = oracle.project_poly(B.astype(np.float64), mode, lam=info["lambda"])
        e = rel_fro(o.cpu().numpy(), ref)
        worst = max(worst, e)
        assert e <= 5e-3, (k, B.shape[0], e)
    say(f"  worst block error {worst:.3e}")


def test_batched_with_zero_sized_and_empty():
    import torch
    X = to_dev(inputs.goe(50, 1))
    Z = torch.zeros(0, 0, device=dev())
    outs = P.project_batched([X, Z, X], mode="fp16")
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[2])
    assert P.project_batched([], mode="fp16") == []


def test_served_results_equal_alone():
    import torch
    rng = np.random.default_rng(5)
    sizes = [64, 300, 1000, 2100, 129, 777, 64, 1500]
    targets = [1e-3, 1e-5, 1e-3, 1e-3, 1e-5, 1e-3, 1e-3, 1e-5]
    Xs = [to_dev(inputs.goe(n, 500 + i)) for i, n in enumerate(sizes)]
    modes = ["fp32_emu" if t <= 1e-4 else "fp8_fp16_split" for t in targets]
    alone = [P.project(X, mode=m) for X, m in zip(Xs, modes)]
    torch.cuda.synchronize()
    outs = [torch.full_like(X, float("nan")) for X in Xs]
    say("serve", sizes)
    with P.Server(slots=3) as s:
        tks = []
        for i in rng.permutation(len(sizes)):
            tks.append((i, s.submit(X=Xs[i], out=outs[i], target=targets[i], tag=int(i))))
        for i, tk in tks:
            r = s.wait(tk, timeout_s=120)
            assert r["status"] == 0 and r["tag"] == i
        st = s.stats()
    assert st["completed"] == len(sizes)
    for i in range(len(sizes)):
        assert torch.equal(outs[i], alone[i]), sizes[i]


def test_served_nonfinite_request_reports_status():
    """A served request whose input holds a NaN completes with
    PSDPROJ_ERR_NONFINITE (10) and a NaN output; a finite request served
    beside it completes normally."""
    import torch
    Xb = inputs.goe(300, 41)
    Xb[5, 9] = Xb[9, 5] = np.nan
    Xbad, Xok = to_dev(Xb), to_dev(inputs.goe(300, 42))
    obad, ook = torch.zeros_like(Xbad), torch.zeros_like(Xok)
    ref = P.project(Xok, mode="fp8_fp16_split")
    torch.cuda.synchronize()
    with P.Server(slots=2) as s:
        t1 = s.submit(X=Xbad, out=obad, target=1e-3, tag=1)
        t2 = s.submit(X=Xok, out=ook, target=1e-3, tag=2)
        r1, r2 = s.wait(t1, timeout_s=60), s.wait(t2, timeout_s=60)
    assert r1["status"] == 10 and r2["status"] == 0
    assert torch.isnan(obad).all()
    assert torch.equal(ook, ref)


def test_served_coalesced_group_equals_alone():
    """Small requests queued behind a long one run as one batched projection
    (same start, one slot); each result is bitwise the request's result
    alone, and a non-finite member is reported for itself only."""
    import torch
    sizes = [64, 90, 128, 200, 257, 311, 400, 512, 640, 1000, 77, 1024]
    Xs = [to_dev(inputs.goe(n, 600 + i)) for i, n in enumerate(sizes)]
    Xb = inputs.goe(150, 41)
    Xb[3, 7] = Xb[7, 3] = np.inf
    Xs.append(to_dev(Xb))
    alone = [P.project(X, mode="fp8_fp16_split") for X in Xs[:-1]]
    big = to_dev(inputs.goe(4000, 7))
    obig = torch.empty_like(big)
    torch.cuda.synchronize()
    outs = [torch.full_like(X, -1.0) for X in Xs]
    say("serve coalesced", sizes)
    with P.Server(slots=1) as s:
        tb = s.submit(X=big, out=obig, target=1e-3)
        tks = [s.submit(X=X, out=o, target=1e-3, tag=i) for i, (X, o) in enumerate(zip(Xs, outs))]
        rb = s.wait(tb, timeout_s=120)
        rs = [s.wait(t, timeout_s=120) for t in tks]
    assert rb["status"] == 0
    assert [r["status"] for r in rs] == [0] * len(sizes) + [10]
    starts = {r["start_ns"] for r in rs}
    say(f"  {len(rs)} requests in {len(starts)} launch(es)")
    assert len(starts) < len(rs)
    for i in range(len(sizes)):
        assert torch.equal(outs[i], alone[i]), sizes[i]
    assert torch.isnan(outs[-1]).all()
