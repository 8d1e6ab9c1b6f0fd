"""The one-workgroup path of small matrices (n <= 128 in the FP16/BF16 work
formats, FP32_EMU included): the whole of Algorithm 2 for one matrix in one
workgroup, one launch for every small matrix of a call.

Against the oracle: the spectral bound (Theorem 2) to 1e-9 and the FP64
composite polynomial with the device's bound, entry by entry and in relative
Frobenius norm, at orders around the 32 x 32 block and 16-wide K edges; the
same matrices through the launch sequence (small-matrix rule off) land on the
same bound and within the same tolerance. Batches mixing small and large
matrices: every result bitwise equal to its single call. Degenerate inputs:
n = 1, the zero matrix, non-finite entries, in place with a padded leading
dimension, the bound override and the forced guard.
"""
import numpy as np
import pytest

import oracle
from paper_2507_09165_amd import inputs
from paper_2507_09165_amd import psdproj as P
from gpu_util import dev, rel_fro, say, to_dev

pytestmark = pytest.mark.gpu

MODES = ["fp16", "bf16", "fp16_split", "fp8_fp16_split", "fp8_bf16_split", "fp32_emu"]
TOL = {"fp32_emu": 1e-5}
TOL_POLY = 5e-3
SIZES = [1, 2, 3, 15, 16, 17, 31, 32, 33, 48, 63, 64, 65, 97, 100, 127, 128]


def _run(X32, mode, **opts):
    import torch
    out, info_t = P.project_ex(to_dev(X32), mode=mode, **opts)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), P.read_info(info_t)


def _matrix(n, seed):
    return inputs.goe(n, seed) if n > 1 else np.array([[-1.75 if seed % 2 else 0.8]], dtype=np.float32)


def _max_abs_bound(ref, tol):
    return 10.0 * tol * max(float(np.linalg.norm(ref)), 1e-300) / ref.shape[0]


@pytest.mark.parametrize("mode", MODES)
def test_small_against_oracle(mode):
    for n in SIZES:
        X32 = _matrix(n, 300 + n)
        say("small", mode, n)
        out, info = _run(X32, mode)
        X = X32.astype(np.float64)
        b = oracle.spectral_bound(X)
        assert info["lanczos_steps"] == b["k"], (n, info["lanczos_steps"], b["k"])
        assert abs(info["lambda"] - b["lam"]) <= 1e-9 * b["lam"], (n, info["lambda"], b["lam"])
        assert abs(info["fro_norm"] - b["fro"]) <= 1e-12 * b["fro"]
        assert abs(info["colmax_norm"] - b["colmax"]) <= 1e-12 * b["colmax"]
        assert info["fallback"] == 0 and info["nonfinite"] == 0
        ref, _ = oracle.project_poly(X, mode, lam=info["lambda"])
        np.testing.assert_array_equal(out, out.T)
        emax = float(np.max(np.abs(out - ref)))
        if n < 15:
            # a tiny matrix may have no positive part (ref near 0): its error
            # is measured against the bound, the scale of every eigenvalue
            e = float(np.linalg.norm(out - ref)) / info["lambda"]
            say(f"  n={n}: vs oracle {e:.3e} of lam")
            assert e <= TOL.get(mode, TOL_POLY), (n, e)
            continue
        e = rel_fro(out, ref)
        say(f"  n={n}: vs oracle {e:.3e}, max abs {emax:.3e}")
        assert e <= TOL.get(mode, TOL_POLY), (n, e)
        assert emax <= _max_abs_bound(ref, TOL.get(mode, TOL_POLY)), (n, emax)


@pytest.mark.parametrize("mode", ["fp16", "fp8_bf16_split"])
def test_small_rule_off_takes_the_sequence(mode):
    """small_max = 0 sends the same matrices through the launch sequence: the
    bound agrees to rounding and both results meet the oracle."""
    try:
        for n in (33, 100, 128):
            X32 = _matrix(n, 400 + n)
            P.tune("small_max", 128)
            a, ia = _run(X32, mode)
            P.tune("small_max", 0)
            b, ib = _run(X32, mode)
            assert abs(ia["lambda"] - ib["lambda"]) <= 1e-12 * ib["lambda"]
            ref, _ = oracle.project_poly(X32.astype(np.float64), mode, lam=ia["lambda"])
            ea, eb = rel_fro(a, ref), rel_fro(b, ref)
            say(f"  {mode} n={n}: one workgroup {ea:.3e}, sequence {eb:.3e}")
            assert ea <= TOL_POLY and eb <= TOL_POLY
    finally:
        P.tune("small_max", 128)


@pytest.mark.parametrize("mode", ["bf16", "fp8_bf16_split", "fp8_fp16_split"])
def test_mixed_batch_equals_single(mode):
    import torch
    sizes = [32, 700, 1, 128, 129, 77, 300, 5]
    Xs = [to_dev(_matrix(n, 500 + n)) for n in sizes]
    outs, infos_t = P.project_batched_ex(Xs, mode=mode)
    alone = [P.project_ex(X, mode=mode) for X in Xs]
    torch.cuda.synchronize()
    infos = P.read_infos(infos_t)
    for i, n in enumerate(sizes):
        assert torch.equal(outs[i], alone[i][0]), n
        assert infos[i]["lambda"] == P.read_info(alone[i][1])["lambda"], n


@pytest.mark.parametrize("mode", ["fp8_fp16_split", "fp16_split"])
def test_small_b_only_stages_split_in_full(mode):
    """The one-workgroup path has no one-sided product: a stage named B-only
    (split_mask bits 16 + t) is split in full there, so the mixed mask gives
    the bits of the full mask over the same stages, and the result meets the
    oracle."""
    sh = P.SPLIT_B_SHIFT
    for n in (40, 128):
        X32 = _matrix(n, 700 + n)
        mixed, info = _run(X32, mode, split_mask=0x4 | (0x3 << sh))
        full, _ = _run(X32, mode, split_mask=0x7)
        np.testing.assert_array_equal(mixed, full)
        ref, _ = oracle.project_poly(X32.astype(np.float64), mode, lam=info["lambda"])
        assert rel_fro(mixed, ref) <= TOL_POLY


def test_small_degenerate_inputs():
    import torch
    n = 50
    # zero matrix: out = 0
    out, info = _run(np.zeros((n, n), np.float32), "fp8_bf16_split")
    assert np.all(out == 0.0) and info["lambda"] == 0.0 and info["nonfinite"] == 0
    # non-finite entry: NaN output and the flag, alone and in a batch
    X32 = _matrix(n, 7)
    Xb = X32.copy()
    Xb[3, 9] = Xb[9, 3] = np.inf
    out, info = _run(Xb, "fp16")
    assert info["nonfinite"] == 1 and np.isnan(out).all()
    good = to_dev(X32)
    outs, infos_t = P.project_batched_ex([good, to_dev(Xb)], mode="fp16")
    ref_good = P.project(good, mode="fp16")
    torch.cuda.synchronize()
    infos = P.read_infos(infos_t)
    assert infos[0]["nonfinite"] == 0 and infos[1]["nonfinite"] == 1
    assert torch.isnan(outs[1]).all() and torch.equal(outs[0], ref_good)
    # in place, leading dimension 70, padding untouched
    ld = 70
    buf = torch.full((n, ld), 1e30, device=dev(), dtype=torch.float32)
    buf[:, :n] = to_dev(X32)
    Xv = buf[:, :n]
    ref_out, _ = _run(X32, "fp8_fp16_split")
    P.project(Xv, Xv, mode="fp8_fp16_split")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Xv.cpu().numpy().astype(np.float64), ref_out)
    assert torch.all(buf[:, n:] == 1e30)


def test_small_override_and_forced_guard():
    X32 = _matrix(90, 11)
    X = X32.astype(np.float64)
    out, info = _run(X32, "fp16", lambda_override=2.5)
    assert info["lambda"] == 2.5
    ref, _ = oracle.project_poly(X, "fp16", lam=2.5)
    assert rel_fro(out, ref) <= TOL_POLY
    out, info = _run(X32, "fp16", force_bound_fallback=True)
    ref, rinfo = oracle.project_poly(X, "fp16", force_fallback=True)
    assert rinfo["fallback"] and info["fallback"] == 1
    assert abs(info["lambda"] - rinfo["lam"]) <= 1e-12 * rinfo["lam"]
    assert rel_fro(out, ref) <= TOL_POLY


def test_small_split_ablation():
    """The split default still pays at small orders: plain BF16 storage at
    every stage is held to nothing, the default FP8-pair split meets the
    target (BF16 keeps 8 significant bits)."""
    X32 = _matrix(128, 13)
    X = X32.astype(np.float64)
    errs = {}
    for name, opts in (("plain", dict(split_mask=0)), ("default", {})):
        out, info = _run(X32, "fp8_bf16_split", **opts)
        ref, _ = oracle.project_poly(X, "fp8_bf16_split", lam=info["lambda"])
        errs[name] = rel_fro(out, ref)
    say("  n=128 fp8_bf16_split plain vs default", errs)
    assert errs["default"] <= TOL_POLY
    assert errs["default"] < errs["plain"]


@pytest.mark.parametrize("mode", ["fp8_bf16_split", "fp16"])
def test_batch_groups_on_streams_equal_single(mode):
    """A batched call runs its matrices as size-balanced groups on concurrent
    streams (batch_streams = 1..4): every result is bitwise the single call's,
    also through a captured graph replayed with eager work in between."""
    import torch
    sizes = [1000, 33, 600, 128, 257, 700, 90, 400, 5, 850]
    Xs = [to_dev(_matrix(n, 600 + n)) for n in sizes]
    alone = [P.project(X, mode=mode) for X in Xs]
    torch.cuda.synchronize()
    try:
        for g in (1, 2, 3, 4):
            P.tune("batch_streams", g)
            outs = P.project_batched(Xs, mode=mode)
            torch.cuda.synchronize()
            for o, a, n in zip(outs, alone, sizes):
                assert torch.equal(o, a), (g, n)
        P.tune("batch_streams", 2)
        s = torch.cuda.Stream()
        outs = [torch.empty_like(X) for X in Xs]
        P.project_batched(Xs, outs, mode=mode, stream=s)
        s.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            P.project_batched(Xs, outs, mode=mode, stream=s)
        for rep in range(3):
            for o in outs:
                o.fill_(-1.0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            for o, a, n in zip(outs, alone, sizes):
                assert torch.equal(o, a), (rep, n)
            P.project(Xs[0], mode="fp16")  # eager work between replays
            torch.cuda.synchronize()
        del graph
    finally:
        P.tune("batch_streams", 2)
