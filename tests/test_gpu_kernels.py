"""Kernel-level GPU tests: the symmetric MFMA GEMM with its epilogues (against
FP64 host products of the same rounded operands) and the FP64 Lanczos bound
(against the oracle). Every call goes through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2507_09165_amd import inputs
from paper_2507_09165_amd import psdproj as P
from gpu_util import dev, rel_fro, say, to_dev

pytestmark = pytest.mark.gpu


def _np_dtype(dt):
    import torch
    return {"fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}[dt]


def _rounded(A, dt):
    """Round an FP64 array through the device dtype (host-side torch cast)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(A)).to(_np_dtype(dt))
    return t, t.to(torch.float64).numpy()


def _sym_upper_ref(M):
    U = np.triu(M)
    return U + np.triu(M, 1).T


@pytest.mark.parametrize("dt", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("n_p", [128, 384])
def test_sym_gemm_plain(dt, n_p):
    import torch
    say("sym_gemm plain", dt, n_p)
    L64 = inputs.goe(n_p, 31, np.float64)
    Lt, L = _rounded(L64, dt)
    Rt, R = _rounded(L64 @ L64 / 3.0, dt)
    C0t, C0 = _rounded(inputs.goe(n_p, 32, np.float64), dt)
    Lg, Rg, C0g = Lt.to(dev()), Rt.to(dev()), C0t.to(dev())
    D = torch.zeros_like(Lg)
    P.sym_gemm(dt, Lg, Rg, D, C0=C0g, alpha=-0.75, beta=1.5, gamma=0.25)
    torch.cuda.synchronize()
    Dh = D.to(torch.float64).cpu().numpy()
    ref = _sym_upper_ref(-0.75 * C0 + 1.5 * (L @ R) + 0.25 * np.eye(n_p))
    np.testing.assert_array_equal(Dh, Dh.T)
    tol = {"fp32": 2e-6, "fp16": 1e-3, "bf16": 8e-3}[dt]
    assert rel_fro(Dh, ref) < tol, rel_fro(Dh, ref)
    # elementwise: one rounding of the output plus FP32 accumulation
    u = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}[dt]
    bound = u * np.abs(ref) + 1e-5 * np.abs(L) @ np.abs(R) + 1e-6
    assert np.all(np.abs(Dh - ref) <= 1.5 * bound)


@pytest.mark.parametrize("dt", ["fp16", "bf16"])
@pytest.mark.parametrize("ls,rs", [(True, True), (False, True), (True, False)])
def test_sym_gemm_split(dt, ls, rs):
    """hi + lo operands: the product recovers ~FP32 accuracy."""
    import torch
    n_p = 256
    say("sym_gemm split", dt, ls, rs)
    S = 2048.0 if dt == "fp16" else 1.0
    A64 = inputs.goe(n_p, 41, np.float64)
    B64 = A64 @ A64 - 0.5 * np.eye(n_p)

    def pair(M):
        hi_t, hi = _rounded(M, dt)
        lo_t, lo = _rounded((M - hi) * S, dt)
        return hi_t.to(dev()), lo_t.to(dev()), hi + lo / S

    def single(M):
        t, x = _rounded(M, dt)
        return t.to(dev()), None, x

    Lh, Ll, Lx = pair(A64) if ls else single(A64)
    Rh, Rl, Rx = pair(B64) if rs else single(B64)
    Dh = torch.zeros_like(Lh)
    Dl = torch.zeros_like(Lh)
    P.sym_gemm(dt, Lh, Rh, Dh, Llo=Ll, Rlo=Rl, Dlo=Dl, beta=1.0)
    torch.cuda.synchronize()
    D = Dh.to(torch.float64).cpu().numpy() + Dl.to(torch.float64).cpu().numpy() / S
    ref = _sym_upper_ref(Lx @ Rx)
    err = rel_fro(D, ref)
    say("  split rel err", err)
    assert err < (2e-6 if dt == "fp16" else 5e-5), err


@pytest.mark.parametrize("n", [1, 2, 5, 20, 256, 777])
def test_lanczos_bound_matches_oracle(n):
    import torch
    say("lanczos", n)
    X = inputs.goe(n, 50 + n) if n > 1 else np.array([[-1.75]], dtype=np.float32)
    info = P.spectral_bound(to_dev(X))
    ref = oracle.spectral_bound(X.astype(np.float64))
    say("  gpu", info["lambda"], "oracle", ref["lam"], "steps", info["lanczos_steps"], ref.get("k"))
    assert info["lanczos_steps"] == ref["k"]
    assert abs(info["lambda"] - ref["lam"]) <= 1e-9 * ref["lam"]
    assert abs(info["sigma"] - ref["sigma"]) <= 1e-10 * ref["sigma"]
    assert abs(info["fro_norm"] - ref["fro"]) <= 1e-12 * ref["fro"]
    assert abs(info["colmax_norm"] - ref["colmax"]) <= 1e-12 * ref["colmax"]
    true = np.max(np.abs(np.linalg.eigvalsh(X.astype(np.float64))))
    assert info["lambda"] >= true * (1 - 1e-12)
    assert info["fallback"] == 0 and info["nonfinite"] == 0


def test_lanczos_bound_constructed_spectrum_valid_and_tight():
    X, Q, lam = inputs.constructed(512, 0, 1)
    info = P.spectral_bound(to_dev(X))
    true = np.max(np.abs(np.linalg.eigvalsh(X.astype(np.float64))))
    assert true <= info["lambda"] <= 1.01 * true
