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


@pytest.mark.parametrize("dt,split", [("fp32", ""), ("fp16", ""), ("fp16", "R"), ("fp16", "LR"),
                                      ("bf16", ""), ("bf16", "LR")])
def test_sym_gemm_tile_shapes_agree(dt, split):
    """The 128 and 256 tiles (each with its own LDS ring depth and row width)
    give bitwise-identical products: every element accumulates its K terms in
    the same order."""
    import torch
    n_p = 768
    say("sym_gemm tiles", dt, split)
    tdt = {"fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}[dt]
    L = to_dev(inputs.goe(n_p, 61)).to(tdt)
    Ll = to_dev(inputs.goe(n_p, 62)).to(tdt) if "L" in split else None
    Rl = to_dev(inputs.goe(n_p, 63)).to(tdt) if "R" in split else None
    outs = []
    try:
        for tile in (128, 256):
            P.tune("gemm_tile", tile)
            D = torch.zeros_like(L)
            Dl = torch.zeros_like(L) if split else None
            P.sym_gemm(dt, L, L, D, Llo=Ll, Rlo=Rl, C0=L, Dlo=Dl, alpha=0.5, beta=-1.25)
            torch.cuda.synchronize()
            outs.append((D.cpu(), Dl.cpu() if split else None))
    finally:
        P.tune("gemm_tile", 0)
    assert torch.equal(outs[0][0], outs[1][0])
    if split:
        assert torch.equal(outs[0][1], outs[1][1])


def _pair8(M, e, dt="fp16"):
    """FP16 (or BF16) hi and the FP8 pair codes of a symmetric FP64 matrix;
    returns the device tensors and the value the pair represents."""
    from gpu_util import e4m3_encode, e4m3_values, pair8_pack
    shift = 11 if dt == "fp16" else 8  # significant bits of the hi format
    hi_t, hi64 = _rounded(M, dt)
    lc = e4m3_encode((M - hi64) * 2.0 ** (shift + e))
    val = hi64 + e4m3_values()[lc] * 2.0 ** -(shift + e)
    return hi_t.to(dev()), to_dev(pair8_pack(lc)), val


@pytest.mark.parametrize("n_p", [256, 384])
def test_sym_gemm_pair8(n_p):
    """FP8-pair product: L_hi R_hi on FP16 MFMAs, both cross terms on the e4m3
    MFMA (the codes of M_hi 2^e formed in registers), the pair addend and the
    pair output. Checked against the FP64 product of the values the pairs
    represent; the output codes are symmetric."""
    import torch
    from gpu_util import e4m3_values, pair8_unpack
    say("sym_gemm pair8", n_p)
    A = inputs.goe(n_p, 71, np.float64)
    Bm = A @ A * 2.5 - 0.75 * np.eye(n_p)          # entries up to ~2.5
    # pair exponents keep |M| 2^e below the e4m3 maximum (448) given the
    # spectral norms: ||A|| <= ~2, ||Bm|| <= ~9.25, ||D|| <= ~22
    eL, eR, eC, eD = 7, 5, 7, 3
    Lh, Lx, Lv = _pair8(A, eL)
    Rh, Rx, Rv = _pair8(Bm, eR)
    Ch, Cx, Cv = _pair8(A, eC)
    D = torch.zeros_like(Lh)
    Dx = torch.zeros(n_p, n_p, dtype=torch.uint8, device=dev())
    P.sym_gemm_pair8(Lh, Rh, D, Lx=Lx, Rx=Rx, C0=Ch, C0x=Cx, Dx=Dx, alpha=0.5, beta=-1.25,
                     exps=(eL, eR, eC, eD))
    torch.cuda.synchronize()
    Dhi = D.cpu().numpy().astype(np.float64)
    lc = pair8_unpack(Dx.cpu().numpy())
    got = Dhi + e4m3_values()[lc] * 2.0 ** -(11 + eD)
    ref = 0.5 * Cv + -1.25 * (Lv @ Rv)
    err = rel_fro(got, ref)
    A16, B16 = A.astype(np.float16).astype(np.float64), Bm.astype(np.float16).astype(np.float64)
    plain = rel_fro((0.5 * A16 - 1.25 * (A16 @ B16)).astype(np.float16), ref)
    say("  pair8 rel err", err, "plain fp16", plain)
    assert err < 1.5e-4 and err < plain / 4, (err, plain)
    np.testing.assert_array_equal(Dhi, Dhi.T)
    tab = e4m3_values()  # compare decoded codes: -0 and +0 are one value
    np.testing.assert_array_equal(tab[lc], tab[lc.T])


@pytest.mark.parametrize("n_p", [256, 384])
def test_sym_gemm_pair8_bf16(n_p):
    """FP8 pairs on a BF16 hi part (codes of (M - M_hi) 2^(8+e)): BF16 hi x hi
    plus both cross terms on the e4m3 MFMA, pair addend and pair output,
    against the FP64 product of the represented values; several times closer
    than BF16 storage alone."""
    import torch
    from gpu_util import e4m3_values, pair8_unpack
    say("sym_gemm pair8 bf16", n_p)
    A = inputs.goe(n_p, 76, np.float64)
    Bm = A @ A * 2.5 - 0.75 * np.eye(n_p)
    eL, eR, eC, eD = 7, 5, 7, 3
    Lh, Lx, Lv = _pair8(A, eL, "bf16")
    Rh, Rx, Rv = _pair8(Bm, eR, "bf16")
    Ch, Cx, Cv = _pair8(A, eC, "bf16")
    D = torch.zeros_like(Lh)
    Dx = torch.zeros(n_p, n_p, dtype=torch.uint8, device=dev())
    P.sym_gemm_pair8(Lh, Rh, D, Lx=Lx, Rx=Rx, C0=Ch, C0x=Cx, Dx=Dx, alpha=0.5, beta=-1.25,
                     exps=(eL, eR, eC, eD))
    torch.cuda.synchronize()
    Dhi = D.to(torch.float64).cpu().numpy()
    lc = pair8_unpack(Dx.cpu().numpy())
    got = Dhi + e4m3_values()[lc] * 2.0 ** -(8 + eD)
    ref = 0.5 * Cv + -1.25 * (Lv @ Rv)
    err = rel_fro(got, ref)
    _, A16 = _rounded(A, "bf16")
    _, B16 = _rounded(Bm, "bf16")
    plain = rel_fro(0.5 * A16 - 1.25 * (A16 @ B16), ref)
    say("  pair8 bf16 rel err", err, "plain bf16 operands", plain)
    assert err < plain / 3, (err, plain)
    assert err < 2e-3, err
    np.testing.assert_array_equal(Dhi, Dhi.T)


@pytest.mark.parametrize("n_p", [512, 768])
def test_sym_gemm_pair8_tile_shapes_agree(n_p):
    """The FP8-pair product on 128 and on 256 tiles: bitwise-identical FP16
    parts and codes (every element takes its 32-K units in the same order)."""
    import torch
    say("sym_gemm pair8 tiles", n_p)
    A = inputs.goe(n_p, 73, np.float64)
    Bm = A @ A * 2.5 - 0.75 * np.eye(n_p)
    Lh, Lx, _ = _pair8(A, 7)
    Rh, Rx, _ = _pair8(Bm, 5)
    outs = []
    try:
        for tile in (128, 256):
            P.tune("gemm_tile", tile)
            D = torch.zeros_like(Lh)
            Dx = torch.zeros(n_p, n_p, dtype=torch.uint8, device=dev())
            P.sym_gemm_pair8(Lh, Rh, D, Lx=Lx, Rx=Rx, C0=Lh, C0x=Lx, Dx=Dx, alpha=0.5, beta=-1.25,
                             exps=(7, 5, 7, 3))
            torch.cuda.synchronize()
            outs.append((D.cpu(), Dx.cpu()))
    finally:
        P.tune("gemm_tile", 0)
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("n_p", [256, 384])
def test_sym_gemm_pair8_one_sided(n_p):
    """One-sided FP8-pair product (L split, R plain FP16): L_hi R_hi on FP16
    MFMAs plus the single cross term L_lo R_hi, two K-units per FP8 MFMA,
    with a pair output. Checked against the FP64 product of the represented
    values (upper triangle, mirrored: the computed triangle is L R at i <= j);
    L rounded to FP16 instead would be several times further off."""
    import torch
    from gpu_util import e4m3_values, pair8_unpack
    say("sym_gemm pair8 one-sided", n_p)
    A = inputs.goe(n_p, 74, np.float64)
    Bm = A @ A * 2.5 - 0.75 * np.eye(n_p)
    Ah = A.astype(np.float16).astype(np.float64)
    # ||Bm|| <= ~9.25 (pair exponent 5), ||4 A + Bm A|| <= ~27 (3)
    eL, eR, eD = 5, 7, 3
    Lh, Lx, Lv = _pair8(Bm, eL)
    R = to_dev(Ah.astype(np.float16))
    D = torch.zeros_like(Lh)
    Dx = torch.zeros(n_p, n_p, dtype=torch.uint8, device=dev())
    P.sym_gemm_pair8(Lh, R, D, Lx=Lx, C0=R, Dx=Dx, alpha=4.0, beta=1.0, exps=(eL, eR, 0, eD))
    torch.cuda.synchronize()
    Dhi = D.cpu().numpy().astype(np.float64)
    lc = pair8_unpack(Dx.cpu().numpy())
    got = Dhi + e4m3_values()[lc] * 2.0 ** -(11 + eD)
    ref = _sym_upper_ref(4.0 * Ah + Lv @ Ah)
    err = rel_fro(got, ref)
    B16 = Bm.astype(np.float16).astype(np.float64)
    plain = rel_fro(_sym_upper_ref(4.0 * Ah + B16 @ Ah), ref)
    say("  one-sided rel err", err, "L rounded to fp16", plain)
    assert err < plain / 4, (err, plain)
    np.testing.assert_array_equal(Dhi, Dhi.T)
    tab = e4m3_values()
    np.testing.assert_array_equal(tab[lc], tab[lc.T])
    # R split without L split is not a supported form
    with pytest.raises(P.PsdprojError):
        P.sym_gemm_pair8(R, Lh, D, Rx=Lx, exps=(eR, eL, 0, 0))


@pytest.mark.parametrize("n_p", [512, 768])
def test_sym_gemm_pair8_one_sided_tile_shapes_agree(n_p):
    """The one-sided product on 128 and on 256 tiles: bitwise-identical
    results (both pair the same K-units into each FP8 MFMA)."""
    import torch
    say("sym_gemm pair8 one-sided tiles", n_p)
    A = inputs.goe(n_p, 75, np.float64)
    Bm = A @ A * 2.5 - 0.75 * np.eye(n_p)
    Lh, Lx, _ = _pair8(Bm, 5)
    R = to_dev(A.astype(np.float16))
    outs = []
    try:
        for tile in (128, 256):
            P.tune("gemm_tile", tile)
            D = torch.zeros_like(Lh)
            P.sym_gemm_pair8(Lh, R, D, Lx=Lx, C0=R, alpha=4.0, beta=1.0, exps=(5, 7, 0, 0))
            torch.cuda.synchronize()
            outs.append(D.cpu())
    finally:
        P.tune("gemm_tile", 0)
    assert torch.equal(outs[0], outs[1])


def test_sym_gemm_pair8_plain_operands_pair_output():
    """Unsplit operands with a pair addend and a pair output (the product that
    feeds the first split stage)."""
    import torch
    from gpu_util import e4m3_values, pair8_unpack
    n_p = 256
    say("sym_gemm pair8 plain operands")
    A = inputs.goe(n_p, 72, np.float64)
    Ah = A.astype(np.float16).astype(np.float64)
    Ch, Cx, Cv = _pair8(A, 7)
    L = to_dev(Ah.astype(np.float16))
    D = torch.zeros_like(L)
    Dx = torch.zeros(n_p, n_p, dtype=torch.uint8, device=dev())
    # ||D|| <= 2 * 2 + 0.75 * 4 = 7: pair exponent 5 keeps codes below 448
    P.sym_gemm_pair8(L, L, D, C0=Ch, C0x=Cx, Dx=Dx, alpha=2.0, beta=0.75, exps=(0, 0, 7, 5))
    torch.cuda.synchronize()
    lc = pair8_unpack(Dx.cpu().numpy())
    got = D.cpu().numpy().astype(np.float64) + e4m3_values()[lc] * 2.0 ** -16
    ref = 2.0 * Cv + 0.75 * (Ah @ Ah)
    assert rel_fro(got, ref) < 5e-5, rel_fro(got, ref)
