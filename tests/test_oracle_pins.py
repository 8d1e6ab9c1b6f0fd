"""Pins of the FP64 oracle against what the paper and the mathematics fix.

No GPU. Each test names the passage it pins. Mistakes these are meant to catch:
a mistyped coefficient (e_float), a dropped or mis-signed term in the matrix
filter (spectral identity, diagonal closed form), a transposed or wrong-sided
product (spectral identity on non-diagonal Q), a wrong bound (Theorem 2
validity and exactness on small n), a broken eigensolver (2x2 closed form,
projection invariants)."""
import os

import numpy as np
import pytest

import oracle
from oracle import tables
from paper_2507_09165_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_efloat():
    out = {}
    with open(os.path.join(GOLDEN, "efloat_printed.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val, pinned = line.split()
            out[name] = (float(val), pinned == "yes")
    return out


# --------------------------------------------------------------------------
# Coefficient tables (Tables 1 and 2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["f_tilde_single", "f_star_half", "f_tilde_half"])
def test_efloat_reproduces_printed_value(name):
    """Tables 1-2 bottom row: e_float recomputed over all float32 in [-1,1]."""
    printed, pinned = _golden_efloat()[name]
    assert pinned
    twice, _ = oracle.efloat(name)
    assert abs(twice / printed - 1.0) < 5e-3, (twice, printed)


def test_efloat_golden_matches_table_module():
    g = _golden_efloat()
    for k, (v, _) in g.items():
        assert tables.PRINTED_EFLOAT[k] == v


def test_fixed_point_stages_are_newton_schulz_quintic():
    """Table 1: the last two Stage-I single stages are (15x - 10x^3 + 3x^5)/8,
    the quintic whose fixed points are +-1 with zero first and second
    derivative (it maps [a,1] into itself once a is close to 1)."""
    ns = np.array([15 / 8, -10 / 8, 3 / 8])
    np.testing.assert_array_equal(tables.F_STAR_SINGLE[8], ns)
    np.testing.assert_array_equal(tables.F_STAR_SINGLE[9], ns)
    # f(1) = 1, f'(1) = 0 for that quintic
    a, b, c = ns
    assert abs(a + b + c - 1.0) < 1e-15 and abs(a + 3 * b + 5 * c) < 1e-15


def test_each_refined_stage_maps_one_near_one():
    """Every stage approximates sign on its interval, so f_t(1) ~ 1 (within
    the Stage-I minimax error of stage 1, about 1 - 0.99)."""
    for name in ("f_tilde_half", "f_tilde_single"):
        for a, b, c in tables.TABLES[name]:
            assert abs(a + b + c - 1.0) < 1.0


def test_gemm_counts():
    """Section 3.3: 31 GEMMs in single, 22 in half precision."""
    assert oracle.gemm_count("fp32") == 31
    assert oracle.gemm_count("fp16") == 22


def test_rescale_reading_keeps_error_small():
    """Section 3.4 rescale: with 1/1.01 after stages 1..6 (reading adopted),
    the ReLU error stays near the table's own; rescaling after stage 7 too
    would leave ~5e-3."""
    twice, _ = oracle.efloat("f_tilde_half", with_rescale=True)
    assert twice / 2 < 5e-5
    rows = tables.TABLES["f_tilde_half"] / 1.01
    x = np.linspace(0.5, 1.0, 2001)
    p = oracle.psd.composite_scalar(x, rows)
    assert np.max(np.abs(0.5 * x * (1 + p) - x)) > 4e-3


# --------------------------------------------------------------------------
# Exact projection (eq. (1), closed form eq. (3))
# --------------------------------------------------------------------------
def test_exact_diagonal():
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.0, 1e-9, -1e-9])
    P = oracle.project_exact(np.diag(d))
    np.testing.assert_array_equal(np.diag(np.diag(P)), P)
    np.testing.assert_allclose(np.diag(P), np.maximum(d, 0.0), rtol=0, atol=1e-15)


@pytest.mark.parametrize("a,b,c", [(1.0, 2.0, -1.0), (0.3, -0.7, 0.1), (-2.0, 0.5, -1.0), (2.0, 0.1, 1.0)])
def test_exact_2x2_closed_form(a, b, c):
    X = np.array([[a, b], [b, c]])
    h = 0.5 * (a + c)
    d = np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    lp, lm = h + d, h - d
    if lp <= 0:
        ref = np.zeros((2, 2))
    elif lm >= 0:
        ref = X
    else:
        ref = lp * (X - lm * np.eye(2)) / (lp - lm)
    np.testing.assert_allclose(oracle.project_exact(X), ref, atol=1e-14)


def _sym(n, seed):
    return inputs.goe(n, seed, np.float64)


def test_exact_projection_invariants():
    X = _sym(48, 3)
    P = oracle.project_exact(X)
    nx = np.linalg.norm(X)
    w = np.linalg.eigvalsh(P)
    assert w.min() > -1e-12 * nx                        # P is PSD
    assert np.linalg.eigvalsh(X - P).max() < 1e-12 * nx  # X - P is NSD
    assert abs(np.sum(P * (X - P))) < 1e-12 * nx * nx    # complementarity
    np.testing.assert_allclose(oracle.project_exact(P), P, atol=1e-12 * nx)  # idempotent
    Pm = oracle.project_exact(-X)
    np.testing.assert_allclose(P - Pm, X, atol=1e-12 * nx)  # Moreau decomposition
    np.testing.assert_allclose(oracle.project_exact(2.5 * X), 2.5 * P, atol=1e-12 * nx)
    Q = inputs.haar_orthogonal(48, 9)
    np.testing.assert_allclose(oracle.project_exact(Q @ X @ Q.T), Q @ P @ Q.T, atol=1e-11 * nx)


def test_exact_matches_constructed_spectrum_and_lapack():
    X32, Q, lam = inputs.constructed(64, 0, 1)
    X = X32.astype(np.float64)
    P = oracle.project_exact(X)
    np.testing.assert_allclose(P, oracle.project_exact_eigh(X), atol=1e-12)
    ref = (Q * np.maximum(lam, 0)) @ Q.T
    # X32 is the FP32 rounding of Q diag(lam) Q^T; the projection is 1-Lipschitz
    assert np.linalg.norm(P - ref) <= np.linalg.norm(X - (Q * lam) @ Q.T) * 1.0001 + 1e-12


def test_jacobi_eigenvalues_match_brute_force_small():
    for n in (1, 2, 3):
        X = _sym(n, 20 + n)
        w, V = oracle.jacobi_eig(X)
        np.testing.assert_allclose(np.sort(w), np.linalg.eigvalsh(X), atol=1e-13)
        np.testing.assert_allclose(V @ np.diag(w) @ V.T, X, atol=1e-13)


# --------------------------------------------------------------------------
# Spectral bound (Theorem 2 + Lanczos)
# --------------------------------------------------------------------------
def test_splitmix64_known_answers():
    want = []
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                want.append(int(line, 16))
    z = oracle.psd.splitmix64(np.arange(len(want), dtype=np.uint64), 0)
    assert [int(v) for v in z] == want


@pytest.mark.parametrize("n", [1, 2, 5, 13, 20])
def test_lanczos_exact_when_krylov_space_is_complete(n):
    """With n <= 20 steps the Krylov space is all of R^n: sigma = ||X||_2^2 and
    the residual vanishes, so the bound equals ||X||_2."""
    X = _sym(n, 100 + n)
    lz = oracle.lanczos_bound(X)
    true = np.max(np.abs(np.linalg.eigvalsh(X)))
    assert abs(lz["lam"] - true) <= 1e-7 * true
    assert abs(lz["sigma"] - true ** 2) <= 1e-12 * true ** 2


def test_bound_valid_and_tight_on_known_spectra():
    """Theorem 2: lam >= ||X||_2; and the 20-step bound is within 1%."""
    cases = [inputs.constructed(256, 0, 1)[0], inputs.clustered(256, 3)[0], inputs.goe(300, 2)]
    for X in cases:
        Xs = X.astype(np.float64)
        true = np.max(np.abs(np.linalg.eigvalsh(Xs)))
        b = oracle.spectral_bound(Xs)
        assert not b["fallback"]
        assert b["lam"] >= true * (1 - 1e-12)
        assert b["lam"] <= 1.01 * true


def test_bound_diagonal():
    d = np.array([0.5, -3.0, 2.0, 1e-3, -2.9])
    b = oracle.spectral_bound(np.diag(d))
    assert 3.0 <= b["lam"] <= 3.0 * 1.01


def test_bound_zero_matrix():
    b = oracle.spectral_bound(np.zeros((7, 7)))
    assert b["lam"] == 0.0


def _golden_start_pair():
    """Normalised Lanczos start vector of order 2, from the SplitMix64 known
    answers (entries 2 (z >> 11) 2^-53 - 1), computed here without the
    oracle's generator."""
    z = []
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                z.append(int(line, 16))
    v = np.array([2.0 * (zi >> 11) * 2.0 ** -53 - 1.0 for zi in z[:2]])
    return v / np.linalg.norm(v)


def test_bound_one_step_closed_form_cap_and_guard():
    """Theorem 2 with a single Lanczos step on X = s * diag(1, 0) or
    s * diag(0, 1): q is the start vector (c, d), sigma = s^2 c^2 (resp.
    s^2 d^2) and ||X^2 q - sigma q|| = s^2 |c d|, so the raw bound is
    s sqrt(c^2 + |c d|) (resp. s sqrt(d^2 + |c d|)). With |c| > |d| the first
    exceeds ||X||_F = s and must be capped to it; the second falls below the
    column-norm lower bound s and the guard must replace it by ||X||_F."""
    c, d = _golden_start_pair()
    assert abs(c) > abs(d)
    s = 3.0
    cap = oracle.spectral_bound(np.diag([s, 0.0]), steps=1)
    raw_cap = s * np.sqrt(c * c + abs(c * d))
    assert raw_cap > s
    assert cap["lanczos_lam"] == pytest.approx(raw_cap, rel=1e-13)
    assert cap["lam"] == pytest.approx(s, rel=1e-15) and not cap["fallback"]
    guard = oracle.spectral_bound(np.diag([0.0, s]), steps=1)
    raw_guard = s * np.sqrt(d * d + abs(c * d))
    assert raw_guard < s
    assert guard["lanczos_lam"] == pytest.approx(raw_guard, rel=1e-13)
    assert guard["lam"] == pytest.approx(s, rel=1e-15) and guard["fallback"]
    assert guard["colmax"] == pytest.approx(s, rel=1e-15)


def test_bound_forced_fallback_gives_frobenius():
    """The guard's branch on a larger input: with the Lanczos bound halved
    (test hook) it falls below max_j ||X e_j|| = max |d_i| of a diagonal
    matrix, so the bound becomes ||X||_F = ||d||_2 and the fallback is
    reported; without the hook the same matrix keeps its Lanczos bound."""
    d = np.array([0.5, -3.0, 2.0, 1e-3, -2.9, 1.25])
    plain = oracle.spectral_bound(np.diag(d))
    assert not plain["fallback"] and plain["lam"] < np.linalg.norm(d)
    forced = oracle.spectral_bound(np.diag(d), force_fallback=True)
    assert forced["fallback"]
    assert forced["lam"] == pytest.approx(np.linalg.norm(d), rel=1e-15)
    assert forced["lanczos_lam"] == pytest.approx(plain["lanczos_lam"], rel=1e-15)
    P, info = oracle.project_poly(np.diag(d), "fp16", force_fallback=True)
    assert info["fallback"] and info["lam"] == forced["lam"]
    lam = forced["lam"]
    np.testing.assert_allclose(np.diag(P), lam * oracle.g_scalar(d / lam, "fp16"), rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------
# Composite polynomial projection (Algorithm 2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["fp16", "fp32"])
def test_poly_spectral_identity(mode):
    """p(X) = Q p(Lambda) Q^T (eq. (4)-(5)): the matrix filter equals the scalar
    function g applied to the scaled eigenvalues."""
    n = 40
    Q = inputs.haar_orthogonal(n, 5)
    lam = np.random.default_rng(6).uniform(-1.3, 0.9, n)
    X = (Q * lam) @ Q.T
    X = 0.5 * (X + X.T)
    lt = 1.37
    P, _ = oracle.project_poly(X, mode, lam=lt)
    ref = oracle.project_spectral(Q, lam, lambda l: lt * oracle.g_scalar(l / lt, mode))
    np.testing.assert_allclose(P, ref, atol=1e-12)


@pytest.mark.parametrize("mode", ["fp16", "fp32"])
def test_poly_diagonal(mode):
    d = np.array([0.9, -0.4, 1e-4, -1e-4, 0.0, 0.33])
    P, info = oracle.project_poly(np.diag(d), mode)
    lt = info["lam"]
    np.testing.assert_allclose(P, np.diag(lt * oracle.g_scalar(d / lt, mode)), atol=1e-15)


@pytest.mark.parametrize("mode,eps", [("fp16", 4.6506e-5), ("fp32", 4.2237e-6)])
def test_poly_error_within_scalar_bound(mode, eps):
    """Every eigenvalue of R_poly is within e_inf * lam of ReLU(lambda), so
    ||R_poly - R_exact||_2 <= e_inf * lam (eq. (12) error on the float grid,
    stage rescale folded in)."""
    X32, Q, lam = inputs.constructed(128, 0, 1)
    X = X32.astype(np.float64)
    P, info = oracle.project_poly(X, mode)
    E = P - oracle.project_exact(X)
    assert np.max(np.abs(np.linalg.eigvalsh(E))) <= eps * info["lam"] * 1.02
    assert np.linalg.eigvalsh(P).min() >= -eps * info["lam"] * 1.02


def test_poly_scalar_efloat_equals_spot_values():
    twice, arg = oracle.efloat("f_tilde_half", with_rescale=True)
    g = oracle.g_scalar(np.array([arg, -arg]), "fp16")
    assert abs(abs(g[0] - arg) - twice / 2) < 1e-12
    assert abs(abs(g[1]) - twice / 2) < 1e-12


def test_poly_n1():
    for x in (2.5, -0.75):
        P, info = oracle.project_poly(np.array([[x]]), "fp16")
        assert abs(info["lam"] - abs(x)) < 1e-12
        assert abs(P[0, 0] - abs(x) * oracle.g_scalar(np.sign(x), "fp16")) < 1e-12


def test_poly_homogeneity_and_symmetry():
    X = _sym(60, 8)
    P1, i1 = oracle.project_poly(X, "fp32")
    P2, i2 = oracle.project_poly(3.0 * X, "fp32")
    assert abs(i2["lam"] / i1["lam"] - 3.0) < 1e-10
    np.testing.assert_allclose(P2, 3.0 * P1, atol=1e-10 * np.linalg.norm(P1))
    np.testing.assert_array_equal(P1, P1.T)


def test_poly_reads_upper_triangle_only():
    X = _sym(30, 4)
    Y = X.copy()
    Y[np.tril_indices(30, -1)] = 1e6
    P1, _ = oracle.project_poly(X, "fp16")
    P2, _ = oracle.project_poly(Y, "fp16")
    np.testing.assert_array_equal(P1, P2)


def test_poly_zero_and_empty():
    P, _ = oracle.project_poly(np.zeros((5, 5)), "fp16")
    assert not P.any()
    P, _ = oracle.project_poly(np.zeros((0, 0)), "fp16")
    assert P.shape == (0, 0)


def test_poly_relative_error_floor_matches_exact_arithmetic():
    """The FP64 composite's distance to the exact projection on the n=256
    workload sits at the approximation floor (~2.4e-6 single table, ~3.5e-5
    half table) — well under the 1e-3 target."""
    X32, Q, lam = inputs.constructed(256, 0, 1)
    X = X32.astype(np.float64)
    R = oracle.project_exact_eigh(X)
    for mode, cap in (("fp32", 5e-6), ("fp16", 6e-5)):
        P, _ = oracle.project_poly(X, mode)
        rel = np.linalg.norm(P - R) / np.linalg.norm(R)
        assert rel < cap, (mode, rel)


# --------------------------------------------------------------------------
# Newton-Schulz baseline (Section 4.1, "Benchmark methods and metrics")
# --------------------------------------------------------------------------
def test_ns_structure_matches_printed_product_counts():
    """10 half-precision iterations give 21 products, 15 single-precision ones
    31 (Section 4.1's list of compared methods)."""
    assert oracle.NS_ITERS == {"ns_fp16": 10, "ns_fp32": 15}
    assert oracle.gemm_count("ns_fp16") == 21
    assert oracle.gemm_count("ns_fp32") == 31


def _ns_by_error_recursion(x, iters):
    """The cubic sign iteration written in its error variable: with
    e = 1 - |x|, one step gives e' = e^2 (3 - e) / 2 (since
    1 - (3y - y^3)/2 = (1 - y)^2 (y + 2) / 2 and y + 2 = 3 - e); odd in x."""
    x = np.asarray(x, dtype=np.float64)
    e = 1.0 - np.abs(x)
    for _ in range(iters):
        e = e * e * (3.0 - e) / 2.0
    return np.sign(x) * (1.0 - e)


def test_ns_scalar_equals_error_recursion():
    x = np.concatenate([np.linspace(-1.0, 1.0, 2001), [1e-4, -3e-3, 0.999]])
    for mode, k in oracle.NS_ITERS.items():
        got = oracle.psd.composite_scalar(x, oracle.stage_rows(mode))
        np.testing.assert_allclose(got, _ns_by_error_recursion(x, k), atol=1e-13)


def test_ns_converges_to_sign_inside_sqrt3_only():
    """The cubic iteration converges to sign(x) for 0 < |x| < sqrt(3); at
    sqrt(3) < |x| < 2 one step flips the sign (it then converges to -sign(x)),
    and beyond |f(x)| > sqrt(3) it diverges (f(3) = -9)."""
    rows = np.tile(np.array([[1.5, -0.5, 0.0]]), (80, 1))
    inside = np.array([1e-3, 0.3, 1.0, 1.5, 1.73, -0.02, -1.7])
    np.testing.assert_allclose(oracle.psd.composite_scalar(inside, rows), np.sign(inside), atol=1e-12)
    flipped = np.array([1.74, 1.9, -1.8])
    np.testing.assert_allclose(oracle.psd.composite_scalar(flipped, rows), -np.sign(flipped), atol=1e-12)
    assert oracle.psd.composite_scalar(np.array([3.0]), rows[:1])[0] == -9.0
    with np.errstate(over="ignore", invalid="ignore"):
        out = oracle.psd.composite_scalar(np.array([3.0, -3.0]), np.tile(rows[:1], (4, 1)))
    assert np.all(~np.isfinite(out) | (np.abs(out) > 1e6))


@pytest.mark.parametrize("mode", ["ns_fp16", "ns_fp32"])
def test_ns_matrix_equals_spectral_form(mode):
    """Projection by the Newton-Schulz baseline on X = Q diag(l) Q^T equals
    Q diag(lam g(l / lam)) Q^T with g(x) = x (1 + s(x)) / 2 and s the
    iteration evaluated through its error recursion."""
    n = 40
    Q = inputs.haar_orthogonal(n, 7)
    lam = np.random.default_rng(8).uniform(-1.2, 1.1, n)
    X = (Q * lam) @ Q.T
    X = 0.5 * (X + X.T)
    lt = 1.31
    P, _ = oracle.project_poly(X, mode, lam=lt)
    k = oracle.NS_ITERS[mode]
    ref = oracle.project_spectral(Q, lam, lambda l: lt * 0.5 * (l / lt) * (1.0 + _ns_by_error_recursion(l / lt, k)))
    np.testing.assert_allclose(P, ref, atol=1e-12)


def test_ns_less_accurate_than_composite_on_dense_spectrum():
    """With a fifth of the eigenvalues within 1e-3 of zero, the composite
    filter is more accurate than Newton-Schulz with about as many products, in
    both settings (Section 4.1, "Results"; in exact arithmetic here)."""
    X = inputs.clustered(200, 3)[0].astype(np.float64)
    ex = oracle.project_exact(X)
    e = {}
    for mode in ("fp16", "ns_fp16", "fp32", "ns_fp32"):
        P, _ = oracle.project_poly(X, mode)
        e[mode] = np.linalg.norm(P - ex) / np.linalg.norm(ex)
    assert e["fp16"] < 1e-4 < e["ns_fp16"]
    assert e["fp32"] < 1e-5 < e["ns_fp32"]


# --------------------------------------------------------------------------
# Deflation of dominant eigenpairs (Section 4.1 "Results"; Section 5)
# --------------------------------------------------------------------------
def _dominant(n, seed, top):
    return inputs.dominant(n, seed, top)


def test_deflation_finds_the_dominant_pairs_with_sign():
    X, Q, lam = _dominant(300, 11, [200.0, -60.0])
    mu, Z, r = oracle.deflation_pairs(X, 4)
    np.testing.assert_allclose(mu, [200.0, -60.0], rtol=1e-12)
    for i in range(2):
        assert abs(abs(Z[:, i] @ Q[:, i]) - 1.0) < 1e-12
    assert np.all(r <= 1e-8 * np.abs(mu))


def test_deflated_projection_spectral_identity():
    """With the dominant pairs removed exactly, the result is ReLU on them and
    the filter with the deflated matrix's own bound on the rest."""
    X, Q, lam = _dominant(300, 11, [200.0, -60.0])
    P, info = oracle.project_deflated(X, "fp16", kmax=2)
    lt = info["lam"]
    assert lt < 1.01  # the bound of the deflated matrix
    f = lt * oracle.g_scalar(lam / lt, "fp16")
    f[:2] = np.maximum(lam[:2], 0.0)
    ref = oracle.project_spectral(Q, lam, lambda l: f)
    np.testing.assert_allclose(P, ref, atol=1e-10)


def test_deflation_gate_leaves_unconverged_spectra_alone():
    X = inputs.goe(200, 2).astype(np.float64)
    mu, Z, r = oracle.deflation_pairs(X, 4)
    assert mu.size == 0
    P0, _ = oracle.project_poly(X, "fp16")
    P1, _ = oracle.project_deflated(X, "fp16", kmax=4)
    np.testing.assert_array_equal(P0, P1)


def test_deflation_fixes_one_dominant_eigenvalue():
    """One eigenvalue 1000x the rest: undeflated, the rest of the spectrum is
    scaled below the filter's resolved interval; deflated, it is filtered at
    the paper's half-precision accuracy."""
    X, Q, lam = _dominant(400, 11, [1000.0])
    ex = oracle.project_exact_eigh(X)
    rest = ex - 1000.0 * np.outer(Q[:, 0], Q[:, 0])
    e = []
    for k in (0, 1):
        P, _ = oracle.project_deflated(X, "fp16", kmax=k)
        e.append(np.linalg.norm(P - ex) / np.linalg.norm(rest))
    assert e[0] > 1e-2 and e[1] < 1e-4


# --------------------------------------------------------------------------
# Adaptive depth (Section 5, "Limitations and future work")
# --------------------------------------------------------------------------
def _quintic_by_error(x):
    """(15 x - 10 x^3 + 3 x^5) / 8 through its fixed-point form:
    1 - f(x) = (1 - x)^3 (3 x^2 + 9 x + 8) / 8 for x >= 0, odd in x."""
    a = np.abs(x)
    return np.sign(x) * (1.0 - (1.0 - a) ** 3 * (3.0 * a * a + 9.0 * a + 8.0) / 8.0)


def test_adaptive_ns_stops_where_the_scalar_iteration_converges():
    """On X = Q diag(l) Q^T the relative change of a Newton-Schulz step is
    ||s_k(l) - s_{k-1}(l)|| / ||s_{k-1}(l)|| with s the scalar iteration (its
    error recursion); the adaptive run stops at the first step whose change is
    at most the tolerance, and equals the fixed run of that many steps."""
    X32, Q, lam = inputs.constructed(300, 0, 1, lo=0.2, hi=1.0)
    X = (Q * lam) @ Q.T
    X = 0.5 * (X + X.T)
    lt = oracle.spectral_bound(X)["lam"]
    x = lam / lt
    changes = []
    for k in range(1, 16):
        xn = _ns_by_error_recursion(x, 1)
        changes.append(np.linalg.norm(xn - x) / np.linalg.norm(x))
        x = xn
    for tol in (2e-3, 1e-5, 1e-8):
        k = next(i + 1 for i, c in enumerate(changes) if c <= tol)
        assert changes[k - 1] < 0.5 * tol and changes[k - 2] > 2.0 * tol  # clear-cut
        P, info = oracle.project_poly(X, "ns_fp32", lam=lt, adaptive_tol=tol)
        assert info["stages"] == k
        ref = oracle.project_spectral(
            Q, lam, lambda l: lt * 0.5 * (l / lt) * (1.0 + _ns_by_error_recursion(l / lt, k)))
        np.testing.assert_allclose(P, ref, atol=1e-12)


def test_adaptive_extra_quintic_stages_spectral_identity():
    """Composite filter plus extra quintic stages: the matrix result is the
    scalar composite followed by the quintic's fixed-point form, per
    eigenvalue; with tol = 0 every extra stage runs."""
    n = 60
    Q = inputs.haar_orthogonal(n, 9)
    lam = np.random.default_rng(10).uniform(-1.0, 1.0, n)
    X = (Q * lam) @ Q.T
    X = 0.5 * (X + X.T)
    lt = 1.05
    P, info = oracle.project_poly(X, "fp16", lam=lt, adaptive_extra=2)
    assert info["stages"] == 9

    def g(l):
        y = oracle.psd.composite_scalar(l / lt, oracle.stage_rows("fp16"))
        y = _quintic_by_error(_quintic_by_error(y))
        return lt * 0.5 * (l / lt) * (1.0 + y)
    np.testing.assert_allclose(P, oracle.project_spectral(Q, lam, g), atol=1e-12)


def test_adaptive_extra_stages_reach_the_exact_projection():
    """On a GOE spectrum one or two quintic stages after the composite filter
    take the exact-arithmetic error from ~3e-5 to rounding level, and the
    tolerance stops them there."""
    X = inputs.goe(300, 1).astype(np.float64)
    ex = oracle.project_exact_eigh(X)
    P0, i0 = oracle.project_poly(X, "fp16")
    P1, i1 = oracle.project_poly(X, "fp16", adaptive_tol=1e-8, adaptive_extra=6)
    e0 = np.linalg.norm(P0 - ex) / np.linalg.norm(ex)
    e1 = np.linalg.norm(P1 - ex) / np.linalg.norm(ex)
    assert e0 > 1e-5 and e1 < 1e-12
    assert i0["stages"] == 7 and 8 <= i1["stages"] <= 10
