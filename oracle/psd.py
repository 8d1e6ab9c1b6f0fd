"""FP64 CPU oracle of the PSD-cone projection by composite polynomial filtering.

ORACLE — test infrastructure only. It shares no code with the HIP library and
is imported only by tests/, the smoke check and the benchmark's CPU-baseline
leg. Everything here is plain FP64 numpy; a matrix product (``@``) and a small
symmetric eigensolver (``numpy.linalg.eigh`` on the Lanczos tridiagonal) are the
only library primitives used as steps.

Functions and the passages they follow:

* ``project_exact``      — the projection problem, eq. (1), solved by the
                           closed form of eq. (3) with a Jacobi eigensolver.
* ``lanczos_bound``      — Theorem 2 (residual-norm bound on ||A||_2) with the
                           largest Ritz pair of a 20-step Lanczos run on X^2
                           (Section 3.4, "Digit loss during matrix rescaling";
                           Algorithm 2, first two steps).
* ``project_poly``       — Algorithm 2 (run-time projection): rescale by the
                           bound, apply the T filter stages, return
                           lambda * X0 (I + X_T) / 2.
* ``g_scalar``           — the scalar function the matrix filter applies to
                           each scaled eigenvalue, eq. (5)/(11):
                           x (1 + p(x)) / 2.
* ``efloat``             — eq. (12), the maximum error over all float32 values
                           in [-1, 1].
* ``project_deflated``   — deflation of converged dominant eigenpairs before
                           filtering, the remedy Section 4.1 ("Results") and
                           Section 5 propose for spectra with a few dominant
                           eigenvalues (our reading: Rayleigh-Ritz pairs of X
                           in the bound's Krylov basis, gated by residual).
* ``newton_schulz_stage``— the cubic Newton-Schulz step of the baseline in
                           Section 4.1 ("Benchmark methods and metrics"); the
                           ``ns_fp16`` / ``ns_fp32`` modes of ``project_poly``
                           run 10 / 15 of them in place of the filter stages.

Readings of the paper taken here (each also listed in the design notes):

* The input is symmetric and only its upper triangle is read.
* The Lanczos start vector is a fixed pseudo-random vector from the SplitMix64
  counter generator (seed 0), normalised; full reorthogonalisation by two
  passes of classical Gram-Schmidt; stop early when beta <= 1e-13 max|alpha|.
* Guard (not in the paper): the bound must be at least the largest column norm
  (a valid lower bound on ||X||_2), else the Frobenius norm is used; the bound
  is also capped by the Frobenius norm, itself an upper bound on ||X||_2.
* Stage rescale placement: see ``oracle.tables``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import tables

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

LANCZOS_STEPS = 20
LANCZOS_SEED = 0
BREAKDOWN_RTOL = 1e-13


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_jacobi_eig.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_double]
        lib.oracle_jacobi_eig.restype = ctypes.c_int
        lib.oracle_project_jacobi.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.oracle_project_jacobi.restype = ctypes.c_int
        lib.oracle_efloat.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_efloat.restype = ctypes.c_double
        _LIB = lib
    return _LIB


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# Input handling
# ---------------------------------------------------------------------------
def sym_from_upper(X) -> np.ndarray:
    """FP64 symmetric matrix built from the upper triangle of X (uplo = 'U')."""
    X = np.asarray(X, dtype=np.float64)
    U = np.triu(X)
    return U + np.triu(X, 1).T


# ---------------------------------------------------------------------------
# Lanczos start vector: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), used as
# a counter-based generator: z_i = mix(seed + (i + 1) * golden_gamma).
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray, seed: int = 0) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def start_vector(n: int, seed: int = LANCZOS_SEED) -> np.ndarray:
    """Entries uniform in [-1, 1): 2 * (z >> 11) * 2^-53 - 1 (not normalised)."""
    z = splitmix64(np.arange(n, dtype=np.uint64), seed)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


# ---------------------------------------------------------------------------
# Spectral bound (Theorem 2 + Lanczos on X^2)
# ---------------------------------------------------------------------------
def lanczos_run(Xs: np.ndarray, steps: int = LANCZOS_STEPS, seed: int = LANCZOS_SEED):
    """``steps`` Lanczos steps on A = X^2 (A applied as X (X v), never formed),
    full reorthogonalisation by two classical Gram-Schmidt passes.

    Returns (V, T) with V the n x k orthonormal Krylov basis and T its k x k
    tridiagonal, k the number of steps taken (early stop on breakdown)."""
    n = Xs.shape[0]
    v = start_vector(n, seed)
    v = v / np.linalg.norm(v)
    V = np.zeros((n, steps), dtype=np.float64)
    V[:, 0] = v
    alpha, beta = [], []
    k = 0
    for j in range(steps):
        w = Xs @ (Xs @ V[:, j])
        h = V[:, : j + 1].T @ w          # first Gram-Schmidt pass
        alpha.append(h[j])                # alpha_j = v_j^T A v_j
        w = w - V[:, : j + 1] @ h
        h2 = V[:, : j + 1].T @ w         # second pass (reorthogonalisation)
        w = w - V[:, : j + 1] @ h2
        b = float(np.linalg.norm(w))
        k = j + 1
        amax = max(abs(a) for a in alpha)
        if j == steps - 1 or not (b > BREAKDOWN_RTOL * amax):
            break
        beta.append(b)
        V[:, j + 1] = w / b
    Tm = np.diag(np.array(alpha[:k])) + np.diag(np.array(beta[: k - 1]), 1) \
        + np.diag(np.array(beta[: k - 1]), -1)
    return V[:, :k], Tm


def lanczos_bound(Xs: np.ndarray, steps: int = LANCZOS_STEPS, seed: int = LANCZOS_SEED):
    """Largest Ritz pair (sigma, q) of ``steps`` Lanczos steps on A = X^2, then
    the bound lambda = sqrt(sigma + ||A q - sigma q||_2) of Theorem 2.

    Returns dict(lam, sigma, r, k) with k the number of Lanczos steps taken."""
    V, Tm = lanczos_run(Xs, steps, seed)
    k = V.shape[1]
    theta, S = np.linalg.eigh(Tm)
    sigma = float(theta[-1])
    q = V @ S[:, -1]
    q = q / np.linalg.norm(q)
    res = Xs @ (Xs @ q) - sigma * q
    r = float(np.linalg.norm(res))
    lam = float(np.sqrt(max(sigma + r, 0.0)))
    return {"lam": lam, "sigma": sigma, "r": r, "k": k}


def spectral_bound(Xs: np.ndarray, steps: int = LANCZOS_STEPS, force_fallback: bool = False):
    """Lanczos bound with the guard and the Frobenius cap. Returns dict with
    lam (the bound used), lanczos_lam (sqrt(sigma + r) before the guard),
    fro, colmax, fallback (bool) and the Lanczos fields.

    Guard: a bound below the largest column norm (itself a lower bound on
    ||X||_2) is invalid and is replaced by ||X||_F. Cap: the bound never
    exceeds ||X||_F, which is also an upper bound on ||X||_2.
    ``force_fallback`` halves the Lanczos bound before the guard, so that the
    guard's branch can be exercised on any input (the library has the same
    test hook)."""
    fro = float(np.sqrt(np.sum(Xs * Xs)))
    colmax = float(np.sqrt(np.max(np.sum(Xs * Xs, axis=0)))) if Xs.size else 0.0
    out = {"fro": fro, "colmax": colmax}
    if fro == 0.0:
        out.update(lam=0.0, lanczos_lam=0.0, sigma=0.0, r=0.0, k=0, fallback=False)
        return out
    lz = lanczos_bound(Xs, steps)
    out.update(lz)
    out["lanczos_lam"] = lz["lam"]
    lam = 0.5 * lz["lam"] if force_fallback else lz["lam"]
    fallback = not (lam >= colmax)
    if fallback:
        lam = fro
    out["lam"] = min(lam, fro)
    out["fallback"] = fallback
    return out


# ---------------------------------------------------------------------------
# Composite filter (Algorithm 2)
# ---------------------------------------------------------------------------
# Newton-Schulz baseline (Section 4.1, "Benchmark methods and metrics"): the
# cubic sign iteration x <- (3 x - x^3) / 2, 10 iterations in half precision
# (21 products) and 15 in single precision (31 products), on the same rescaled
# input and with the same final step as Algorithm 2.
NS_ITERS = {"ns_fp16": 10, "ns_fp32": 15}


def stage_rows(mode: str) -> np.ndarray:
    """(a, b, c) per stage with the stage rescale folded in, FP64. The
    Newton-Schulz modes are the cubic (1.5, -0.5, 0) repeated."""
    if mode in NS_ITERS:
        return np.tile(np.array([[1.5, -0.5, 0.0]]), (NS_ITERS[mode], 1))
    return tables.runtime_table(tables.MODE_TABLE[mode])


def composite_scalar(x, rows: np.ndarray):
    x = np.asarray(x, dtype=np.float64)
    for a, b, c in rows:
        x2 = x * x
        x = x * (a + x2 * (b + x2 * c))
    return x


def g_scalar(x, mode: str = "fp16"):
    """x (1 + p(x)) / 2 — the approximation of ReLU on the scaled interval."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + composite_scalar(x, stage_rows(mode)))


def filter_stage(Y: np.ndarray, a: float, b: float, c: float) -> np.ndarray:
    """One odd quintic stage f(Y) = a Y + b Y^3 + c Y^5 of Algorithm 2, with
    the three matrix products A = Y Y, B = b A + c A A, Y' = a Y + Y B."""
    A = Y @ Y
    B = b * A + c * (A @ A)
    return a * Y + Y @ B


def newton_schulz_stage(Y: np.ndarray) -> np.ndarray:
    """One cubic Newton-Schulz step Y' = (3 Y - Y^3) / 2 with two matrix
    products: A = Y Y, Y' = 1.5 Y - 0.5 Y A."""
    A = Y @ Y
    return 1.5 * Y - 0.5 * (Y @ A)


def final_combine(X0: np.ndarray, Y: np.ndarray, lam: float) -> np.ndarray:
    """Return step of Algorithm 2: lam X0 (I + X_T) / 2, symmetrised."""
    P = lam * 0.5 * (X0 + X0 @ Y)
    return 0.5 * (P + P.T)


# Adaptive depth (Section 5, "Limitations and future work": the depth
# adjusted online from spectral estimates). Our reading: the change of the
# iterate in a stage, ||X_{t+1} - X_t||_F / ||X_t||_F, measures how far the
# spectrum still is from the fixed points +-1 of a sign iteration; stages of a
# sign iteration without rescale stop as soon as it is at most `adaptive_tol`.
# Those stages are every Newton-Schulz step, and `adaptive_extra` quintic
# Newton-Schulz steps (15 x - 10 x^3 + 3 x^5) / 8 appended to the composite
# filter (the paper's single table ends with two such stages). The designed
# composite stages themselves always run: their rescale keeps the iterate off
# +-1 until the last one.
NS_QUINTIC = (15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0)


def relative_change(Y_new: np.ndarray, Y: np.ndarray) -> float:
    ny = float(np.linalg.norm(Y))
    return float(np.linalg.norm(Y_new - Y)) / ny if ny > 0.0 else 0.0


def project_poly(X, mode: str = "fp16", lam: float | None = None,
                 steps: int = LANCZOS_STEPS, force_fallback: bool = False,
                 adaptive_tol: float = 0.0, adaptive_extra: int = 0):
    """Algorithm 2 in FP64. ``lam`` overrides the spectral bound (so that the
    oracle evaluates exactly the function the device evaluated).
    ``adaptive_tol`` > 0 stops the adaptive stages (see above) at the first
    relative change <= the tolerance; ``info["stages"]`` counts the stages run.

    Returns (P, info) with P FP64 n x n symmetric."""
    Xs = sym_from_upper(X)
    n = Xs.shape[0]
    if n == 0:
        return Xs.copy(), {"lam": 0.0}
    if not np.all(np.isfinite(Xs)):
        raise ValueError("non-finite input")
    if lam is None:
        info = spectral_bound(Xs, steps, force_fallback)
        lam = info["lam"]
    else:
        info = {"lam": float(lam), "fro": float(np.sqrt(np.sum(Xs * Xs)))}
    if lam == 0.0:
        return np.zeros_like(Xs), info
    X0 = Xs / lam
    Y = X0
    stages = 0
    if mode in NS_ITERS:
        for _ in range(NS_ITERS[mode]):
            Y_new = newton_schulz_stage(Y)
            d = relative_change(Y_new, Y)
            Y = Y_new
            stages += 1
            if adaptive_tol > 0.0 and d <= adaptive_tol:
                break
    else:
        for a, b, c in stage_rows(mode):
            Y = filter_stage(Y, a, b, c)
            stages += 1
        for _ in range(int(adaptive_extra)):
            Y_new = filter_stage(Y, *NS_QUINTIC)
            d = relative_change(Y_new, Y)
            Y = Y_new
            stages += 1
            if adaptive_tol > 0.0 and d <= adaptive_tol:
                break
    info["stages"] = stages
    return final_combine(X0, Y, lam), info


# ---------------------------------------------------------------------------
# Deflation of dominant eigenpairs before filtering (Section 4.1 "Results",
# Section 5 "Limitations and future work")
# ---------------------------------------------------------------------------
DEFLATE_RTOL = 1e-8


def deflation_pairs(Xs: np.ndarray, kmax: int, steps: int = LANCZOS_STEPS, rtol: float = DEFLATE_RTOL):
    """Dominant eigenpairs of X for deflation, from the Krylov basis V of the
    bound's Lanczos run on X^2: the Rayleigh-Ritz pairs of X itself in that
    basis, (mu_i, z_i = V s_i) with V^T X V s_i = mu_i s_i, resolve the sign
    that X^2 loses. Of the kmax pairs of largest |mu|, those whose residual
    ||X z_i - mu_i z_i|| is at most rtol |mu_i| (converged, so that removing
    them is exact to that level) are returned, largest |mu| first.

    Returns (mu, Z, resid) with Z n x d (unit columns), d <= kmax."""
    V, _ = lanczos_run(Xs, steps)
    XV = Xs @ V
    H = V.T @ XV
    H = 0.5 * (H + H.T)
    mu, S = np.linalg.eigh(H)
    order = np.argsort(-np.abs(mu), kind="stable")[: max(0, int(kmax))]
    keep_mu, keep_z, keep_r = [], [], []
    for i in order:
        z = V @ S[:, i]
        nz = np.linalg.norm(z)
        z = z / nz
        r = float(np.linalg.norm(Xs @ z - mu[i] * z))
        if r <= rtol * abs(mu[i]):
            keep_mu.append(float(mu[i]))
            keep_z.append(z)
            keep_r.append(r)
    Z = np.array(keep_z).T if keep_z else np.zeros((Xs.shape[0], 0))
    return np.array(keep_mu), Z, np.array(keep_r)


def project_deflated(X, mode: str = "fp16", kmax: int = 1, lam: float | None = None,
                     steps: int = LANCZOS_STEPS):
    """Projection with deflation: remove the converged dominant pairs,
    X' = X - sum_i mu_i z_i z_i^T, project X' with Algorithm 2 (its own
    spectral bound, or ``lam``), and add back the PSD part of what was
    removed: P = P(X') + sum_i max(mu_i, 0) z_i z_i^T. For exact eigenpairs
    this is Pi(X) up to the filter's error on X' (the z_i are eigenvectors
    of X' with eigenvalue 0, and Pi acts on each eigenspace separately).

    Returns (P, info) with info of the inner projection plus mu, Z."""
    Xs = sym_from_upper(X)
    if Xs.shape[0] == 0:
        return Xs.copy(), {"lam": 0.0, "mu": np.zeros(0), "Z": np.zeros((0, 0))}
    if not np.all(np.isfinite(Xs)):
        raise ValueError("non-finite input")
    mu, Z, r = deflation_pairs(Xs, kmax, steps)
    Xd = Xs - (Z * mu) @ Z.T
    P, info = project_poly(Xd, mode, lam=lam, steps=steps)
    P = P + (Z * np.maximum(mu, 0.0)) @ Z.T
    info = dict(info, mu=mu, Z=Z, resid=r)
    return 0.5 * (P + P.T), info


def gemm_count(mode: str) -> int:
    """3 products per odd quintic stage (2 per cubic Newton-Schulz step)
    plus the final X0 X_T."""
    per = 2 if mode in NS_ITERS else 3
    return per * stage_rows(mode).shape[0] + 1


# ---------------------------------------------------------------------------
# Exact projection (eq. (1) via the closed form eq. (3))
# ---------------------------------------------------------------------------
def project_exact(X, return_eigs: bool = False):
    """Q diag(max(lambda, 0)) Q^T with a cyclic Jacobi eigensolver (plain C)."""
    Xs = np.ascontiguousarray(sym_from_upper(X))
    n = Xs.shape[0]
    out = np.zeros_like(Xs)
    w = np.zeros(max(n, 1))
    if n:
        sweeps = _lib().oracle_project_jacobi(n, _dp(Xs), _dp(out), _dp(w))
        if sweeps < 0:
            raise RuntimeError("Jacobi did not converge")
    return (out, w[:n]) if return_eigs else out


def jacobi_eig(X):
    """Eigenvalues and eigenvectors (columns) of a symmetric FP64 matrix."""
    A = np.ascontiguousarray(sym_from_upper(X)).copy()
    n = A.shape[0]
    V = np.zeros_like(A)
    w = np.zeros(max(n, 1))
    sweeps = _lib().oracle_jacobi_eig(n, _dp(A), _dp(V), _dp(w), 60, 1e-15)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return w[:n], V


def project_exact_eigh(X):
    """Same closed form with LAPACK's eigh (a library cross-check, any n)."""
    Xs = sym_from_upper(X)
    w, Q = np.linalg.eigh(Xs)
    return (Q * np.maximum(w, 0.0)) @ Q.T


def project_spectral(Q: np.ndarray, lam_vals: np.ndarray, fn) -> np.ndarray:
    """Q diag(fn(lambda)) Q^T for a matrix built from a known spectrum — the
    spectral-operator identity (eq. (4)/(5)) used as an exact reference."""
    return (Q * fn(np.asarray(lam_vals, dtype=np.float64))) @ Q.T


# ---------------------------------------------------------------------------
# e_float (eq. (12))
# ---------------------------------------------------------------------------
def efloat(table: str, with_rescale: bool = False):
    """Returns (twice_err, argmax): max over float32 x in [0, 1] of
    |x p(x) - x|. The literal ReLU error of eq. (12) is half of it."""
    rows = tables.runtime_table(table) if with_rescale else tables.TABLES[table]
    return efloat_rows(rows)


def efloat_rows(rows):
    """``efloat`` for any T x 3 table of odd quintic stages (a, b, c)."""
    rows = np.asarray(rows, dtype=np.float64)
    abc = np.ascontiguousarray(rows, dtype=np.float64).reshape(-1)
    arg = ctypes.c_double(0.0)
    e = _lib().oracle_efloat(rows.shape[0], _dp(abc), ctypes.byref(arg))
    return float(e), float(arg.value)
