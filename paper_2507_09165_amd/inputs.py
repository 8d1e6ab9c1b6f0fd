"""Seeded synthetic inputs for the PSD-projection workloads.

This module only draws random matrices; it holds none of the projection
method's arithmetic. Both the tests' oracle side and the device side consume
the same FP32 bytes produced here.

The paper benchmarks on public dense matrix collections and SDP instances that
are not available here; these generators stand in for them with the sizes and
spectral structure of the workloads (dense, symmetric, eigenvalues of both
signs):

* ``constructed``        X = Q diag(lam) Q^T, Q from the QR of a Gaussian matrix.
* ``goe``                X = (G + G^T) / sqrt(2 n), G Gaussian (semicircle on [-2, 2]).
* ``clustered``          20% of the eigenvalues in [-1e-3, 1e-3], 80% in [-1, 1].
* ``dominant``           a few dominant eigenvalues over a dense [-1, 1] spectrum.
* ``lowrank_noise``      W W^T / n + sqrt(1e-2) (H + H^T) / sqrt(2 n), rank 500.
* ``batch_sizes``        256 block sizes, log-uniform in [32, 1024].
* ``serving_trace``      Poisson arrivals, log-uniform sizes, ADMM-like drift.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def haar_orthogonal(n: int, seed: int) -> np.ndarray:
    G = _rng(seed).standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    # sign fix so the distribution is Haar and the result deterministic
    Q = Q * np.sign(np.diag(R))[None, :]
    return Q


def constructed(n: int, seed_q: int, seed_lam: int, lo: float = -1.0, hi: float = 1.0):
    """Returns (X32, Q, lam): X = Q diag(lam) Q^T formed in FP64, stored FP32."""
    Q = haar_orthogonal(n, seed_q)
    lam = _rng(seed_lam).uniform(lo, hi, size=n)
    X = (Q * lam) @ Q.T
    X = 0.5 * (X + X.T)
    return X.astype(np.float32), Q, lam


def from_spectrum(Q: np.ndarray, lam: np.ndarray) -> np.ndarray:
    X = (Q * lam) @ Q.T
    return (0.5 * (X + X.T)).astype(np.float32)


def dominant(n: int, seed: int, top=(1000.0,)):
    """A few dominant eigenvalues over a dense spectrum (the shape of the
    paper's hard case: one extremal eigenvalue and many small ones): X = Q
    diag(lam) Q^T with lam_i = top[i] for the first len(top) and uniform in
    [-1, 1] otherwise. Returns (X64, Q, lam); X64 is FP64 and symmetric."""
    Q = haar_orthogonal(n, seed)
    lam = _rng(seed + 1).uniform(-1.0, 1.0, n)
    lam[: len(top)] = top
    X = (Q * lam) @ Q.T
    return 0.5 * (X + X.T), Q, lam


def goe(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    G = _rng(seed).standard_normal((n, n), dtype=np.float64)
    X = (G + G.T) * (1.0 / np.sqrt(2.0 * n))
    return X.astype(dtype)


def clustered(n: int, seed: int):
    """20% of eigenvalues uniform in [-1e-3, 1e-3], the rest uniform in [-1, 1]."""
    rng = _rng(seed + 1000)
    m = int(round(0.2 * n))
    lam = np.concatenate([rng.uniform(-1e-3, 1e-3, size=m), rng.uniform(-1.0, 1.0, size=n - m)])
    rng.shuffle(lam)
    Q = haar_orthogonal(n, seed)
    return from_spectrum(Q, lam), Q, lam


def lowrank_noise(n: int, seed_w: int, seed_h: int, rank: int = 500, noise_var: float = 1e-2):
    W = _rng(seed_w).standard_normal((n, rank))
    H = _rng(seed_h).standard_normal((n, n))
    X = (W @ W.T) / n + np.sqrt(noise_var) * (H + H.T) / np.sqrt(2.0 * n)
    return X.astype(np.float32)


def batch_sizes(count: int = 256, seed: int = 7, lo: int = 32, hi: int = 1024) -> np.ndarray:
    u = _rng(seed).uniform(np.log(lo), np.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), lo, hi)


def batch_blocks(sizes, seed: int = 7):
    """One GOE block per size, block i seeded with seed * 100003 + i."""
    return [goe(int(n), seed * 100003 + i) for i, n in enumerate(sizes)]


def serving_trace(num: int, rate_per_s: float, seed: int = 11, lo: int = 64, hi: int = 8192,
                  p_fp16: float = 0.7, clients: int = 8):
    """Poisson arrival times, log-uniform sizes per client stream, accuracy target
    1e-3 (probability p_fp16) or 1e-5. Returns a list of dicts."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=num)
    t = np.cumsum(gaps)
    client_n = np.clip(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=clients))), lo, hi).astype(int)
    reqs = []
    for i in range(num):
        c = int(rng.integers(clients))
        reqs.append({"t": float(t[i]), "client": c, "n": int(client_n[c]),
                     "target": 1e-3 if rng.uniform() < p_fp16 else 1e-5})
    return reqs


def admm_like_iterate(Y_prev: np.ndarray, seed: int, var: float = 1e-3) -> np.ndarray:
    """Y_k = Y_{k-1} + symmetric Gaussian perturbation with entry variance var/n."""
    n = Y_prev.shape[0]
    return (Y_prev.astype(np.float64) + np.sqrt(var) * goe(n, seed, np.float64)).astype(np.float32)
