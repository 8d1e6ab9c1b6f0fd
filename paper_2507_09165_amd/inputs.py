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
* ``householder_spectrum`` eigenvalues uniform in [-1, 1] and a unit vector u:
                         X = H diag(d) H with H = I - 2 u u^T, dense, with a
                         known spectrum at any order (the matrix itself is
                         formed by the caller, e.g. on the device).
* ``batch_sizes``        256 block sizes, log-uniform in [32, 1024].
* ``maxcut_graph``       random graphs for the Max-Cut SDPs of the ADMM client.
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


def householder_spectrum(n: int, seed: int, lo: float = -1.0, hi: float = 1.0):
    """(d, u), FP64: eigenvalues d uniform in [lo, hi] and a unit vector u;
    X = H diag(d) H with the reflector H = I - 2 u u^T has the eigenvalues d
    and eigenvectors the columns of H."""
    rng = _rng(seed)
    d = rng.uniform(lo, hi, size=n)
    u = rng.standard_normal(n)
    return d, u / np.linalg.norm(u)


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


def maxcut_graph(n: int, seed: int, avg_degree: float = 5.0):
    """Edges (i, j), i < j, of an Erdos-Renyi graph with the given mean degree
    and unit weights: the shape of the Max-Cut SDP instances of Section 4.2
    (G55: n = 5000, 12498 edges). Returns an (m, 2) int array."""
    rng = _rng(seed)
    m = int(round(avg_degree * n / 2))
    seen = set()
    edges = []
    while len(edges) < m:
        i, j = (int(v) for v in rng.integers(0, n, size=2))
        if i == j:
            continue
        a, b = (i, j) if i < j else (j, i)
        if (a, b) in seen:
            continue
        seen.add((a, b))
        edges.append((a, b))
    return np.array(edges, dtype=np.int64)


def laplacian(n: int, edges) -> np.ndarray:
    """Graph Laplacian L = D - W (unit weights), FP64."""
    L = np.zeros((n, n))
    for a, b in edges:
        L[a, b] -= 1.0
        L[b, a] -= 1.0
        L[a, a] += 1.0
        L[b, b] += 1.0
    return L
