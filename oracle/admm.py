"""FP64 three-step ADMM for SDP with a pluggable PSD-cone projection.

ORACLE — test infrastructure only (the same rules as ``oracle.psd``): plain
FP64 numpy, no code shared with the library.

The problem is the primal-dual pair of Section 4.2,

    min <C, X>  s.t.  A X = b, X PSD        max b^T y  s.t.  A^T y + S = C, S PSD,

solved by the three-step ADMM scheme of Section 4.2 (the ADMM equation
there), with penalty sigma:

    y_{k+1} = (A A^T)^{-1} (b / sigma - A(X_k / sigma + S_k - C))
    S_{k+1} = Pi(C - A^T y_{k+1} - X_k / sigma)
    X_{k+1} = X_k + sigma (S_{k+1} + A^T y_{k+1} - C).

``maxcut_ops`` gives the maps of the Max-Cut SDP family (A X = diag(X),
A^T y = Diag(y), A A^T = I). ``surrogate`` is the three-term residual the paper
monitors while no eigenvalues are computed; ``kkt`` adds the two eigenvalue
terms of its full residual eta. The switch rule (low-precision projections
until the surrogate first drops below 1e-2, then the exact projection) is
``solve``'s ``switch_at``.
"""
from __future__ import annotations

import numpy as np

from .psd import project_exact_eigh, project_poly


def maxcut_ops(n: int):
    """A X = diag(X), A^T y = Diag(y), (A A^T)^{-1} = I."""
    A = lambda X: np.diag(X).copy()  # noqa: E731
    AT = lambda y: np.diag(y)  # noqa: E731
    AAT_solve = lambda v: v  # noqa: E731
    return A, AT, AAT_solve


def surrogate(C, b, X, y, S, A, AT):
    """The three residual terms monitored before the precision switch."""
    r_p = np.linalg.norm(A(X) - b) / (1.0 + np.linalg.norm(b))
    r_d = np.linalg.norm(AT(y) + S - C) / (1.0 + np.linalg.norm(C))
    pobj, dobj = float(np.sum(C * X)), float(b @ y)
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return max(r_p, r_d, gap), (r_p, r_d, gap, pobj, dobj)


def kkt(C, b, X, y, S, A, AT):
    """The full residual eta: the surrogate and the negative parts of the
    smallest eigenvalues of X and S (an eigensolver here)."""
    s, parts = surrogate(C, b, X, y, S, A, AT)
    ex = min(0.0, float(np.linalg.eigvalsh(0.5 * (X + X.T))[0])) / (1.0 + np.linalg.norm(b))
    es = min(0.0, float(np.linalg.eigvalsh(0.5 * (S + S.T))[0])) / (1.0 + np.linalg.norm(C))
    return max(s, abs(ex), abs(es))


def step(C, b, X, S, sigma, A, AT, AAT_solve, project):
    """One ADMM iteration; returns (X, y, S)."""
    y = AAT_solve(b / sigma - A(X / sigma + S - C))
    W = C - AT(y) - X / sigma
    S = project(0.5 * (W + W.T))
    X = X + sigma * (S + AT(y) - C)
    return X, y, S


def solve(C, b, sigma: float, iters: int, project_low=None, switch_at: float = 1e-2,
          A=None, AT=None, AAT_solve=None, X0=None, S0=None):
    """ADMM from X0 = S0 = 0 (or the given ones). ``project_low`` (a function of
    a symmetric matrix) is used until the surrogate first drops below
    ``switch_at``, the exact FP64 projection afterwards (and throughout when it
    is None). Returns dict(X, y, S, history, switched_at)."""
    n = C.shape[0]
    if A is None:
        A, AT, AAT_solve = maxcut_ops(n)
    X = np.zeros((n, n)) if X0 is None else np.array(X0, dtype=np.float64)
    S = np.zeros((n, n)) if S0 is None else np.array(S0, dtype=np.float64)
    y = np.zeros(len(b))
    hist = []
    low = project_low is not None
    switched = None
    for k in range(iters):
        proj = project_low if low else project_exact_eigh
        X, y, S = step(C, b, X, S, sigma, A, AT, AAT_solve, proj)
        sur, parts = surrogate(C, b, X, y, S, A, AT)
        hist.append((sur,) + parts)
        if low and sur < switch_at:
            low = False
            switched = k
    return {"X": X, "y": y, "S": S, "history": np.array(hist), "switched_at": switched}


def poly_projection(mode: str):
    """Algorithm 2 in FP64 (the oracle's composite filter) as a projection."""
    return lambda W: project_poly(W, mode)[0]
