"""Three-step ADMM for SDPs with a diagonal constraint map (Section 4.2),
driving the library: the dual and primal steps are psdproj_admm_dual /
psdproj_admm_primal, the PSD-cone projection psdproj_project_ex. This module
only marshals arguments and runs the loop (one 48-byte residual read-back per
iteration for the stopping test and the precision switch).

Problem: min <C, X> s.t. diag(X) = b, X PSD (Max-Cut: C = -L/4, b = 1).
Precision schedule (Section 4.2): projections in a low-precision mode until
the surrogate residual (three terms, no eigenvalues) first drops below
`switch_at`, then in a high-precision mode (the library's FP32 form by
default; the paper switches to an FP64 eigendecomposition, which a caller can
pass as `high_projection`).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import psdproj as P

RES_DOUBLES = 8 + 4 * 512  # PSDPROJ_ADMM_RES_DOUBLES


def dual_step(X, S, C, b, sigma, y, W, stream=None):
    n, ld = P._check_matrix(X)
    P._check(P.lib().psdproj_admm_dual(n, ld, P._ptr(X), P._ptr(S), P._ptr(C), P._ptr(b), float(sigma),
                                       P._ptr(y), P._ptr(W), P._stream(stream)), "psdproj_admm_dual")


def primal_step(X, S, C, y, b, sigma, res, stream=None):
    n, ld = P._check_matrix(X)
    P._check(P.lib().psdproj_admm_primal(n, ld, P._ptr(X), P._ptr(S), P._ptr(C), P._ptr(y), P._ptr(b),
                                         float(sigma), P._ptr(res), P._stream(stream)), "psdproj_admm_primal")


def surrogate(r):
    """The paper's three-term residual from psdproj_admm_primal's res."""
    rp, rd, pobj, dobj, nb, nc = (float(v) for v in r[:6])
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return max(rp / (1.0 + nb), rd / (1.0 + nc), gap), (rp / (1.0 + nb), rd / (1.0 + nc), gap, pobj, dobj)


def solve(C, b, sigma=1.0, iters=100, low_mode="fp16", high_mode="fp32", switch_at=1e-2,
          high_projection=None, low_projection=None, stream=None):
    """Run `iters` ADMM iterations from X = S = 0. C: (n, n) float32 CUDA
    tensor (symmetric), b: (n,) float64 CUDA tensor. low_mode None: no
    low-precision phase. Returns dict(X, y, S, history, switched_at)."""
    import torch
    n = C.shape[0]
    X = torch.zeros_like(C)
    S = torch.zeros_like(C)
    W = torch.empty_like(C)
    y = torch.zeros(n, dtype=torch.float64, device=C.device)
    res = torch.zeros(RES_DOUBLES, dtype=torch.float64, device=C.device)
    low = low_mode is not None or low_projection is not None
    switched = None
    hist = []

    def project(mode, fn):
        if fn is not None:
            S.copy_(fn(W))
        else:
            P.project_ex(W, S, stream=stream, info=False, mode=mode)

    for k in range(iters):
        dual_step(X, S, C, b, sigma, y, W, stream)
        if low:
            project(low_mode, low_projection)
        else:
            project(high_mode, high_projection)
        primal_step(X, S, C, y, b, sigma, res, stream)
        sur, parts = surrogate(res[:6].cpu().numpy())
        hist.append((sur,) + parts)
        if low and sur < switch_at:
            low = False
            switched = k
    return {"X": X, "y": y, "S": S, "history": np.array(hist), "switched_at": switched}
