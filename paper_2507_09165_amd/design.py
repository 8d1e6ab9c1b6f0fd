"""Offline designer of composite odd-polynomial filter coefficients.

Produces the tables the projection runs on (Tables 1 and 2 are two outputs of
it) for any stage count T, stage degree d and sign-gap epsilon:

* Stage I (Section 3.1, Algorithm 1): the minimax composite approximation of
  sign(x) on [-1, -eps] U [eps, 1], built one stage at a time. Stage t is the
  odd polynomial of degree d closest to 1 in the uniform norm on the current
  interval [a_t, b_t] (by oddness this is the minimax fit of sign on the
  symmetric pair of intervals); the next interval is the image of [a_t, b_t]
  under it. Each stage is one Remez run.
* Remez (Appendix A, Algorithm 3): alternation system on d' + 1 reference
  points (d' = (d + 1) / 2 odd basis functions x, x^3, ..., x^d), roots of the
  residual between consecutive points, one extremum of the residual per
  sub-interval as the new reference, until the reference stops moving.
  Carried out in 50-digit arithmetic (mpmath): late stages work on intervals
  [1 - delta, 1 + delta] with tiny delta, where the alternation system in the
  odd monomial basis is too ill-conditioned for FP64.
* Stage II (Section 3.2): refinement of the composite for the ReLU objective,
  max over [-1, 1] of |x (1 + p(x)) / 2 - ReLU(x)| (eq. (10)), evaluated on a
  dense sample of [0, 1] (the error is even in x because p is odd), starting
  from the Stage-I composite. The paper names gradient descent on all
  coefficients. From f* that descent is stiff: the image of x = 1 under each
  stage is the right end of the next stage's interval, where the next stage
  has a slope of about 10, so a coefficient change is amplified about tenfold
  per stage at x = 1 and any step large enough to matter blows the composite
  up there (steps of 1e-5 relative were needed). The refinement therefore
  first moves along the Stage-I family itself: the same loss as a function of
  the sign gap eps' of Algorithm 1 (a log-spaced scan and a golden-section
  step over [eps / 30, eps]); a smaller gap sharpens the transition at 0 at the
  price of sign accuracy near 1, which is exactly the trade the ReLU objective
  asks for. It then refines all T x d' coefficients locally from the best
  member, with the loss's gradients (the Jacobian of the composite with
  respect to every stage's coefficients, by the chain rule through the
  stages) in a trust-region sequence of linear programs that only accepts
  steps that lower the maximum.

CPU only (numpy, scipy, mpmath); nothing here runs on the device or is needed
at run time.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

try:
    import mpmath as _mp
except ImportError as _e:  # pragma: no cover - mpmath ships with this image
    raise ImportError("the coefficient designer needs mpmath") from _e

_DPS = 50


# ---------------------------------------------------------------------------
# Remez for an odd polynomial approximating the constant 1 on [a, b], a > 0
# ---------------------------------------------------------------------------
@dataclass
class RemezResult:
    coef: list            # c_1..c_m of x, x^3, ..., x^(2m-1) (mpf)
    E: object             # levelled error (mpf, signed as in the alternation system)
    ref: list             # final reference points (mpf)
    iters: int
    history: list = field(default_factory=list)


def _odd_eval(coef, x):
    """sum_l c_l x^(2l - 1) (Horner in x^2)."""
    x2 = x * x
    acc = 0
    for c in reversed(coef):
        acc = acc * x2 + c
    return acc * x


def _odd_deriv_roots(coef, a, b):
    """Points of (a, b) where d/dx sum c_l x^(2l-1) = sum (2l-1) c_l u^(l-1)
    vanishes (u = x^2), in increasing order."""
    m = len(coef)
    if m < 2:
        return []
    # polynomial in u of degree m-1, highest degree first for polyroots
    pc = [(2 * l - 1) * coef[l - 1] for l in range(m, 0, -1)]
    while len(pc) > 1 and pc[0] == 0:
        pc = pc[1:]
    if len(pc) < 2:
        return []
    try:
        us = _mp.polyroots(pc, maxsteps=200, extraprec=200)
    except _mp.libmp.libhyper.NoConvergence:  # pragma: no cover
        us = _mp.polyroots(pc, maxsteps=2000, extraprec=800)
    out = []
    for u in us:
        if abs(_mp.im(u)) > _mp.mpf(10) ** (-_DPS // 2) * (1 + abs(u)):
            continue
        u = _mp.re(u)
        if u <= 0:
            continue
        x = _mp.sqrt(u)
        if a < x < b:
            out.append(x)
    return sorted(out)


def remez_odd_one(a, b, m: int, tol=None, max_iter: int = 100) -> RemezResult:
    """Minimax odd polynomial sum_{l<=m} c_l x^(2l-1) for the constant 1 on
    [a, b] (Algorithm 3 with basis x, x^3, ..., x^(2m-1) and g = 1)."""
    with _mp.workdps(_DPS):
        a, b = _mp.mpf(a), _mp.mpf(b)
        tol = _mp.mpf(10) ** (-30) * (b - a) if tol is None else _mp.mpf(tol)
        # m + 1 Chebyshev (extrema) nodes on [a, b], endpoints included
        ref = [(a + b) / 2 - (b - a) / 2 * _mp.cos(_mp.pi * i / m) for i in range(m + 1)]
        hist = []
        for it in range(1, max_iter + 1):
            # (1) alternation system: sum_l c_l phi_l(x_i) - 1 = (-1)^i E
            A = _mp.matrix(m + 1, m + 1)
            rhs = _mp.matrix(m + 1, 1)
            for i, x in enumerate(ref):
                for l in range(m):
                    A[i, l] = x ** (2 * l + 1)
                A[i, m] = -((-1) ** i)
                rhs[i] = 1
            sol = _mp.lu_solve(A, rhs)
            coef = [sol[l] for l in range(m)]
            E = sol[m]
            err = lambda x: _odd_eval(coef, x) - 1  # noqa: E731
            # (2) roots of the residual between consecutive reference points
            z = [a]
            for i in range(m):
                lo, hi = ref[i], ref[i + 1]
                flo = err(lo)
                for _ in range(400):  # bisection: the residual changes sign here
                    mid = (lo + hi) / 2
                    fm = err(mid)
                    if (fm > 0) == (flo > 0):
                        lo, flo = mid, fm
                    else:
                        hi = mid
                    if hi - lo <= _mp.mpf(10) ** (-_DPS + 5) * (1 + abs(hi)):
                        break
                z.append((lo + hi) / 2)
            z.append(b)
            # (3) one extremum of the residual per sub-interval, with the sign
            # the residual has at the old reference point there
            crit = _odd_deriv_roots(coef, a, b)
            new = []
            for i in range(m + 1):
                lo, hi = z[i], z[i + 1]
                s = 1 if err(ref[i]) > 0 else -1
                cands = [lo, hi] + [x for x in crit if lo < x < hi]
                new.append(max(cands, key=lambda x: s * err(x)))
            move = max(abs(y - x) for x, y in zip(ref, new))
            hist.append((it, E, move))
            ref = new
            # (4) stop when the reference no longer moves
            if move <= tol:
                break
        # final solve on the converged reference
        A = _mp.matrix(m + 1, m + 1)
        rhs = _mp.matrix(m + 1, 1)
        for i, x in enumerate(ref):
            for l in range(m):
                A[i, l] = x ** (2 * l + 1)
            A[i, m] = -((-1) ** i)
            rhs[i] = 1
        sol = _mp.lu_solve(A, rhs)
        return RemezResult([sol[l] for l in range(m)], sol[m], ref, it, hist)


def odd_range(coef, a, b):
    """(min, max) of the odd polynomial over [a, b]: endpoints and critical
    points."""
    with _mp.workdps(_DPS):
        a, b = _mp.mpf(a), _mp.mpf(b)
        pts = [a, b] + _odd_deriv_roots(coef, a, b)
        vals = [_odd_eval(coef, x) for x in pts]
        return min(vals), max(vals)


# ---------------------------------------------------------------------------
# Stage I: Algorithm 1
# ---------------------------------------------------------------------------
@dataclass
class SignComposite:
    rows: np.ndarray        # T x m FP64 coefficients (x, x^3, ..., x^d)
    intervals: list         # [a_t, b_t] per stage (floats)
    errors: list            # levelled error |E_t| of each stage on its interval
    remez: list             # RemezResult per stage (high precision)


def sign_composite(eps: float, T: int, d: int = 5) -> SignComposite:
    """Algorithm 1: minimax composite of T odd degree-d stages for sign on
    [-1, -eps] U [eps, 1]."""
    if d % 2 != 1 or d < 1:
        raise ValueError("odd stage degree required")
    if not 0.0 < eps < 1.0:
        raise ValueError("eps in (0, 1) required")
    m = (d + 1) // 2
    with _mp.workdps(_DPS):
        a, b = _mp.mpf(eps), _mp.mpf(1)
        rows, ivs, errs, rr = [], [], [], []
        for _t in range(T):
            r = remez_odd_one(a, b, m)
            rows.append([float(c) for c in r.coef])
            ivs.append((float(a), float(b)))
            errs.append(float(abs(r.E)))
            rr.append(r)
            a, b = odd_range(r.coef, a, b)   # the next interval: image of [a, b]
        return SignComposite(np.array(rows), ivs, errs, rr)


# ---------------------------------------------------------------------------
# Composite evaluation and its Jacobian (FP64)
# ---------------------------------------------------------------------------
def composite(rows: np.ndarray, x: np.ndarray) -> np.ndarray:
    """p(x) = f_T(...f_1(x)) for stage rows of odd-power coefficients."""
    y = np.asarray(x, dtype=np.float64)
    for r in rows:
        y2 = y * y
        acc = np.zeros_like(y)
        for c in r[::-1]:
            acc = acc * y2 + c
        y = acc * y
    return y


def composite_jacobian(rows: np.ndarray, x: np.ndarray):
    """(p(x), J) with J[i, t*m + l] = d p(x_i) / d rows[t, l] (chain rule
    through the stages: dp/dc_{t,l} = prod_{s>t} f_s'(y_{s-1}) y_{t-1}^(2l+1))."""
    T, m = rows.shape
    ys = [np.asarray(x, dtype=np.float64)]
    for r in rows:
        y = ys[-1]
        y2 = y * y
        acc = np.zeros_like(y)
        for c in r[::-1]:
            acc = acc * y2 + c
        ys.append(acc * y)
    J = np.empty((ys[0].size, T * m))
    g = np.ones_like(ys[0])  # d p / d y_t, from the last stage backwards
    for t in range(T - 1, -1, -1):
        y = ys[t]
        pw = y.copy()
        y2 = y * y
        for l in range(m):
            J[:, t * m + l] = g * pw
            pw = pw * y2
        # f_t'(y) = sum_l (2l + 1) c_l y^(2l)
        d = np.zeros_like(y)
        for l in range(m - 1, -1, -1):
            d = d * y2 + (2 * l + 1) * rows[t, l]
        g = g * d
    return ys[-1], J


def relu_error(rows: np.ndarray, x: np.ndarray) -> np.ndarray:
    """|x (1 + p(x)) / 2 - ReLU(x)|; for x >= 0 this is x |p(x) - 1| / 2."""
    x = np.asarray(x, dtype=np.float64)
    p = composite(rows, x)
    return np.abs(0.5 * x * (1.0 + p) - np.maximum(x, 0.0))


def design_grid(eps: float, n_log: int = 40000, n_lin: int = 160000) -> np.ndarray:
    """Dense sample of (0, 1]: geometric near 0 (down to eps^2), uniform above."""
    g1 = np.geomspace(eps * eps, 1.0, n_log)
    g2 = np.linspace(0.0, 1.0, n_lin + 1)[1:]
    return np.unique(np.concatenate([g1, g2]))


# ---------------------------------------------------------------------------
# Stage II: local refinement for the ReLU objective
# ---------------------------------------------------------------------------
@dataclass
class Refinement:
    rows: np.ndarray
    loss: float            # max over the design grid of |x(1+p)/2 - ReLU|
    loss0: float           # the same for the starting rows
    iters: int
    history: list


def refine_relu(rows0: np.ndarray, grid: np.ndarray | None = None, eps: float = 1e-3,
                iters: int = 200, radius: float = 1e-2, tol: float = 1e-12,
                refine_points: int = 2000) -> Refinement:
    """Minimise the maximum of e(x) = x |p(x) - 1| / 2 over the grid by a
    trust-region sequence of linear programs in all coefficients. Each step
    linearises p around the current rows on the points where e is within a
    factor of the current maximum (plus a fixed subsample), solves
        min s  s.t.  -s <= x_i (p_i + J_i dv - 1) / 2 <= s,  |dv_k| <= r |v_k|,
    and accepts the step if the true maximum over the whole grid decreased
    (the radius shrinks otherwise and grows after a success)."""
    from scipy.optimize import linprog

    rows = np.array(rows0, dtype=np.float64)
    T, m = rows.shape
    x = design_grid(eps) if grid is None else np.asarray(grid, dtype=np.float64)
    x = x[x > 0]

    def full_max(r):
        p = composite(r, x)
        return float(np.max(0.5 * x * np.abs(p - 1.0)))

    cur = full_max(rows)
    loss0 = cur
    hist = [cur]
    base_idx = np.unique(np.linspace(0, x.size - 1, refine_points).astype(int))
    r = radius
    k = 0
    for k in range(1, iters + 1):
        p = composite(rows, x)
        e = 0.5 * x * np.abs(p - 1.0)
        act = np.nonzero(e >= 0.5 * cur)[0]
        # local maxima of e, so every extremal point is represented
        lm = np.nonzero((e[1:-1] >= e[:-2]) & (e[1:-1] >= e[2:]))[0] + 1
        lm = lm[e[lm] >= 0.05 * cur]
        idx = np.unique(np.concatenate([act, lm, base_idx]))
        xs = x[idx]
        pv, J = composite_jacobian(rows, xs)
        v = rows.reshape(-1)
        nv = v.size
        h = 0.5 * xs
        # variables: dv (nv), s; minimise s
        c = np.zeros(nv + 1)
        c[-1] = 1.0
        A1 = np.hstack([h[:, None] * J, -np.ones((xs.size, 1))])        # h (p + J dv - 1) <= s
        b1 = -h * (pv - 1.0)
        A2 = np.hstack([-h[:, None] * J, -np.ones((xs.size, 1))])       # -h (p + J dv - 1) <= s
        b2 = h * (pv - 1.0)
        A = np.vstack([A1, A2])
        bb = np.concatenate([b1, b2])
        lim = r * np.maximum(np.abs(v), 1e-3)
        bounds = [(-l, l) for l in lim] + [(0, None)]
        res = linprog(c, A_ub=A, b_ub=bb, bounds=bounds, method="highs")
        if res.status != 0:
            r *= 0.5
            if r < 1e-10:
                break
            continue
        trial = (v + res.x[:nv]).reshape(T, m)
        new = full_max(trial)
        if new < cur:
            rel = (cur - new) / cur
            rows, cur = trial, new
            hist.append(cur)
            r = min(2.0 * r, radius)
            if rel < tol:
                break
        else:
            r *= 0.5
            if r < 1e-10:
                break
    return Refinement(rows, cur, loss0, k, hist)


@dataclass
class EpsSearch:
    eps: float             # best sign gap found
    rows: np.ndarray       # its Stage-I composite
    loss: float            # its ReLU loss on the design grid
    scanned: list          # (eps', loss) pairs evaluated


def relu_loss(rows: np.ndarray, grid: np.ndarray) -> float:
    with np.errstate(all="ignore"):
        e = relu_error(rows, grid)
    m = float(np.max(e))
    return m if np.isfinite(m) else float("inf")


def search_eps(eps: float, T: int, d: int = 5, lo_ratio: float = 30.0, points: int = 16,
               golden_steps: int = 8, grid: np.ndarray | None = None) -> EpsSearch:
    """Minimise the ReLU loss over the Stage-I composites of gap eps' in
    [eps / lo_ratio, eps]: a log-spaced scan, then golden-section steps in
    log eps' around the best scanned point."""
    x = design_grid(eps / lo_ratio) if grid is None else grid
    cache = {}

    def loss_of(e):
        if e not in cache:
            rows = sign_composite(e, T, d).rows
            cache[e] = (relu_loss(rows, x), rows)
        return cache[e][0]

    les = np.linspace(np.log(eps / lo_ratio), np.log(eps), points)
    vals = [loss_of(float(np.exp(v))) for v in les]
    k = int(np.argmin(vals))
    a = les[max(k - 1, 0)]
    b = les[min(k + 1, points - 1)]
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c1, c2 = b - g * (b - a), a + g * (b - a)
    f1, f2 = loss_of(float(np.exp(c1))), loss_of(float(np.exp(c2)))
    for _ in range(golden_steps):
        if f1 <= f2:
            b, c2, f2 = c2, c1, f1
            c1 = b - g * (b - a)
            f1 = loss_of(float(np.exp(c1)))
        else:
            a, c1, f1 = c1, c2, f2
            c2 = a + g * (b - a)
            f2 = loss_of(float(np.exp(c2)))
    best = min(cache, key=lambda e: cache[e][0])
    return EpsSearch(best, cache[best][1], cache[best][0], sorted((e, v[0]) for e, v in cache.items()))


def refine_stage2(f_star: np.ndarray, eps: float, T: int, d: int = 5, local_iters: int = 60,
                  scan_points: int = 16) -> dict:
    """Stage II from the Stage-I composite f_star (gap eps): the Stage-I family
    search, then the local coefficient refinement; keeps whichever of f_star
    and the result has the lower loss on the common design grid."""
    grid = design_grid(eps / 30.0)
    base = relu_loss(f_star, grid)
    es = search_eps(eps, T, d, points=scan_points, grid=grid)
    start = es.rows if es.loss < base else np.array(f_star, dtype=np.float64)
    loc = refine_relu(start, grid=grid, iters=local_iters)
    rows = loc.rows if loc.loss <= min(base, es.loss) else start
    return {"rows": rows, "loss_f_star": base, "eps_search": es, "local": loc,
            "loss": relu_loss(rows, grid)}


def design_tables(eps: float, T: int, d: int = 5, local_iters: int = 60, scan_points: int = 16):
    """Stage I then Stage II: returns (f_star rows, f_tilde rows, details)."""
    sc = sign_composite(eps, T, d)
    st2 = refine_stage2(sc.rows, eps, T, d, local_iters=local_iters, scan_points=scan_points)
    return sc.rows, st2["rows"], {"stage1": sc, "stage2": st2}


if __name__ == "__main__":  # pragma: no cover
    import sys
    eps = float(sys.argv[1]) if len(sys.argv) > 1 else 1e-3
    T = int(sys.argv[2]) if len(sys.argv) > 2 else 7
    fs, ft, info = design_tables(eps, T)
    np.set_printoptions(precision=10, suppress=True, linewidth=120)
    print("f* (Stage I):\n", fs)
    print("levelled errors:", info["stage1"].errors)
    print("f~ (Stage II):\n", ft)
    st2 = info["stage2"]
    print("ReLU loss on the design grid: f* %.4e, best eps' %.3e %.4e, refined %.4e"
          % (st2["loss_f_star"], st2["eps_search"].eps, st2["eps_search"].loss, st2["loss"]))
