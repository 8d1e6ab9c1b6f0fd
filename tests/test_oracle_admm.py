"""Pins of the FP64 ADMM oracle (Section 4.2, the three-step ADMM scheme) on
Max-Cut SDPs, against what the mathematics fixes:
* the complete graph K_n, whose SDP value is n^2 / 4 (X = n/(n-1) (I - J/n)
  attains it; <L, X> <= n^2 because L = n I - J and 1^T X 1 >= 0);
* small random graphs, where the SDP value bounds the brute-force maximum cut
  from above and the Goemans-Williamson ratio 0.878 bounds it from below;
* the iteration's own invariants: every X_k and S_k is PSD (X_{k+1} =
  sigma Pi(-W) by the Moreau decomposition W = Pi(W) - Pi(-W)), and at convergence the duality
  gap and <X, S> vanish;
* the paper's observation that low-precision projections before the switch do
  not slow convergence (here: the composite filter's FP64 form)."""
import numpy as np
import pytest

from oracle import admm
from paper_2507_09165_amd import inputs


def _kn(n):
    L = n * np.eye(n) - np.ones((n, n))
    return -L / 4.0, np.ones(n)


@pytest.mark.parametrize("n", [6, 10])
def test_complete_graph_closed_form(n):
    C, b = _kn(n)
    r = admm.solve(C, b, sigma=1.0, iters=400)
    assert abs(-np.sum(C * r["X"]) - n * n / 4.0) < 1e-9
    A, AT, _ = admm.maxcut_ops(n)
    assert admm.kkt(C, b, r["X"], r["y"], r["S"], A, AT) < 1e-10


def test_random_graph_between_maxcut_and_gw_bound():
    n = 12
    L = inputs.laplacian(n, inputs.maxcut_graph(n, 3, avg_degree=4))
    C, b = -L / 4.0, np.ones(n)
    r = admm.solve(C, b, sigma=1.0, iters=2000)
    sdp = -np.sum(C * r["X"])
    best = 0.0
    for bits in range(1 << (n - 1)):
        x = np.where((bits >> np.arange(n)) & 1, 1.0, -1.0)
        best = max(best, x @ L @ x / 4.0)
    assert best <= sdp + 1e-8 and best >= 0.878 * sdp
    np.testing.assert_allclose(np.diag(r["X"]), 1.0, atol=1e-9)
    assert abs(np.sum(r["X"] * r["S"])) < 1e-8


def test_iterates_stay_psd_and_x_is_moreau_part():
    n = 20
    L = inputs.laplacian(n, inputs.maxcut_graph(n, 5))
    C, b = -L / 4.0, np.ones(n)
    A, AT, AAT = admm.maxcut_ops(n)
    X = np.zeros((n, n))
    S = np.zeros((n, n))
    sigma = 0.7
    for _ in range(15):
        y = AAT(b / sigma - A(X / sigma + S - C))
        W = C - AT(y) - X / sigma
        Xn, yn, Sn = admm.step(C, b, X, S, sigma, A, AT, AAT, admm.project_exact_eigh)
        np.testing.assert_allclose(Xn, sigma * admm.project_exact_eigh(-W), atol=1e-12)
        assert np.linalg.eigvalsh(Xn).min() > -1e-12 and np.linalg.eigvalsh(Sn).min() > -1e-12
        X, S = Xn, Sn


def test_low_precision_warm_start_does_not_slow_convergence():
    n = 60
    L = inputs.laplacian(n, inputs.maxcut_graph(n, 7))
    C, b = -L / 4.0, np.ones(n)
    exact = admm.solve(C, b, sigma=1.0, iters=300)
    warm = admm.solve(C, b, sigma=1.0, iters=300, project_low=admm.poly_projection("fp16"))
    assert warm["switched_at"] is not None
    e_exact, e_warm = exact["history"][-1][0], warm["history"][-1][0]
    assert e_warm < 10.0 * max(e_exact, 1e-12) or e_warm < 1e-6
    assert abs(warm["history"][-1][4] - exact["history"][-1][4]) < 1e-4 * abs(exact["history"][-1][4])
