"""The ADMM client (Section 4.2) on the GPU: its elementwise steps against FP64
numpy on the same inputs, and whole runs on a Max-Cut SDP against the FP64
ADMM oracle (exact projections): the library's FP32 projection throughout,
and the paper's schedule (half precision until the surrogate residual drops
below 1e-2, then the high-precision projection)."""
import numpy as np
import pytest

from oracle import admm as oadmm
from paper_2507_09165_amd import admm
from paper_2507_09165_amd import inputs
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _sym(n, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return ((G + G.T) / np.sqrt(2.0 * n)).astype(np.float32)


def test_admm_steps_match_fp64():
    import torch
    n, sigma = 333, 0.7
    X, S, C = _sym(n, 1), _sym(n, 2), _sym(n, 3)
    b = np.random.default_rng(4).uniform(0.5, 1.5, n)
    Xd, Sd, Cd = to_dev(X), to_dev(S), to_dev(C)
    bd = torch.from_numpy(b).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    W = torch.empty_like(Xd)
    admm.dual_step(Xd, Sd, Cd, bd, sigma, y, W)
    X64, S64, C64 = X.astype(np.float64), S.astype(np.float64), C.astype(np.float64)
    y_ref = b / sigma - np.diag(X64 / sigma + S64 - C64)
    W_ref = C64 - np.diag(y_ref) - X64 / sigma
    torch.cuda.synchronize()
    np.testing.assert_allclose(y.cpu().numpy(), y_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(W.cpu().numpy(), W_ref, rtol=0, atol=4e-7 * np.abs(W_ref).max())
    res = torch.zeros(admm.RES_DOUBLES, dtype=torch.float64, device="cuda")
    admm.primal_step(Xd, Sd, Cd, y, bd, sigma, res)
    X_ref = X64 + sigma * (S64 + np.diag(y_ref) - C64)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Xd.cpu().numpy(), X_ref, rtol=0, atol=4e-7 * np.abs(X_ref).max())
    Xn = Xd.cpu().numpy().astype(np.float64)  # the stored (rounded) iterate the sums read
    r = res[:6].cpu().numpy()
    ref = [np.linalg.norm(np.diag(Xn) - b), np.linalg.norm(np.diag(y_ref) + S64 - C64), np.sum(C64 * Xn),
           b @ y_ref, np.linalg.norm(b), np.linalg.norm(C64)]
    np.testing.assert_allclose(r, ref, rtol=1e-9)


@pytest.mark.timeout(300)
def test_maxcut_admm_against_oracle():
    import torch
    n, iters, sigma = 200, 150, 1.0
    L = inputs.laplacian(n, inputs.maxcut_graph(n, 11))
    C64, b = -L / 4.0, np.ones(n)
    say("admm oracle")
    ref = oadmm.solve(C64, b, sigma, iters)
    Cd = to_dev(C64.astype(np.float32))
    bd = torch.from_numpy(b).cuda()
    say("admm fp32")
    hi = admm.solve(Cd, bd, sigma, iters, low_mode=None, high_mode="fp32")
    say("admm fp16 -> fp32")
    warm = admm.solve(Cd, bd, sigma, iters, low_mode="fp16", high_mode="fp32")
    e_ref, e_hi, e_warm = ref["history"][-1][0], hi["history"][-1][0], warm["history"][-1][0]
    o_ref, o_hi, o_warm = ref["history"][-1][4], hi["history"][-1][4], warm["history"][-1][4]
    say(f"  surrogate after {iters}: oracle {e_ref:.3e}, fp32 {e_hi:.3e}, fp16->fp32 {e_warm:.3e} "
        f"(switch at {warm['switched_at']}); objective {o_ref:.6f} {o_hi:.6f} {o_warm:.6f}")
    assert warm["switched_at"] is not None
    assert abs(o_hi - o_ref) <= 1e-4 * abs(o_ref) and abs(o_warm - o_ref) <= 1e-4 * abs(o_ref)
    assert e_hi <= 10.0 * e_ref + 1e-5 and e_warm <= 10.0 * e_ref + 1e-5
    # the early iterates follow the oracle's trajectory closely
    np.testing.assert_allclose(hi["history"][:20, 4], ref["history"][:20, 4], rtol=1e-4)
