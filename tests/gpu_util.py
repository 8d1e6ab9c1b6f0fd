"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch.device("cuda:0")


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def to_dev(A, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(A))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel_fro(A, B):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / (nb if nb > 0 else 1.0))


# e4m3 (OCP FP8: 1 sign, 4 exponent bits with bias 7, 3 mantissa bits, no
# infinities, S.1111.111 = NaN) as a plain codec for building and reading the
# FP8 pair buffers of the split FP8 mode.
def e4m3_values():
    b = np.arange(256)
    s, e, m = b >> 7, (b >> 3) & 15, b & 7
    v = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (e - 7.0))
    v = np.where(s == 1, -v, v)
    v[(e == 15) & (m == 7)] = np.nan
    return v


def e4m3_encode(x):
    """Round to nearest even code after clamping to [-448, 448]."""
    x = np.asarray(x, dtype=np.float64)
    pos = e4m3_values()[:127]                     # codes 0x00..0x7E, increasing
    a = np.minimum(np.abs(x), 448.0)
    hi = np.clip(np.searchsorted(pos, a), 1, 126)  # pos[hi-1] < a <= pos[hi]
    lo = hi - 1
    dl, dh = a - pos[lo], pos[hi] - a
    code = np.where(dl < dh, lo, np.where(dh < dl, hi, np.where(lo % 2 == 0, lo, hi)))
    code = np.where(a == 0, 0, code)
    return (code | np.where(np.signbit(x), 128, 0)).astype(np.uint8)


def pair8_index(n, ld=None):
    """Byte offset of the code of element (row i, column j), as an (n, n)
    array indexed [j, i]: columns grouped by 4, rows by 32, a block of 32 rows
    x 4 columns in one 128-byte line, rows permuted within a column's 32
    bytes as 16 ((i // 8) % 2) + 8 ((i // 16) % 2) + i % 8."""
    ld = n if ld is None else ld
    i = np.arange(n)[None, :]
    j = np.arange(n)[:, None]
    return ((j >> 2) * 4 * ld + 128 * (i >> 5) + 32 * (j & 3) + 16 * ((i >> 3) & 1) + 8 * ((i >> 4) & 1)
            + (i & 7))


def pair8_pack(lo_codes):
    """(n, n) code matrix indexed [j, i] -> (n, n) uint8 code buffer."""
    n = lo_codes.shape[0]
    B = np.zeros(n * n, dtype=np.uint8)
    B[pair8_index(n).ravel()] = lo_codes.ravel()
    return B.reshape(n, n)


def pair8_unpack(buf):
    n = buf.shape[0]
    return np.ascontiguousarray(buf.ravel()[pair8_index(n)])


def rocsolver_eigh64(X):
    """FP64 eigendecomposition of a symmetric device matrix with rocSOLVER's
    dsyevd (the library reference of the full-size tests; its upper triangle,
    read as column-major, is the matrix). Returns (w, Q) on the device with
    the eigenvectors in the rows of Q, so that X = Q^T diag(w) Q."""
    import ctypes
    import torch
    blas = ctypes.CDLL("librocblas.so")
    sol = ctypes.CDLL("librocsolver.so")
    h = ctypes.c_void_p()
    assert blas.rocblas_create_handle(ctypes.byref(h)) == 0
    try:
        st = torch.cuda.current_stream()
        assert blas.rocblas_set_stream(h, ctypes.c_void_p(st.cuda_stream)) == 0
        n = X.shape[0]
        A = X.double().contiguous().clone()
        w = torch.empty(n, dtype=torch.float64, device=X.device)
        E = torch.empty(n, dtype=torch.float64, device=X.device)
        info = torch.zeros(1, dtype=torch.int32, device=X.device)
        # rocblas_evect_original = 211, rocblas_fill_upper = 121
        assert sol.rocsolver_dsyevd(h, 211, 121, n, ctypes.c_void_p(A.data_ptr()), n, ctypes.c_void_p(w.data_ptr()),
                                    ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(info.data_ptr())) == 0
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        return w, A
    finally:
        blas.rocblas_destroy_handle(h)
