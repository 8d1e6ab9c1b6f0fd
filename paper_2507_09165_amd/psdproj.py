"""ctypes binding of libpsdproj (argument marshalling only).

Every step of the projection runs in the HIP library; PyTorch only provides
device memory (tensor ``data_ptr()``) and the stream
(``torch.cuda.current_stream().cuda_stream``). If the library is not built the
import fails loudly — there is no fallback path.

Layout note: a row-major torch tensor ``T`` of shape (n, n) with stride (n, 1)
is the column-major matrix ``T^T`` with leading dimension n. For symmetric
inputs the two coincide; the library reads the upper triangle of the
column-major matrix, i.e. ``torch.tril(T)`` in torch indexing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsdproj.so")

MODES = {"fp32": 0, "fp16": 1, "bf16": 2, "fp16_split": 3, "fp32_emu": 4, "fp8_fp16_split": 5,
         "ns_fp16": 6, "ns_fp32": 7, "fp8_bf16_split": 8}
DTYPES = {"fp32": 0, "fp16": 1, "bf16": 2}

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of device memory",
          4: "HIP error", 5: "rejected", 6: "cancelled", 7: "timeout", 8: "not found",
          9: "pending", 10: "non-finite input", 11: "exceeds the fixed scratch"}


class PsdprojError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} ({status})")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
                ("split_mask", ctypes.c_uint32), ("split_final", ctypes.c_int),
                ("lambda_override", ctypes.c_double), ("force_bound_fallback", ctypes.c_int),
                ("deflate", ctypes.c_int), ("adaptive_tol", ctypes.c_double), ("adaptive_extra", ctypes.c_int)]


INFO_DTYPE = np.dtype([("lambda", "<f8"), ("lanczos_lambda", "<f8"), ("sigma", "<f8"),
                       ("residual", "<f8"), ("fro_norm", "<f8"), ("colmax_norm", "<f8"),
                       ("lanczos_steps", "<i4"), ("nonfinite", "<i4"), ("fallback", "<i4"),
                       ("stages", "<i4"), ("deflated", "<i4"), ("reserved", "<i4")])
INFO_BYTES = INFO_DTYPE.itemsize
assert INFO_BYTES == 72

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python paper_2507_09165_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    i64, vp, c_int = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    L.psdproj_project.argtypes = [i64, i64, vp, vp, c_int, vp]
    L.psdproj_project_ex.argtypes = [ctypes.POINTER(Opts), i64, i64, vp, vp, vp, vp]
    L.psdproj_project_noalloc.argtypes = [ctypes.POINTER(Opts), i64, i64, vp, vp, vp, vp]
    L.psdproj_spectral_bound.argtypes = [i64, i64, vp, c_int, vp, vp]
    L.psdproj_project_batched.argtypes = [c_int, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                          ctypes.POINTER(vp), ctypes.POINTER(vp), c_int, vp]
    L.psdproj_project_batched_ex.argtypes = [ctypes.POINTER(Opts), c_int, ctypes.POINTER(i64),
                                             ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                             vp, vp]
    L.psdproj_workspace_bytes.argtypes = [i64, c_int]
    L.psdproj_workspace_bytes.restype = ctypes.c_size_t
    L.psdproj_gemm_count.argtypes = [ctypes.POINTER(Opts), c_int]
    L.psdproj_gemm_count.restype = ctypes.c_double
    L.psdproj_coefficients.argtypes = [c_int, ctypes.POINTER(ctypes.c_double), c_int]
    L.psdproj_release.argtypes = []
    L.psdproj_status_string.argtypes = [c_int]
    L.psdproj_status_string.restype = ctypes.c_char_p
    L.psdproj_tune.argtypes = [ctypes.c_char_p, i64]
    L.psdproj_tune.restype = c_int
    L.psdproj_sym_gemm.argtypes = [c_int, i64, i64, vp, vp, vp, vp, vp, vp,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp, vp]
    L.psdproj_sym_gemm_pair8.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, vp, vp, c_int, c_int, c_int, c_int, vp]
    L.psdproj_sym_gemm_pair8_bf16.argtypes = L.psdproj_sym_gemm_pair8.argtypes
    L.psdproj_autotune.argtypes = [c_int, ctypes.POINTER(i64), c_int, ctypes.c_char_p, vp]
    L.psdproj_tune_load.argtypes = [ctypes.c_char_p]
    L.psdproj_admm_dual.argtypes = [i64, i64, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp]
    L.psdproj_admm_primal.argtypes = [i64, i64, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp]
    L.psdproj_gemm_timing_start.argtypes = []
    L.psdproj_gemm_timing_stop.argtypes = [ctypes.c_void_p, c_int]
    for name in ("psdproj_gemm_timing_start", "psdproj_gemm_timing_stop",
                 "psdproj_project", "psdproj_project_ex", "psdproj_project_noalloc",
                 "psdproj_spectral_bound",
                 "psdproj_project_batched", "psdproj_project_batched_ex",
                 "psdproj_coefficients",
                 "psdproj_release", "psdproj_sym_gemm", "psdproj_sym_gemm_pair8", "psdproj_sym_gemm_pair8_bf16",
                 "psdproj_admm_dual", "psdproj_admm_primal", "psdproj_autotune", "psdproj_tune_load"):
        getattr(L, name).restype = c_int
    _lib = L
    return L


def _check(st: int, what: str):
    if st != 0:
        raise PsdprojError(st, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _mode(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _check_matrix(X, name="X"):
    import torch
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32):
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if X.dim() != 2 or X.shape[0] != X.shape[1]:
        raise ValueError(f"{name} must be square")
    if X.stride(1) != 1 or X.stride(0) < max(1, X.shape[0]):
        raise ValueError(f"{name} must have unit stride in its last dimension")
    return X.shape[0], X.stride(0)


EXPLICIT_MASK = 0x80000000
# split_mask flag: in the masked stages only B = b A + c A^2 is split
SPLIT_B_ONLY = 0x40000000
# split_mask bits SPLIT_B_SHIFT + t: stage t + 1 splits only its B product
SPLIT_B_SHIFT = 16


def make_opts(mode="fp16", lanczos_steps=0, split_mask=None, split_final=-1, lambda_override=0.0,
              force_bound_fallback=False, deflate=0, adaptive_tol=0.0, adaptive_extra=0) -> Opts:
    """split_mask None selects the mode's default split stages; an integer
    (0 included) is taken as given (the library's explicit-mask bit)."""
    mask = 0 if split_mask is None else (int(split_mask) | EXPLICIT_MASK)
    return Opts(_mode(mode), int(lanczos_steps), mask, int(split_final),
                float(lambda_override), int(bool(force_bound_fallback)), int(deflate),
                float(adaptive_tol), int(adaptive_extra))


def project(X, out=None, mode="fp16", stream=None):
    """out = Pi(X) (Algorithm 2). X: (n, n) float32 CUDA tensor; out may be X."""
    import torch
    n, ld = _check_matrix(X)
    if out is None:
        out = torch.empty_like(X)
    n2, ldo = _check_matrix(out, "out")
    if n2 != n or ldo != ld:
        raise ValueError("out must match X in shape and stride")
    _check(lib().psdproj_project(n, ld, _ptr(X), _ptr(out), _mode(mode), _stream(stream)),
           "psdproj_project")
    return out


def project_ex(X, out=None, stream=None, info=True, **opts):
    """Projection with options; returns (out, info_tensor). Call
    ``read_info(info_tensor)`` after synchronising to get a dict."""
    import torch
    n, ld = _check_matrix(X)
    if out is None:
        out = torch.empty_like(X)
    o = make_opts(**opts)
    info_t = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=X.device) if info else None
    _check(lib().psdproj_project_ex(ctypes.byref(o), n, ld, _ptr(X), _ptr(out), _stream(stream),
                                    _ptr(info_t)), "psdproj_project_ex")
    return out, info_t


def project_noalloc(X, out, info_t=None, stream=None, **opts):
    """psdproj_project_noalloc: the projection with its workspace in the
    library's fixed device array (no device allocation by the library). out
    (and info_t, INFO_BYTES bytes of device memory, if given) are the caller's."""
    n, ld = _check_matrix(X)
    if _check_matrix(out, "out") != (n, ld):
        raise ValueError("out must match X in shape and stride")
    o = make_opts(**opts)
    _check(lib().psdproj_project_noalloc(ctypes.byref(o), n, ld, _ptr(X), _ptr(out), _stream(stream),
                                         _ptr(info_t)), "psdproj_project_noalloc")
    return out


NOALLOC_SCRATCH_BYTES = 80 << 20  # PSDPROJ_NOALLOC_SCRATCH_BYTES


def read_info(info_t) -> dict:
    raw = info_t.cpu().numpy().tobytes()
    rec = np.frombuffer(raw, dtype=INFO_DTYPE)[0]
    return {k: rec[k].item() for k in INFO_DTYPE.names}


def spectral_bound(X, lanczos_steps=20, stream=None) -> dict:
    import torch
    n, ld = _check_matrix(X)
    info_t = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=X.device)
    _check(lib().psdproj_spectral_bound(n, ld, _ptr(X), int(lanczos_steps), _stream(stream),
                                        _ptr(info_t)), "psdproj_spectral_bound")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return read_info(info_t)


def _batch_args(Xs, outs):
    cnt = len(Xs)
    ns = (ctypes.c_int64 * cnt)()
    lds = (ctypes.c_int64 * cnt)()
    xp = (ctypes.c_void_p * cnt)()
    op = (ctypes.c_void_p * cnt)()
    for i, (X, O) in enumerate(zip(Xs, outs)):
        n, ld = _check_matrix(X)
        if _check_matrix(O, "out") != (n, ld):
            raise ValueError("out must match X in shape and stride")
        ns[i], lds[i], xp[i], op[i] = n, ld, X.data_ptr(), O.data_ptr()
    return cnt, ns, lds, xp, op


def project_batched(Xs, outs=None, mode="bf16", stream=None):
    import torch
    if outs is None:
        outs = [torch.empty_like(X) for X in Xs]
    cnt, ns, lds, xp, op = _batch_args(Xs, outs)
    _check(lib().psdproj_project_batched(cnt, ns, lds, xp, op, _mode(mode), _stream(stream)),
           "psdproj_project_batched")
    return outs


def project_batched_ex(Xs, outs=None, stream=None, info=True, **opts):
    """Batched projection with options; returns (outs, info_tensor) with one
    INFO_BYTES-byte info record per matrix (``read_infos``)."""
    import torch
    if outs is None:
        outs = [torch.empty_like(X) for X in Xs]
    cnt, ns, lds, xp, op = _batch_args(Xs, outs)
    o = make_opts(**opts)
    info_t = None
    if info and cnt:
        info_t = torch.zeros(INFO_BYTES * cnt, dtype=torch.uint8, device=Xs[0].device)
    _check(lib().psdproj_project_batched_ex(ctypes.byref(o), cnt, ns, lds, xp, op, _stream(stream),
                                            _ptr(info_t)), "psdproj_project_batched_ex")
    return outs, info_t


def read_infos(info_t) -> list:
    raw = info_t.cpu().numpy().tobytes()
    recs = np.frombuffer(raw, dtype=INFO_DTYPE)
    return [{k: r[k].item() for k in INFO_DTYPE.names} for r in recs]


def workspace_bytes(n: int, mode="fp16") -> int:
    return int(lib().psdproj_workspace_bytes(int(n), _mode(mode)))


def gemm_count(mode="fp16", **opts) -> float:
    o = make_opts(mode=mode, **opts)
    return float(lib().psdproj_gemm_count(ctypes.byref(o), _mode(mode)))


def coefficients(mode="fp16") -> np.ndarray:
    buf = (ctypes.c_double * 96)()
    T = lib().psdproj_coefficients(_mode(mode), buf, 96)
    if T < 0:
        raise PsdprojError(1, "psdproj_coefficients")
    return np.array(buf[: 3 * T]).reshape(T, 3)


def tune(key: str, value: int):
    _check(lib().psdproj_tune(key.encode(), int(value)), f"psdproj_tune({key})")


def autotune(mode, sizes, cache_path=None, stream=None):
    """Time the tile policies of each order's size class and keep the fastest
    (psdproj_autotune); writes cache_path when given."""
    arr = (ctypes.c_int64 * len(sizes))(*[int(n) for n in sizes])
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().psdproj_autotune(_mode(mode), arr, len(sizes), path, _stream(stream)), "psdproj_autotune")


def tune_load(path) -> int:
    """Apply a tuning cache file; returns the number of lines applied."""
    r = int(lib().psdproj_tune_load(str(path).encode()))
    if r < 0:
        raise PsdprojError(-r, "psdproj_tune_load")
    return r


def release():
    _check(lib().psdproj_release(), "psdproj_release")


def sym_gemm(dtype, L, R, D, Llo=None, Rlo=None, C0=None, C0lo=None, Dlo=None,
             alpha=0.0, beta=1.0, gamma=0.0, stream=None):
    """D = alpha C0 + beta L R + gamma I on n_p x n_p symmetric work matrices."""
    n_p = L.shape[0]
    ld = L.stride(0)
    _check(lib().psdproj_sym_gemm(DTYPES[dtype], n_p, ld, _ptr(L), _ptr(Llo), _ptr(R), _ptr(Rlo),
                                  _ptr(C0), _ptr(C0lo), float(alpha), float(beta), float(gamma),
                                  _ptr(D), _ptr(Dlo), _stream(stream)), "psdproj_sym_gemm")
    return D


def sym_gemm_pair8(L, R, D, Lx=None, Rx=None, C0=None, C0x=None, Dx=None, alpha=0.0, beta=1.0,
                   gamma=0.0, exps=(0, 0, 0, 0), stream=None):
    """D = alpha C0 + beta L R + gamma I on FP16 (or, for bfloat16 tensors,
    BF16) work matrices whose split parts are FP8 pair codes (uint8 tensors of
    n_p * ld bytes in the tiled layout documented in psdproj.h); exps are the
    pair exponents of (L, R, C0, D)."""
    import torch
    n_p = L.shape[0]
    ld = L.stride(0)
    e = [int(v) for v in exps]
    name = "psdproj_sym_gemm_pair8_bf16" if L.dtype == torch.bfloat16 else "psdproj_sym_gemm_pair8"
    _check(getattr(lib(), name)(n_p, ld, _ptr(L), _ptr(Lx), _ptr(R), _ptr(Rx), _ptr(C0), _ptr(C0x),
                                float(alpha), float(beta), float(gamma), _ptr(D), _ptr(Dx),
                                e[0], e[1], e[2], e[3], _stream(stream)), name)
    return D


GEMM_CLASSES = ("plain", "plain_split_out", "pair", "pair_split_out", "final", "pair_final")


class _TimingEntry(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


def gemm_timing_start():
    """Bracket every filter product of later projections with HIP events."""
    _check(lib().psdproj_gemm_timing_start(), "psdproj_gemm_timing_start")


def gemm_timing_stop():
    """Stop, wait for the recorded events, and return
    {class: {"launches": k, "total_ms": t, "avg_ms": t / k}}."""
    arr = (_TimingEntry * len(GEMM_CLASSES))()
    _check(lib().psdproj_gemm_timing_stop(ctypes.cast(arr, ctypes.c_void_p), len(GEMM_CLASSES)),
           "psdproj_gemm_timing_stop")
    return {name: {"launches": int(e.launches), "total_ms": float(e.total_ms),
                   "avg_ms": float(e.total_ms) / e.launches if e.launches else None}
            for name, e in zip(GEMM_CLASSES, arr)}


# ---------------------------------------------------------------------------
# serving loop
# ---------------------------------------------------------------------------
class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int),
                ("max_bypass", ctypes.c_int), ("fake_executor", ctypes.c_int),
                ("fake_tflops", ctypes.c_double), ("coalesce_max_n", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("X", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("target", ctypes.c_double), ("mode", ctypes.c_int),
                ("tag", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("mode", ctypes.c_int), ("tag", ctypes.c_uint64),
                ("submit_ns", ctypes.c_int64), ("start_ns", ctypes.c_int64), ("end_ns", ctypes.c_int64),
                ("slot", ctypes.c_int)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("cancelled", ctypes.c_uint64),
                ("pending", ctypes.c_uint64), ("running", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("throughput_per_s", ctypes.c_double),
                ("bytes_held", ctypes.c_size_t), ("peak_bytes_held", ctypes.c_size_t)]


def _serve_sigs(L):
    vp = ctypes.c_void_p
    L.psdproj_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
    L.psdproj_serve_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.psdproj_serve_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(Result)]
    L.psdproj_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.psdproj_serve_cancel.argtypes = [vp, ctypes.c_uint64]
    L.psdproj_serve_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    L.psdproj_serve_destroy.argtypes = [vp]
    for nm in ("create", "submit", "wait", "poll", "cancel", "stats", "destroy"):
        getattr(L, "psdproj_serve_" + nm).restype = ctypes.c_int


def _res_dict(r: Result) -> dict:
    return {k: getattr(r, k) for k, _ in Result._fields_}


class Server:
    """Continuous-batching projection server (psdproj_serve_*)."""

    def __init__(self, hbm_budget_bytes=0, slots=0, max_bypass=0, fake_executor=False, fake_tflops=0.0,
                 coalesce_max_n=0):
        L = lib()
        _serve_sigs(L)
        self._L = L
        cfg = ServeConfig(int(hbm_budget_bytes), int(slots), int(max_bypass), int(bool(fake_executor)),
                          float(fake_tflops), int(coalesce_max_n))
        h = ctypes.c_void_p()
        _check(L.psdproj_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "psdproj_serve_create")
        self._h = h

    def submit(self, n=None, X=None, out=None, target=1e-3, mode=-1, tag=0, ld=None):
        """Returns a ticket, or raises PsdprojError (e.g. status 5 = rejected).
        With X given, n and ld come from it; out must match X."""
        if X is not None:
            n, ld = _check_matrix(X)
            if out is None or _check_matrix(out, "out") != (n, ld):
                raise ValueError("out must match X in shape and stride")
        if n is None:
            raise ValueError("n or X is required")
        req = Request(int(n), int(ld if ld is not None else max(1, n)),
                      None if X is None else X.data_ptr(), None if out is None else out.data_ptr(),
                      float(target), _mode(mode) if isinstance(mode, str) else int(mode), int(tag))
        tk = ctypes.c_uint64()
        _check(self._L.psdproj_serve_submit(self._h, ctypes.byref(req), ctypes.byref(tk)), "psdproj_serve_submit")
        return tk.value

    def wait(self, ticket, timeout_s=None):
        r = Result()
        t = -1 if timeout_s is None else int(timeout_s * 1e9)
        st = self._L.psdproj_serve_wait(self._h, ticket, t, ctypes.byref(r))
        if st != 0:
            raise PsdprojError(st, "psdproj_serve_wait")
        return _res_dict(r)

    def poll(self, ticket):
        r = Result()
        st = self._L.psdproj_serve_poll(self._h, ticket, ctypes.byref(r))
        if st == 9:
            return None
        _check(st, "psdproj_serve_poll")
        return _res_dict(r)

    def cancel(self, ticket) -> int:
        return int(self._L.psdproj_serve_cancel(self._h, ticket))

    def stats(self) -> dict:
        s = ServeStats()
        _check(self._L.psdproj_serve_stats(self._h, ctypes.byref(s)), "psdproj_serve_stats")
        return {k: getattr(s, k) for k, _ in ServeStats._fields_}

    def close(self):
        if self._h:
            _check(self._L.psdproj_serve_destroy(self._h), "psdproj_serve_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
