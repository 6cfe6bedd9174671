"""Thin ctypes binding over libatsne.so (C ABI in include/atsne.h).

Argument marshalling only: every step of the similarity path runs in the HIP
library.  Tensors are torch CUDA (HIP) tensors used as device buffers; the
stream is torch's current stream unless one is given.  The binding raises
if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
from pathlib import Path

import torch

_HERE = Path(__file__).resolve().parent
LIBPATH = _HERE / "libatsne.so"

OK, E_INVALID_ARG, E_K_RANGE, E_NOMEM, E_HIP, E_NOT_CONVERGED, E_BUSY, E_UNSUPPORTED = range(8)
PREC = {"fp32": 0, "bf16": 1, "fp8": 2, "fp8_e4m3": 2, "fp32x3": 3}
FLAG_FP64_RERANKED, FLAG_NOT_CONVERGED, FLAG_DEGENERATE, FLAG_EXACT_SCAN, FLAG_TOL_LIMITED = 1, 2, 4, 8, 16

# symbols declared by include/atsne.h
EXPORTS = [
    "atsne_last_error", "atsne_version", "atsne_device_info", "atsne_profile_enable", "atsne_profile_read",
    "atsne_knn_workspace_size", "atsne_knn", "atsne_knn_subset",
    "atsne_calibrate_p",
    "atsne_symmetrize_workspace_size", "atsne_symmetrize", "atsne_symmetrize_csr", "atsne_symmetrize_noalloc",
    "atsne_ivf_build", "atsne_ivf_partition", "atsne_ivf_knn", "atsne_ivf_fit", "atsne_ivf_destroy",
    "atsne_attractive_forces", "atsne_order_workspace_size", "atsne_order_density", "atsne_order_neighbourhood",
    "atsne_serve_create", "atsne_serve_submit_insert", "atsne_serve_submit_refine", "atsne_serve_submit_delete",
    "atsne_serve_poll",
    "atsne_serve_wait", "atsne_serve_release", "atsne_serve_stats_get", "atsne_serve_snapshot",
    "atsne_serve_destroy",
]


class AtsneError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("atsne status %d: %s" % (status, msg))
        self.status = status


_lib = None

_p = ctypes.c_void_p
_i32, _i64, _f32, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("capacity_rows", ctypes.c_int64), ("max_batch_rows", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("kind", ctypes.c_int32), ("status", ctypes.c_int32),
                ("epoch", ctypes.c_uint64), ("n_rows", ctypes.c_int64), ("k", ctypes.c_int32),
                ("perplexity", ctypes.c_float), ("row_ids", _p), ("nbr_idx", _p), ("nbr_d2", _p),
                ("P_cond", _p), ("beta", _p), ("flags", _p), ("n_changed", ctypes.c_int64), ("changed", _p),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_complete_ms", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("released", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("rows_processed", ctypes.c_uint64), ("corpus_rows", ctypes.c_int64),
                ("bytes_in_flight", ctypes.c_size_t), ("peak_bytes_in_flight", ctypes.c_size_t),
                ("max_concurrent", ctypes.c_int32), ("max_requests_per_launch", ctypes.c_int32)]


def load(path: Path | None = None) -> ctypes.CDLL:
    """Load libatsne.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    path = Path(path) if path is not None else LIBPATH
    if not path.exists():
        raise RuntimeError("libatsne.so not built at %s: run python -m paper_1512_01655_amd.build" % path)
    L = ctypes.CDLL(str(path))
    L.atsne_last_error.restype = ctypes.c_char_p
    L.atsne_version.restype = ctypes.c_char_p
    sig = {
        "atsne_device_info": [_p, _p, _p],
        "atsne_profile_enable": [_i32],
        "atsne_profile_read": [ctypes.c_char_p, _p, _p],
        "atsne_knn_workspace_size": [_i64, _i64, _i32, ctypes.c_int, _i32, _i32, _p],
        "atsne_knn": [_p, _i64, _i32, _i64, ctypes.c_int, _i32, _i32, _p, _p, _p, _p, _p, _sz, _p],
        "atsne_knn_subset": [_p, _i64, _i32, _i64, _p, _i64, ctypes.c_int, _i32, _i32, _p, _p, _p, _p, _p, _sz,
                             _p],
        "atsne_calibrate_p": [_p, _p, _i64, _i32, _f32, _f32, _i32, _i32, _p, _p, _p, _p, _p],
        "atsne_symmetrize_workspace_size": [_i64, _i64, _p],
        "atsne_symmetrize": [_p, _p, _i64, _i32, _p, _p, _p, _p, _p, _sz, _p],
        "atsne_symmetrize_noalloc": [_p, _p, _i64, _i32, _p, _p, _p, _p, _p],
        "atsne_symmetrize_csr": [_p, _p, _p, _i64, _i64, _p, _p, _p, _p, _p, _sz, _p],
        "atsne_attractive_forces": [_p, _p, _p, _i64, _i64, _p, _i32, _p, _f32, _f32, _i32, _f32, _p, _p],
        "atsne_ivf_build": [_p, _i64, _i32, _i32, _p, _i32, _p, _p],
        "atsne_ivf_partition": [_p, _p, _p, _p, _p, _p],
        "atsne_ivf_knn": [_p, _i32, _i32, _p, _p, _p, _p, _p],
        "atsne_ivf_fit": [_p, _i32, _f32, _p, _i32, _p, _p, _p],
        "atsne_ivf_destroy": [_p],
        "atsne_order_workspace_size": [_i64, _p],
        "atsne_order_density": [_p, _i64, _p, _i64, _p, _p, ctypes.c_size_t, _p],
        "atsne_order_neighbourhood": [_p, _p, _i64, _i32, _p, _i64, _i32, _i32, _p, _p, _p, _p, ctypes.c_size_t,
                                      _p],
        "atsne_serve_create": [_p, _p, _i64, _i32, _f32, _p],
        "atsne_serve_submit_insert": [_p, _p, _i32, _p],
        "atsne_serve_submit_refine": [_p, _p, _i32, _f32, _p],
        "atsne_serve_submit_delete": [_p, _p, _i32, _p],
        "atsne_serve_poll": [_p, ctypes.c_uint64, _p],
        "atsne_serve_wait": [_p, ctypes.c_uint64, _p],
        "atsne_serve_release": [_p, ctypes.c_uint64],
        "atsne_serve_stats_get": [_p, _p],
        "atsne_serve_snapshot": [_p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p],
        "atsne_serve_destroy": [_p, _i32],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    if path == LIBPATH:
        _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise AtsneError(status, load().atsne_last_error().decode())


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(X: torch.Tensor, dtype, name):
    if not (X.is_cuda and X.dtype == dtype):
        raise ValueError("%s must be a %s device tensor" % (name, dtype))


def knn(X: torch.Tensor, k: int, prec: str = "fp32", k_cand: int = 0, query_ids: torch.Tensor | None = None,
        stream=None, workspace: torch.Tensor | None = None, d2_lo: torch.Tensor | None = None):
    """Exact kNN (atsne_knn / atsne_knn_subset).  Returns (nbr_idx int32, nbr_d2 float32, flags uint8);
    ``d2_lo`` (optional float32 [M, k] device tensor) receives the distances' residuals."""
    L = load()
    _dev(X, torch.float32, "X")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit column stride")
    N, D = X.shape
    ld = X.stride(0)
    M = N if query_ids is None else query_ids.numel()
    if query_ids is not None:
        _dev(query_ids, torch.int32, "query_ids")
    need = ctypes.c_size_t()
    _check(L.atsne_knn_workspace_size(N, M, D, PREC[prec], k, k_cand, ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(1, need.value), dtype=torch.uint8, device=X.device)
    idx = torch.empty((M, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((M, k), dtype=torch.float32, device=X.device)
    flags = torch.zeros((M,), dtype=torch.uint8, device=X.device)
    if d2_lo is not None:
        _dev(d2_lo, torch.float32, "d2_lo")
        if tuple(d2_lo.shape) != (M, k) or not d2_lo.is_contiguous():
            raise ValueError("d2_lo must be a contiguous [%d, %d] tensor" % (M, k))
    if query_ids is None:
        _check(L.atsne_knn(_ptr(X), N, D, ld, PREC[prec], k, k_cand, _ptr(idx), _ptr(d2), _ptr(d2_lo), _ptr(flags),
                           _ptr(workspace), workspace.numel(), _stream(stream)))
    else:
        _check(L.atsne_knn_subset(_ptr(X), N, D, ld, _ptr(query_ids), M, PREC[prec], k, k_cand, _ptr(idx),
                                  _ptr(d2), _ptr(d2_lo), _ptr(flags), _ptr(workspace), workspace.numel(),
                                  _stream(stream)))
    return idx, d2, flags


def knn_workspace_size(N: int, M: int, D: int, k: int, prec: str = "fp32", k_cand: int = 0) -> int:
    need = ctypes.c_size_t()
    _check(load().atsne_knn_workspace_size(N, M, D, PREC[prec], k, k_cand, ctypes.byref(need)))
    return need.value


def calibrate_p(nbr_d2: torch.Tensor, perplexity: float, tol: float = 0.0, max_iter: int = 0, strict: bool = False,
                flags: torch.Tensor | None = None, stream=None, d2_lo: torch.Tensor | None = None):
    """Perplexity bisection (atsne_calibrate_p).  Returns (P_cond, beta, perp, flags).  ``d2_lo``: the
    distances' residuals from knn (optional)."""
    L = load()
    _dev(nbr_d2, torch.float32, "nbr_d2")
    nbr_d2 = nbr_d2.contiguous()
    if d2_lo is not None:
        _dev(d2_lo, torch.float32, "d2_lo")
        d2_lo = d2_lo.contiguous()
        if d2_lo.shape != nbr_d2.shape:
            raise ValueError("d2_lo must match nbr_d2")
    N, k = nbr_d2.shape
    P = torch.empty_like(nbr_d2)
    beta = torch.empty((N,), dtype=torch.float32, device=nbr_d2.device)
    perp = torch.empty((N,), dtype=torch.float32, device=nbr_d2.device)
    if flags is None:
        flags = torch.zeros((N,), dtype=torch.uint8, device=nbr_d2.device)
    _check(L.atsne_calibrate_p(_ptr(nbr_d2), _ptr(d2_lo), N, k, float(perplexity), float(tol), int(max_iter), int(strict),
                               _ptr(P), _ptr(beta), _ptr(perp), _ptr(flags), _stream(stream)))
    return P, beta, perp, flags


def symmetrize(nbr_idx: torch.Tensor, P_cond: torch.Tensor, stream=None, workspace: torch.Tensor | None = None):
    """Symmetric joint P as CSR (atsne_symmetrize).  Returns (row_ptr int64, col int32, val float32)."""
    L = load()
    _dev(nbr_idx, torch.int32, "nbr_idx")
    _dev(P_cond, torch.float32, "P_cond")
    nbr_idx, P_cond = nbr_idx.contiguous(), P_cond.contiguous()
    N, k = nbr_idx.shape
    need = ctypes.c_size_t()
    _check(L.atsne_symmetrize_workspace_size(N, N * k, ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(1, need.value), dtype=torch.uint8, device=nbr_idx.device)
    row_ptr = torch.empty((N + 1,), dtype=torch.int64, device=nbr_idx.device)
    col = torch.empty((2 * N * k,), dtype=torch.int32, device=nbr_idx.device)
    val = torch.empty((2 * N * k,), dtype=torch.float32, device=nbr_idx.device)
    nnz = ctypes.c_int64()
    _check(L.atsne_symmetrize(_ptr(nbr_idx), _ptr(P_cond), N, k, _ptr(row_ptr), _ptr(col), _ptr(val),
                              ctypes.byref(nnz), _ptr(workspace), workspace.numel(), _stream(stream)))
    return row_ptr, col[:nnz.value], val[:nnz.value]


def symmetrize_noalloc(nbr_idx: torch.Tensor, P_cond: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor,
                       val: torch.Tensor, stream=None) -> int:
    """atsne_symmetrize_noalloc into caller-allocated outputs (row_ptr [N+1] int64, col/val with capacity 2*N*k);
    returns nnz.  The call itself allocates nothing."""
    L = load()
    _dev(nbr_idx, torch.int32, "nbr_idx")
    _dev(P_cond, torch.float32, "P_cond")
    N, k = nbr_idx.shape
    if not (nbr_idx.is_contiguous() and P_cond.is_contiguous() and P_cond.shape == nbr_idx.shape):
        raise ValueError("contiguous nbr_idx and P_cond of one shape are required")
    if row_ptr.numel() < N + 1 or col.numel() < 2 * N * k or val.numel() < 2 * N * k:
        raise ValueError("output capacity too small")
    nnz = ctypes.c_int64()
    _check(L.atsne_symmetrize_noalloc(_ptr(nbr_idx), _ptr(P_cond), N, k, _ptr(row_ptr), _ptr(col), _ptr(val),
                                      ctypes.byref(nnz), _stream(stream)))
    return nnz.value


def symmetrize_csr(in_ptr: torch.Tensor, in_col: torch.Tensor, in_val: torch.Tensor, stream=None):
    """Symmetrise variable-length conditional rows given as CSR (atsne_symmetrize_csr)."""
    L = load()
    N = in_ptr.numel() - 1
    nnz_in = int(in_ptr[-1].item())
    need = ctypes.c_size_t()
    _check(L.atsne_symmetrize_workspace_size(N, nnz_in, ctypes.byref(need)))
    ws = torch.empty(max(1, need.value), dtype=torch.uint8, device=in_ptr.device)
    row_ptr = torch.empty((N + 1,), dtype=torch.int64, device=in_ptr.device)
    col = torch.empty((max(1, 2 * nnz_in),), dtype=torch.int32, device=in_ptr.device)
    val = torch.empty((max(1, 2 * nnz_in),), dtype=torch.float32, device=in_ptr.device)
    nnz = ctypes.c_int64()
    _check(L.atsne_symmetrize_csr(_ptr(in_ptr), _ptr(in_col), _ptr(in_val), N, nnz_in, _ptr(row_ptr), _ptr(col),
                                  _ptr(val), ctypes.byref(nnz), _ptr(ws), ws.numel(), _stream(stream)))
    return row_ptr, col[:nnz.value], val[:nnz.value]


def similarity(X: torch.Tensor, perplexity: float, prec: str = "fp32", k: int | None = None, k_cand: int = 0,
               stream=None):
    """kNN -> calibration -> symmetrisation, K = floor(3 mu) unless k is given."""
    if k is None:
        k = int(math.floor(3.0 * perplexity))
    M = X.shape[0]
    d2_lo = torch.empty((M, k), dtype=torch.float32, device=X.device)
    idx, d2, flags = knn(X, k, prec=prec, k_cand=k_cand, stream=stream, d2_lo=d2_lo)
    P, beta, perp, flags = calibrate_p(d2, perplexity, flags=flags, stream=stream, d2_lo=d2_lo)
    row_ptr, col, val = symmetrize(idx, P, stream=stream)
    return dict(idx=idx, d2=d2, flags=flags, P=P, beta=beta, perp=perp, row_ptr=row_ptr, col=col, val=val)


def attractive_forces(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, Y: torch.Tensor,
                      t_ref: torch.Tensor | None = None, tau: float = 1.0, decay: float = 1.0, t_now: int = 0,
                      global_exaggeration: float = 1.0, stream=None, out: torch.Tensor | None = None):
    """F_attr of Eq. 7 over the symmetric CSR P (Sec. 4.3 exaggeration); returns F [N, dims]."""
    _dev(row_ptr, torch.int64, "row_ptr")
    _dev(Y, torch.float32, "Y")
    N, dims = Y.shape
    nnz = int(col.shape[0])
    if nnz:
        _dev(col, torch.int32, "col")
        _dev(val, torch.float32, "val")
    if t_ref is not None:
        _dev(t_ref, torch.int32, "t_ref")
    Yc = Y.contiguous()
    F = out if out is not None else torch.empty((N, dims), dtype=torch.float32, device=Y.device)
    _check(load().atsne_attractive_forces(_ptr(row_ptr), _ptr(col) if nnz else None, _ptr(val) if nnz else None,
                                          N, nnz, _ptr(Yc), dims, _ptr(t_ref), float(tau),
                                          float(decay), int(t_now), float(global_exaggeration), _ptr(F),
                                          _stream(stream)))
    return F


def order_density(beta: torch.Tensor, ids: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Density-based refinement order (Sec. 5.1): ids by sigma descending, ties by index."""
    _dev(beta, torch.float32, "beta")
    N = beta.shape[0]
    if ids is not None:
        _dev(ids, torch.int32, "ids")
    M = N if ids is None else ids.shape[0]
    out = torch.empty((M,), dtype=torch.int32, device=beta.device)
    _check(load().atsne_order_density(_ptr(beta), N, _ptr(ids), M, _ptr(out), None, 0, _stream(stream)))
    return out


def order_neighbourhood(nbr_idx: torch.Tensor, nbr_d2: torch.Tensor | None, seeds: torch.Tensor,
                        weighted: bool = False, max_depth: int = -1, stream=None):
    """Breadth-first refinement order (Sec. 5.1).  Returns (order [n_reached], key [N])."""
    _dev(nbr_idx, torch.int32, "nbr_idx")
    _dev(seeds, torch.int32, "seeds")
    if weighted:
        _dev(nbr_d2, torch.float32, "nbr_d2")
    N, k = nbr_idx.shape
    key = torch.empty((N,), dtype=torch.float32, device=nbr_idx.device)
    order = torch.empty((N,), dtype=torch.int32, device=nbr_idx.device)
    n = ctypes.c_int64()
    _check(load().atsne_order_neighbourhood(_ptr(nbr_idx.contiguous()), _ptr(nbr_d2) if weighted else None, N, k,
                                            _ptr(seeds), seeds.shape[0], 1 if weighted else 0, int(max_depth),
                                            _ptr(key), _ptr(order), ctypes.byref(n), None, 0, _stream(stream)))
    return order[: n.value], key


class IVF:
    """Precision-controlled approximate kNN (atsne_ivf_*): cluster-pruned search."""

    def __init__(self, X: torch.Tensor, n_clusters: int, iters: int = 10, seed: int = 0, init_ids=None, stream=None):
        import numpy as np

        _dev(X, torch.float32, "X")
        X = X.contiguous()
        self.N, self.D = X.shape
        self.C = int(n_clusters)
        if init_ids is None:
            init_ids = np.random.default_rng(seed).choice(self.N, size=self.C, replace=False)
        ids = np.ascontiguousarray(init_ids, dtype=np.int32)
        self.h = ctypes.c_void_p()
        _check(load().atsne_ivf_build(_ptr(X), self.N, self.D, self.C, ids.ctypes.data_as(_p), int(iters),
                                      ctypes.byref(self.h), _stream(stream)))

    def partition(self, stream=None):
        """(assign [N] int32, centroids [C, D] FP32 device; cluster_start [C+1], probe [C, C] numpy)."""
        import numpy as np

        assign = torch.empty((self.N,), dtype=torch.int32, device="cuda")
        cent = torch.empty((self.C, self.D), dtype=torch.float32, device="cuda")
        start = np.empty((self.C + 1,), np.int64)
        probe = np.empty((self.C, self.C), np.int32)
        _check(load().atsne_ivf_partition(self.h, _ptr(assign), _ptr(cent), start.ctypes.data_as(_p),
                                          probe.ctypes.data_as(_p), _stream(stream)))
        return assign, cent, start, probe

    def knn(self, k: int, n_probe: int, stream=None):
        """(idx [N, k] int32, d2 [N, k] FP32, flags [N] uint8, candidate fraction)."""
        idx = torch.empty((self.N, k), dtype=torch.int32, device="cuda")
        d2 = torch.empty((self.N, k), dtype=torch.float32, device="cuda")
        fl = torch.zeros((self.N,), dtype=torch.uint8, device="cuda")
        frac = ctypes.c_double()
        _check(load().atsne_ivf_knn(self.h, int(k), int(n_probe), _ptr(idx), _ptr(d2), _ptr(fl), ctypes.byref(frac),
                                    _stream(stream)))
        return idx, d2, fl, frac.value

    def fit(self, k: int, rho: float, sample_clusters, stream=None):
        """Smallest n_probe reaching precision rho on the sample clusters: (n_probe, sample precision)."""
        import numpy as np

        sc = np.ascontiguousarray(sample_clusters, dtype=np.int32)
        n, r = ctypes.c_int32(), ctypes.c_float()
        _check(load().atsne_ivf_fit(self.h, int(k), float(rho), sc.ctypes.data_as(_p), sc.size, ctypes.byref(n),
                                    ctypes.byref(r), _stream(stream)))
        return n.value, r.value

    def close(self):
        if getattr(self, "h", None):
            _check(load().atsne_ivf_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_info():
    n_cu, clk, major = _i32(), _i32(), _i32()
    _check(load().atsne_device_info(ctypes.byref(n_cu), ctypes.byref(clk), ctypes.byref(major)))
    return dict(n_cu=n_cu.value, clock_khz=clk.value, arch_major=major.value)


def profile_enable(on: bool = True):
    """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
    _check(load().atsne_profile_enable(1 if on else 0))


def profile_read(name: str):
    """(total_ms, launches) of library kernels whose name starts with `name`."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(load().atsne_profile_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# --------------------------------------------------------------------------- serving
_hip = None


def _hip_lib():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [_p, _p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def _d2h(ptr, shape, dtype):
    import numpy as np

    out = np.empty(shape, dtype=dtype)
    if out.size:
        rc = _hip_lib().hipMemcpy(out.ctypes.data_as(_p), ctypes.c_void_p(ptr), out.nbytes, 2)  # DeviceToHost
        if rc != 0:
            raise RuntimeError("hipMemcpy D2H failed (%d)" % rc)
    return out


class Server:
    """Continuous-batching server over a device-resident corpus (atsne_serve_*)."""

    def __init__(self, corpus: torch.Tensor, perplexity: float, hbm_budget_bytes: int = 0, max_slots: int = 0,
                 capacity_rows: int = 0, max_batch_rows: int = 0):
        L = load()
        _dev(corpus, torch.float32, "corpus")
        corpus = corpus.contiguous()
        self.N0, self.D = corpus.shape
        cfg = ServeConfig(hbm_budget_bytes, max_slots, capacity_rows, max_batch_rows, -1)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(L.atsne_serve_create(ctypes.byref(cfg), _ptr(corpus), self.N0, self.D, float(perplexity),
                                    ctypes.byref(h)))
        self.h = h
        self.perplexity = perplexity

    def insert(self, X_new: torch.Tensor) -> int:
        _dev(X_new, torch.float32, "X_new")
        X_new = X_new.contiguous()
        torch.cuda.synchronize()
        rid = ctypes.c_uint64()
        _check(load().atsne_serve_submit_insert(self.h, _ptr(X_new), X_new.shape[0], ctypes.byref(rid)))
        return rid.value

    def refine(self, ids, perplexity: float) -> int:
        import numpy as np

        ids = np.ascontiguousarray(ids, dtype=np.int32)
        rid = ctypes.c_uint64()
        _check(load().atsne_serve_submit_refine(self.h, ids.ctypes.data_as(_p), ids.size, float(perplexity),
                                                ctypes.byref(rid)))
        return rid.value

    def delete(self, ids) -> int:
        """Remove live points (Sec. 5.3); later requests no longer see them."""
        import numpy as np

        ids = np.ascontiguousarray(ids, dtype=np.int32)
        rid = ctypes.c_uint64()
        _check(load().atsne_serve_submit_delete(self.h, ids.ctypes.data_as(_p), ids.size, ctypes.byref(rid)))
        return rid.value

    @staticmethod
    def _result(r: Result, fetch: bool):
        import numpy as np

        out = dict(req_id=r.req_id, kind=("insert", "refine", "delete")[r.kind], status=r.status, epoch=r.epoch,
                   n_rows=r.n_rows, k=r.k, perplexity=r.perplexity, n_changed=r.n_changed,
                   t_submit_ms=r.t_submit_ms, t_admit_ms=r.t_admit_ms, t_complete_ms=r.t_complete_ms)
        if fetch and r.status == OK:
            n, k = r.n_rows, r.k
            out["row_ids"] = _d2h(r.row_ids, (n,), np.int32)
            if r.kind != 2:
                out["idx"] = _d2h(r.nbr_idx, (n, k), np.int32)
                out["d2"] = _d2h(r.nbr_d2, (n, k), np.float32)
                out["P"] = _d2h(r.P_cond, (n, k), np.float32)
                out["beta"] = _d2h(r.beta, (n,), np.float32)
                out["flags"] = _d2h(r.flags, (n,), np.uint8)
            if r.kind != 1:
                out["changed"] = _d2h(r.changed, (r.n_changed,), np.int32)
        return out

    def poll(self, rid: int, fetch: bool = True):
        r = Result()
        st = load().atsne_serve_poll(self.h, rid, ctypes.byref(r))
        if st == E_BUSY:
            return None
        _check(st)
        return self._result(r, fetch)

    def wait(self, rid: int, fetch: bool = True):
        r = Result()
        _check(load().atsne_serve_wait(self.h, rid, ctypes.byref(r)))
        return self._result(r, fetch)

    def release(self, rid: int):
        _check(load().atsne_serve_release(self.h, rid))

    def stats(self):
        st = ServeStats()
        _check(load().atsne_serve_stats_get(self.h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServeStats._fields_}

    def snapshot(self):
        """(corpus, idx, d2, P, beta, rho, alive) numpy copies of the state once
        every submitted insert and delete is applied."""
        st = self.stats()
        cap = st["corpus_rows"]
        K = int(math.floor(3 * self.perplexity))
        X = torch.empty((cap, self.D), dtype=torch.float32, device="cuda")
        idx = torch.empty((cap, K), dtype=torch.int32, device="cuda")
        d2 = torch.empty((cap, K), dtype=torch.float32, device="cuda")
        P = torch.empty((cap, K), dtype=torch.float32, device="cuda")
        beta = torch.empty((cap,), dtype=torch.float32, device="cuda")
        rho = torch.empty((cap,), dtype=torch.float32, device="cuda")
        alive = torch.empty((cap,), dtype=torch.uint8, device="cuda")
        n, ep = ctypes.c_int64(), ctypes.c_uint64()
        torch.cuda.synchronize()
        _check(load().atsne_serve_snapshot(self.h, cap, _ptr(X), _ptr(idx), _ptr(d2), _ptr(P), _ptr(beta), _ptr(rho),
                                           _ptr(alive), ctypes.byref(n), ctypes.byref(ep)))
        n = n.value
        return tuple(t[:n].cpu().numpy() for t in (X, idx, d2, P, beta, rho, alive))

    def close(self, force: bool = True):
        if getattr(self, "h", None):
            _check(load().atsne_serve_destroy(self.h, 1 if force else 0))
            self.h = None

    def __del__(self):
        try:
            self.close(True)
        except Exception:
            pass
