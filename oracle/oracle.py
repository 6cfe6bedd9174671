"""FP64 CPU oracle for the A-tSNE similarity path -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``atsne_oracle.c`` (plain C, double precision).
Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module; the GPU library never does, and the two share no
code.

Functions (each follows the passage cited in the C source):
  knn(X, K, query_ids=None)          exact brute-force kNN, key (d, j)   -- Eq. 3, Eq. 8
  knn_candidates(X, K, q, ptr, idx)  the same over per-query candidate rows (approximate search)
  calibrate(d2, mu)                  bisection on beta to perplexity mu  -- Eq. 3, Eq. 4, Eq. 8
  symmetrize(idx_or_ptr, ...)        p_ij = (p_{j|i} + p_{i|j}) / 2N      -- Eq. 2, Eq. 10
  similarity(X, mu)                  the three steps chained, K = floor(3 mu)
  attractive(row_ptr, col, val, Y)   F_attr of the gradient over sparse P  -- Eq. 5-7, Sec. 4.3

Parity status: all functions pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
SOURCE = _HERE / "atsne_oracle.c"
LIBPATH = _HERE / "liboracle.so"

FLAG_NOT_CONVERGED = 2
FLAG_DEGENERATE = 4


def build(mutant: int = 0, out: Path | None = None) -> Path:
    """Compile the oracle with gcc (OpenMP).  ``mutant`` > 0 plants a bug."""
    out = Path(out) if out is not None else LIBPATH
    tmp = out.with_suffix(".so.tmp%d" % os.getpid())
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-DORACLE_MUTANT=%d" % int(mutant), str(SOURCE), "-o", str(tmp), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class Oracle:
    """Handle on one compiled oracle library (the default, or a mutant)."""

    def __init__(self, path: Path | None = None):
        path = Path(path) if path is not None else LIBPATH
        if not path.exists() or (path == LIBPATH and path.stat().st_mtime < SOURCE.stat().st_mtime):
            build(out=path)
        self.lib = ctypes.CDLL(str(path))
        L = self.lib
        p = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.atsne_oracle_knn.argtypes = [p, i64, i32, i64, p, i64, i32, p, p, p, i32]
        L.atsne_oracle_knn.restype = ctypes.c_int
        L.atsne_oracle_calibrate.argtypes = [p, i64, i32, p, f64, i32, p, p, p, p, i32]
        L.atsne_oracle_calibrate.restype = ctypes.c_int
        L.atsne_oracle_symmetrize.argtypes = [p, p, p, i64, p, p, p, i64]
        L.atsne_oracle_symmetrize.restype = ctypes.c_int64
        L.atsne_oracle_knn_candidates.argtypes = [p, i64, i32, i64, p, i64, p, p, i32, p, p, p, i32]
        L.atsne_oracle_knn_candidates.restype = ctypes.c_int
        L.atsne_oracle_attractive.argtypes = [p, p, p, i64, p, i32, p, f64, f64, i32, f64, p]
        L.atsne_oracle_attractive.restype = ctypes.c_int
        L.atsne_oracle_mutant.restype = ctypes.c_int
        L.atsne_oracle_max_threads.restype = ctypes.c_int
        self.mutant = L.atsne_oracle_mutant()

    @staticmethod
    def _ptr(a: np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)

    def max_threads(self) -> int:
        return int(self.lib.atsne_oracle_max_threads())

    def knn(self, X: np.ndarray, K: int, query_ids=None, nthreads: int = 0):
        """Exact kNN of rows ``query_ids`` (default: all) against all rows of X.

        Returns (idx int32[M,K], d2 float64[M,K], d2_next float64[M]).
        """
        X = np.ascontiguousarray(X, dtype=np.float32)
        N, D = X.shape
        if query_ids is None:
            qids = None
            M = N
        else:
            qids = np.ascontiguousarray(query_ids, dtype=np.int32)
            M = qids.shape[0]
        idx = np.empty((M, K), np.int32)
        d2 = np.empty((M, K), np.float64)
        nxt = np.empty((M,), np.float64)
        rc = self.lib.atsne_oracle_knn(self._ptr(X), N, D, D,
                                       None if qids is None else self._ptr(qids), M, K,
                                       self._ptr(idx), self._ptr(d2), self._ptr(nxt), int(nthreads))
        if rc != 0:
            raise ValueError("oracle knn: bad arguments")
        return idx, d2, nxt

    def knn_candidates(self, X: np.ndarray, K: int, query_ids, cand_ptr, cand_idx, nthreads: int = 0):
        """Exact kNN of each query over its own candidate rows (absent tail: -1, +inf).

        Returns (idx int32[M,K], d2 float64[M,K], d2_next float64[M]).
        """
        X = np.ascontiguousarray(X, dtype=np.float32)
        N, D = X.shape
        qids = np.ascontiguousarray(query_ids, dtype=np.int32)
        M = qids.shape[0]
        cp = np.ascontiguousarray(cand_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(cand_idx, dtype=np.int32)
        idx = np.empty((M, K), np.int32)
        d2 = np.empty((M, K), np.float64)
        nxt = np.empty((M,), np.float64)
        rc = self.lib.atsne_oracle_knn_candidates(self._ptr(X), N, D, D, self._ptr(qids), M, self._ptr(cp),
                                                  self._ptr(ci), K, self._ptr(idx), self._ptr(d2), self._ptr(nxt),
                                                  int(nthreads))
        if rc != 0:
            raise ValueError("oracle knn_candidates: bad arguments")
        return idx, d2, nxt

    def calibrate(self, d2: np.ndarray, mu, max_iter: int = 2000, nthreads: int = 0):
        """Bisection to perplexity ``mu`` (scalar or per row) on squared distances.

        Returns (P float64[M,K], beta float64[M], perp float64[M], flags uint8[M]).
        """
        d2 = np.ascontiguousarray(d2, dtype=np.float64)
        M, K = d2.shape
        if np.ndim(mu) == 0:
            mu_arr, mu_s = None, float(mu)
        else:
            mu_arr, mu_s = np.ascontiguousarray(mu, dtype=np.float64), 0.0
        P = np.empty((M, K), np.float64)
        beta = np.empty((M,), np.float64)
        perp = np.empty((M,), np.float64)
        flags = np.empty((M,), np.uint8)
        rc = self.lib.atsne_oracle_calibrate(self._ptr(d2), M, K,
                                             None if mu_arr is None else self._ptr(mu_arr), mu_s,
                                             int(max_iter), self._ptr(P), self._ptr(beta),
                                             self._ptr(perp), self._ptr(flags), int(nthreads))
        if rc != 0:
            raise ValueError("oracle calibrate: bad arguments (need 1 <= mu < K)")
        return P, beta, perp, flags

    def symmetrize_csr(self, in_ptr, in_col, in_val, N: int):
        """Symmetrise CSR conditional rows.  Returns (row_ptr int64, col int32, val float64)."""
        in_ptr = np.ascontiguousarray(in_ptr, dtype=np.int64)
        in_col = np.ascontiguousarray(in_col, dtype=np.int32)
        in_val = np.ascontiguousarray(in_val, dtype=np.float64)
        cap = 2 * int(in_ptr[N]) + 1
        row_ptr = np.empty((N + 1,), np.int64)
        col = np.empty((cap,), np.int32)
        val = np.empty((cap,), np.float64)
        nnz = self.lib.atsne_oracle_symmetrize(self._ptr(in_ptr), self._ptr(in_col), self._ptr(in_val),
                                               N, self._ptr(row_ptr), self._ptr(col), self._ptr(val), cap)
        if nnz < 0:
            raise ValueError("oracle symmetrize: bad arguments")
        return row_ptr, col[:nnz].copy(), val[:nnz].copy()

    def symmetrize(self, idx: np.ndarray, P: np.ndarray):
        """Symmetrise fixed-K rows (idx[N,K], P[N,K])."""
        N, K = idx.shape
        ptr = np.arange(0, N * K + 1, K, dtype=np.int64)
        return self.symmetrize_csr(ptr, idx.reshape(-1), P.reshape(-1), N)

    def attractive(self, row_ptr, col, val, Y, t_ref=None, tau: float = 1.0, decay: float = 1.0, t_now: int = 0,
                   global_exag: float = 1.0):
        """Attractive forces m_i sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2) (Eq. 5-7, Sec. 4.3)."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        N, dims = Y.shape
        tr = None if t_ref is None else np.ascontiguousarray(t_ref, dtype=np.int32)
        F = np.empty((N, dims), np.float64)
        rc = self.lib.atsne_oracle_attractive(self._ptr(row_ptr), self._ptr(col), self._ptr(val), N, self._ptr(Y),
                                              dims, None if tr is None else self._ptr(tr), float(tau), float(decay),
                                              int(t_now), float(global_exag), self._ptr(F))
        if rc != 0:
            raise ValueError("oracle attractive: bad arguments")
        return F

    def similarity(self, X: np.ndarray, mu: float, K: int | None = None, nthreads: int = 0):
        """kNN -> calibration -> symmetrisation with K = floor(3 mu) (Sec. 3.1)."""
        if K is None:
            K = int(math.floor(3.0 * mu))
        idx, d2, nxt = self.knn(X, K, nthreads=nthreads)
        P, beta, perp, flags = self.calibrate(d2, mu, nthreads=nthreads)
        row_ptr, col, val = self.symmetrize(idx, P)
        return dict(idx=idx, d2=d2, d2_next=nxt, P=P, beta=beta, perp=perp, flags=flags,
                    row_ptr=row_ptr, col=col, val=val)


_default: Oracle | None = None


def get() -> Oracle:
    """The default (non-mutant) oracle, built on first use."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def check_rows(rows: np.ndarray, query_ids=None, n: int | None = None) -> None:
    """Raise ValueError unless every row is a valid neighbour list: distinct
    ids, none equal to the row's own id (``query_ids``, when given), each in
    [0, n) (when ``n`` is given); -1 marks an absent entry (Sec. 5.3) and may
    only follow the listed ids."""
    rows = np.asarray(rows)
    if rows.ndim != 2:
        raise ValueError("neighbour lists must be a 2-D array")
    own = None if query_ids is None else np.asarray(query_ids).reshape(-1)
    if own is not None and own.shape[0] != rows.shape[0]:
        raise ValueError("one query id per row")
    for r in range(rows.shape[0]):
        row = [int(v) for v in rows[r]]
        listed = [v for v in row if v != -1]
        if row[:len(listed)] != listed:
            raise ValueError("row %d: an absent entry (-1) before a listed id" % r)
        if len(set(listed)) != len(listed):
            raise ValueError("row %d lists an id twice" % r)
        if any(v < 0 or (n is not None and v >= n) for v in listed):
            raise ValueError("row %d lists an id outside [0, %s)" % (r, n))
        if own is not None and int(own[r]) in listed:
            raise ValueError("row %d lists its own id %d" % (r, int(own[r])))


def recall(approx: np.ndarray, exact: np.ndarray, query_ids=None, n: int | None = None) -> float:
    """The precision rho of Eq. 9: the mean over rows of |N^A_i & N_i| / |N_i|,
    N^A_i the approximate (or low-precision) neighbour list and N_i the exact
    one of the same row.  Both are validated first (``check_rows``): a list
    with a repeated, self or out-of-range id raises ValueError instead of
    being scored, and an absent entry (-1) is a miss."""
    approx = np.asarray(approx)
    exact = np.asarray(exact)
    if approx.shape[0] != exact.shape[0]:
        raise ValueError("approximate and exact lists cover different rows")
    check_rows(approx, query_ids, n)
    check_rows(exact, query_ids, n)
    M, K = exact.shape
    if M == 0:
        return 1.0
    tot = 0
    for a, b in zip(approx.tolist(), exact.tolist()):
        tot += len(set(a) & set(b) - {-1})
    return tot / float(M * K)
