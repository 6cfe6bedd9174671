"""Parity rules between the GPU path and the FP64 oracle.

Tolerances (from the exact-path contract):
  * neighbour sets bit-exact, except where the oracle's K-th and (K+1)-th
    squared distances differ by less than 1e-5 relative: there the GPU set S
    is accepted iff |S| = K and A <= S <= B with
        A = {j : d_ij < d_K (1 - 1e-5)},  B = {j : d_ij <= d_K (1 + 1e-5)};
  * every P entry within 1e-6 absolute (conditional p_{j|i}, and 2N * p_ij
    for the joint, both of order 1/mu);
  * every row's perplexity within 1e-4 of the target.
"""
from __future__ import annotations

import numpy as np

TIE_REL = 1e-5
P_TOL = 1e-6
PERP_TOL = 1e-4
D2_REL = 8e-6  # FP32 direct-difference distance vs FP64 (relative)


def true_d2(X: np.ndarray, rows: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """FP64 squared distances (direct differences) from X[rows[r]] to X[idx[r, t]].

    Entries with idx < 0 (absent) get +inf.  Uses torch's multithreaded CPU
    kernels when torch is importable (full-size checks), numpy otherwise."""
    rows = np.asarray(rows)
    idx = np.asarray(idx)
    safe = np.where(idx >= 0, idx, 0)
    out = np.empty(idx.shape, np.float64)
    try:
        import torch

        Xt = torch.from_numpy(np.ascontiguousarray(X))
        for s in range(0, len(rows), 1024):
            e = min(len(rows), s + 1024)
            q = Xt[torch.from_numpy(rows[s:e].astype(np.int64))].double()
            g = Xt[torch.from_numpy(safe[s:e].astype(np.int64))].double()
            out[s:e] = ((g - q[:, None, :]) ** 2).sum(-1).numpy()
    except ImportError:
        X64 = X.astype(np.float64)
        for s in range(0, len(rows), 256):
            e = min(len(rows), s + 256)
            diff = X64[rows[s:e], None, :] - X64[safe[s:e]]
            out[s:e] = np.einsum("rkd,rkd->rk", diff, diff)
    out[idx < 0] = np.inf
    return out


def check_rows_valid(X, rows, g_idx, g_d2, d2_rel=D2_REL):
    """Every returned row is a valid neighbour list: distinct ids in [0, N),
    not the row itself, distances ascending and each within the FP32
    direct-difference error of the FP64 distance.  Returns the FP64 distances."""
    rows = np.asarray(rows)
    N = X.shape[0]
    assert np.all((g_idx >= 0) & (g_idx < N)), "neighbour id outside [0, N)"
    assert not np.any(g_idx == rows[:, None]), "self returned as neighbour"
    srt = np.sort(g_idx, axis=1)
    assert not np.any(srt[:, 1:] == srt[:, :-1]), "a neighbour listed twice"
    assert np.all(np.diff(g_d2, axis=1) >= 0), "distances not ascending"
    td = true_d2(X, rows, g_idx)
    err = np.abs(g_d2.astype(np.float64) - td)
    assert np.all(err <= d2_rel * np.maximum(td, 1e-30) + 1e-30), "max rel d2 error %g" % (
        (err / np.maximum(td, 1e-30)).max())
    return td


def recall_tie_aware(td, o_d2, o_idx, g_idx, rel=TIE_REL):
    """Eq. 9 counting a returned neighbour as found when it is one of the
    oracle's neighbours or lies within the tie band of the oracle's K-th
    distance (td: FP64 distances of the returned neighbours)."""
    K = o_idx.shape[1]
    dK = o_d2[:, K - 1]
    hit = np.zeros(g_idx.shape, bool)
    for r in range(g_idx.shape[0]):
        hit[r] = np.isin(g_idx[r], o_idx[r])
    hit |= td <= (dK * (1 + rel))[:, None]
    return float(hit.mean())


def union_dP(g_idx, g_P, o_idx, o_P):
    """max over rows and over the union of the two rows' supports of
    |p_gpu - p_oracle|, an entry absent from one side counting as 0."""
    M, K = o_idx.shape
    r = np.repeat(np.arange(M, dtype=np.int64), K)
    N = int(max(g_idx.max(), o_idx.max())) + 1
    gk = r * N + g_idx.reshape(-1).astype(np.int64)
    ok = r * N + o_idx.reshape(-1).astype(np.int64)
    keys = np.union1d(gk, ok)
    gv = np.zeros(keys.shape, np.float64)
    ov = np.zeros(keys.shape, np.float64)
    gv[np.searchsorted(keys, gk)] = g_P.reshape(-1)
    ov[np.searchsorted(keys, ok)] = o_P.reshape(-1)
    return float(np.abs(gv - ov).max()) if keys.size else 0.0


def union_dP_sym(N, g_csr, o_csr, exclude_pairs=None):
    """max of 2N |p_ij(gpu) - p_ij(oracle)| over the union of the two CSR
    patterns, absent entries counting as 0; keys i*N + j listed in
    exclude_pairs are skipped."""
    def keys(csr):
        rp, col, val = csr
        rows = np.repeat(np.arange(N, dtype=np.int64), np.diff(np.asarray(rp)))
        return rows * N + np.asarray(col, np.int64), np.asarray(val, np.float64)

    gk, gv0 = keys(g_csr)
    okk, ov0 = keys(o_csr)
    allk = np.union1d(gk, okk)
    gv = np.zeros(allk.shape)
    ov = np.zeros(allk.shape)
    gv[np.searchsorted(allk, gk)] = gv0
    ov[np.searchsorted(allk, okk)] = ov0
    d = np.abs(gv - ov) * 2 * N
    if exclude_pairs is not None and len(exclude_pairs):
        d = d[~np.isin(allk, np.asarray(exclude_pairs, np.int64))]
    return float(d.max()) if d.size else 0.0


def check_knn(X, rows, g_idx, g_d2, o_idx, o_d2, o_next, rel=TIE_REL, d2_rel=D2_REL):
    """Assert the GPU kNN rows satisfy the set rule; returns (n_tie_rows, n_exact_rows)."""
    rows = np.asarray(rows)
    M, K = o_idx.shape
    assert g_idx.shape == (M, K)
    assert np.all((g_idx >= 0) & (g_idx < X.shape[0]))
    assert not np.any(g_idx == rows[:, None]), "self returned as neighbour"
    td = true_d2(X, rows, g_idx)
    dK = o_d2[:, K - 1]
    ties = 0
    for r in range(M):
        S = g_idx[r]
        assert len(set(S.tolist())) == K, "duplicate neighbour in row %d" % r
        A = o_idx[r][o_d2[r] < dK[r] * (1 - rel)]
        assert set(A.tolist()) <= set(S.tolist()), "row %d misses a certain neighbour" % rows[r]
        assert np.all(td[r] <= dK[r] * (1 + rel)), "row %d has a non-neighbour" % rows[r]
        if o_next[r] <= dK[r] * (1 + rel):
            ties += 1
        else:
            assert set(S.tolist()) == set(o_idx[r].tolist())
    # distances: FP32 direct difference close to FP64, ascending
    err = np.abs(g_d2.astype(np.float64) - td)
    assert np.all(err <= d2_rel * np.maximum(td, 1e-30) + 1e-30), "max rel d2 error %g" % (
        (err / np.maximum(td, 1e-30)).max())
    assert np.all(np.diff(g_d2, axis=1) >= 0), "distances not ascending"
    return ties, M - ties


def check_p_rows(g_idx, g_P, o_idx, o_P, o_d2, o_next, rel=TIE_REL, tol=P_TOL):
    """Compare conditional rows: by index where the set is exact, by distance
    rank where the tie rule applied.  Returns max |dP|."""
    M, K = o_idx.shape
    worst = 0.0
    dK = o_d2[:, K - 1]
    for r in range(M):
        if o_next[r] > dK[r] * (1 + rel):
            gm = dict(zip(g_idx[r].tolist(), g_P[r].tolist()))
            ov = np.array([gm[j] for j in o_idx[r].tolist()])
            e = np.abs(ov - o_P[r]).max()
        else:
            e = np.abs(np.sort(g_P[r])[::-1] - np.sort(o_P[r])[::-1]).max()
        worst = max(worst, e)
    assert worst <= tol, "max |dP| = %g" % worst
    return worst


def perplexity_of_rows(P: np.ndarray) -> np.ndarray:
    P = P.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        H = -np.where(P > 0, P * np.log(P), 0.0).sum(1)
    return np.exp(H)


def csr_to_dict(row_ptr, col, val, rows=None):
    out = {}
    rng = range(len(row_ptr) - 1) if rows is None else rows
    for i in rng:
        for t in range(row_ptr[i], row_ptr[i + 1]):
            out[(i, int(col[t]))] = float(val[t])
    return out
