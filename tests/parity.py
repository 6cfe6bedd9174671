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
    """FP64 squared distances from X[rows[r]] to X[idx[r, t]]."""
    X64 = X.astype(np.float64)
    out = np.empty(idx.shape, np.float64)
    for s in range(0, len(rows), 256):
        e = min(len(rows), s + 256)
        diff = X64[rows[s:e], None, :] - X64[idx[s:e]]
        out[s:e] = np.einsum("rkd,rkd->rk", diff, diff)
    return out


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
