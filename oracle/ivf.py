"""Cluster-pruned search: the precision-controlled approximate kNN --
TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module; the GPU library never does, and
the two share no code.  The paper reaches a requested precision rho (Eq. 9)
with a randomized kd-forest whose parameters are fitted to rho (Sec. 4.2).
The GPU path reaches it with a cluster-pruned brute-force search instead,
and this module holds that search's definition, step by step, in FP64:

  lloyd_update(X, assign, prev)  k-means update: each centroid is the mean of
                                 its members; an empty cluster keeps its centroid.
  nearest_centroid(X, cent)      k-means assignment: the nearest centroid by
                                 (squared distance, index).
  cluster_order(assign, C)       the corpus sorted by (cluster, index): the
                                 permutation and each cluster's row range.
  probe_order(cent)              per cluster, all clusters by (distance
                                 between centroids, index), itself first.
  candidate_clusters(start, probe, n_probe, K)
                                 per cluster, its first n_probe probe
                                 clusters, extended with further probe
                                 clusters until their rows number at least
                                 K + 1.  A point's candidates are the rows of
                                 its own cluster's candidate clusters.
  search(X, K, assign, C, cent, n_probe)
                                 exact kNN of every point over its candidates.
  precision(approx, exact)       Eq. 9: mean over rows of |N^A_i & N_i| / K.

Parity status: pinned by ``tests/test_oracle_ivf.py`` (reduction to plain
kNN, brute force on small inputs, scipy distances, hand examples, the k-means
objective never increasing, precision never falling as candidates grow).
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

def sqdist(A, B):
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    out = np.empty((A.shape[0], B.shape[0]))
    step = max(1, (1 << 22) // max(1, B.shape[0] * A.shape[1]))
    for s in range(0, A.shape[0], step):
        diff = A[s:s + step, None, :] - B[None, :, :]
        out[s:s + step] = np.einsum("rbd,rbd->rb", diff, diff)
    return out


def lloyd_update(X, assign, prev):
    X = np.asarray(X, np.float64)
    cent = np.array(prev, np.float64, copy=True)
    for c in range(cent.shape[0]):
        mem = np.flatnonzero(assign == c)
        if mem.size:
            cent[c] = X[mem].mean(axis=0)
    return cent


def nearest_centroid(X, cent):
    D = sqdist(X, cent)
    # ties by the lower centroid index: argmin returns the first minimum
    return np.argmin(D, axis=1).astype(np.int32)


def cluster_order(assign, C):
    assign = np.asarray(assign, np.int64)
    perm = np.lexsort((np.arange(assign.size), assign)).astype(np.int32)
    counts = np.bincount(assign, minlength=C)
    start = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return perm, start


def probe_order(cent):
    D = sqdist(cent, cent)
    C = D.shape[0]
    out = np.empty((C, C), np.int32)
    for c in range(C):
        key = D[c].copy()
        key[c] = -1.0  # itself first
        out[c] = np.lexsort((np.arange(C), key))
    return out


def candidate_clusters(start, probe, n_probe, K):
    """Per cluster, the probe clusters whose rows are its points' candidates:
    the first n_probe of its probe order, then further ones until their rows
    number at least K + 1 (an empty cluster counts towards n_probe)."""
    probe = np.asarray(probe)
    out = []
    for c in range(probe.shape[0]):
        chosen, rows = [], 0
        for p in probe[c]:
            if len(chosen) >= n_probe and rows >= K + 1:
                break
            chosen.append(int(p))
            rows += int(start[p + 1]) - int(start[p])
        out.append(chosen)
    return out


def search(X, K, assign, C, cent, n_probe, oracle=None, probe=None, rows=None):
    """Approximate kNN of the points `rows` (default: all; original ids); also
    returns each row's candidate count.  `probe` overrides the probe order
    computed from `cent` (the partition is an input of the search)."""
    ora = oracle or O.get()
    N = X.shape[0]
    assign = np.asarray(assign)
    perm, start = cluster_order(assign, C)
    clusters = candidate_clusters(start, probe_order(cent) if probe is None else np.asarray(probe), n_probe, K)
    rows = np.arange(N, dtype=np.int32) if rows is None else np.asarray(rows, np.int32)
    ptr = [0]
    cand = []
    for i in rows:
        for p in clusters[assign[i]]:
            cand.extend(perm[start[p]:start[p + 1]].tolist())
        ptr.append(len(cand))
    idx, d2, nxt = ora.knn_candidates(X, K, rows, np.array(ptr), np.array(cand, np.int32))
    return idx, d2, nxt, np.diff(np.array(ptr))


def precision(approx, exact):
    """Eq. 9 over all rows (the validated recall of the oracle)."""
    return O.recall(approx, exact)
