"""The GPU's reading of the cluster-pruned search's candidate set.

The oracle (oracle/ivf.py) defines a point's candidates as the rows of its
cluster's candidate clusters.  The matrix-core tile kernel works on whole
256-row tiles of the cluster-sorted corpus, so the library searches the rows
of every tile that overlaps those clusters: a superset of the candidates.
Its result is then the exact kNN over that superset, which can only be as
close or closer at every rank than the oracle's over the candidates.  This
helper spells the rounding out for the tests; it is not part of the oracle.
"""
from __future__ import annotations

import numpy as np

from oracle import ivf as IV
from oracle import oracle as O

TILE = 256  # rows per key tile of the library's contraction kernel


def tile_rounded_rows(start, clusters, N):
    """Per cluster, the sorted-corpus rows of the tiles overlapping its candidate clusters."""
    out = []
    for chosen in clusters:
        tiles = set()
        for p in chosen:
            lo, hi = int(start[p]), int(start[p + 1])
            if hi > lo:
                tiles.update(range(lo // TILE, (hi - 1) // TILE + 1))
        rows = [r for t in sorted(tiles) for r in range(t * TILE, min(N, (t + 1) * TILE))]
        out.append(np.array(rows, np.int64))
    return out


def search_tile_rounded(X, K, assign, C, probe, n_probe, rows=None):
    """Exact kNN of each point over the tile-rounded candidates (the library's reading)."""
    N = X.shape[0]
    assign = np.asarray(assign)
    perm, start = IV.cluster_order(assign, C)
    clusters = IV.candidate_clusters(start, np.asarray(probe), n_probe, K)
    cover = tile_rounded_rows(start, clusters, N)
    rows = np.arange(N, dtype=np.int32) if rows is None else np.asarray(rows, np.int32)
    ptr, cand = [0], []
    for i in rows:
        cand.extend(perm[cover[assign[i]]].tolist())
        ptr.append(len(cand))
    idx, d2, nxt = O.get().knn_candidates(X, K, rows, np.array(ptr), np.array(cand, np.int32))
    return idx, d2, nxt, np.diff(np.array(ptr))
