"""Refinement orderings of Sec. 5.1 -- TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module; the GPU library never does, and
the two share no code.  Plain textbook algorithms in FP64:

  density_order(beta, ids)      Density-based refinement: points of sparse
                                regions first, i.e. sigma_i descending
                                (sigma_i = 1/sqrt(2 beta_i), so beta_i
                                ascending), ties by index.
  bfs_levels(nbr_idx, seeds)    Breadth-first visit of the graph of the kNN
                                relationships from the user selection: the
                                hop count from the nearest seed along edges
                                i -> j, j in N_i.
  path_lengths(nbr_idx, nbr_d2, seeds)
                                The same visit driven by a priority queue
                                keyed on high-dimensional distance: the
                                shortest path length from the selection with
                                edge weight ||x_i - x_j|| (Dijkstra).
  order_by_key(key)             Reached points sorted by (key, index).

Readings taken (the paper names the strategies but not their details):
  * the graph is directed (i -> j for j in N_i), as the KNN lists define it;
    absent entries (index -1) carry no edge;
  * the priority is the accumulated high-dimensional path length from the
    selection, so the order is unique up to equal keys, which are broken by
    index;
  * density order sorts by sigma_i, the bandwidth of Eq. 3, not by a
    separate density estimate.

``mutant`` > 0 plants one deliberate mistake so the pins can show they catch
it: 1 treats the graph as undirected, 2 weights edges by squared distance,
3 reverses the density order.

Parity status: pinned by ``tests/test_oracle_refine_order.py`` (scipy's
csgraph shortest paths, hand graphs, invariants).
"""
from __future__ import annotations

import heapq
import math
from collections import deque

import numpy as np


def density_order(beta, ids=None, mutant: int = 0) -> np.ndarray:
    beta = np.asarray(beta, np.float64)
    ids = np.arange(beta.shape[0], dtype=np.int64) if ids is None else np.asarray(ids, np.int64)
    with np.errstate(divide="ignore"):
        sigma = 1.0 / np.sqrt(2.0 * beta[ids])  # +inf for beta = 0, 0 for beta = +inf
    key = sigma if mutant == 3 else -sigma
    # lexsort: last key is primary
    return ids[np.lexsort((ids, key))].astype(np.int32)


def _edges(nbr_idx, mutant):
    N, k = nbr_idx.shape
    adj = [[] for _ in range(N)]
    for i in range(N):
        for s in range(k):
            j = int(nbr_idx[i, s])
            if j >= 0:
                adj[i].append((j, s))
                if mutant == 1:
                    adj[j].append((i, -1 - s))
    return adj


def bfs_levels(nbr_idx, seeds, max_depth: int = -1, mutant: int = 0) -> np.ndarray:
    nbr_idx = np.asarray(nbr_idx)
    N = nbr_idx.shape[0]
    adj = _edges(nbr_idx, mutant)
    level = np.full(N, -1, np.int64)
    q = deque()
    for s in seeds:
        if level[s] < 0:
            level[s] = 0
            q.append(int(s))
    while q:
        i = q.popleft()
        if max_depth >= 0 and level[i] >= max_depth:
            continue
        for j, _ in adj[i]:
            if level[j] < 0:
                level[j] = level[i] + 1
                q.append(j)
    return level


def path_lengths(nbr_idx, nbr_d2, seeds, mutant: int = 0) -> np.ndarray:
    nbr_idx = np.asarray(nbr_idx)
    d2 = np.asarray(nbr_d2, np.float64)
    N = nbr_idx.shape[0]
    adj = _edges(nbr_idx, mutant)
    dist = np.full(N, math.inf)
    heap = []
    for s in seeds:
        if dist[s] > 0:
            dist[s] = 0.0
            heap.append((0.0, int(s)))
    heapq.heapify(heap)
    while heap:
        d, i = heapq.heappop(heap)
        if d > dist[i]:
            continue
        for j, s in adj[i]:
            w2 = d2[i, s] if s >= 0 else d2[j, -1 - s]
            w = w2 if mutant == 2 else math.sqrt(w2)
            if d + w < dist[j]:
                dist[j] = d + w
                heapq.heappush(heap, (d + w, j))
    return dist


def order_by_key(key) -> np.ndarray:
    """Indices with a reached key (finite, >= 0), sorted by (key, index)."""
    key = np.asarray(key, np.float64)
    ids = np.flatnonzero(np.isfinite(key) & (key >= 0))
    return ids[np.lexsort((ids, key[ids]))].astype(np.int32)
