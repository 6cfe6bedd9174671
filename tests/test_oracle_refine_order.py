"""Pins of the refinement-ordering oracle (Sec. 5.1): scipy's csgraph
shortest paths as an independent library, hand graphs, invariants, and
planted mistakes that must fail."""
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra, shortest_path

from oracle import oracle as O
from oracle import refine_order as RO
from paper_1512_01655_amd import datagen


def _graph(seed=3, n=400, d=8, k=6):
    X = datagen.mixture_isotropic(n=n, d=d, seed=seed)
    idx, d2, _ = O.get().knn(X, k)
    return X, idx, d2


def _csr(idx, w):
    N, k = idx.shape
    rows = np.repeat(np.arange(N), k)
    m = idx.reshape(-1) >= 0
    return csr_matrix((w.reshape(-1)[m], (rows[m], idx.reshape(-1)[m])), shape=(N, N))


def pin_bfs_scipy(mutant=0):
    _, idx, d2 = _graph()
    seeds = np.array([5, 17, 301])
    lv = RO.bfs_levels(idx, seeds, mutant=mutant)
    ref = shortest_path(_csr(idx, np.ones(idx.shape)), unweighted=True, directed=True, indices=seeds).min(axis=0)
    assert np.array_equal(np.where(lv < 0, np.inf, lv), ref)


def pin_bfs_hand(mutant=0):
    # chain 0 -> 1 -> 2 -> 3, with 4 -> 0 (nothing points to 4) and 5 isolated
    idx = np.array([[1], [2], [3], [-1], [0], [-1]])
    lv = RO.bfs_levels(idx, [0], mutant=mutant)
    assert lv.tolist() == [0, 1, 2, 3, -1, -1]
    assert RO.bfs_levels(idx, [0], max_depth=2, mutant=mutant).tolist() == [0, 1, 2, -1, -1, -1]
    assert RO.order_by_key(lv).tolist() == [0, 1, 2, 3]


def pin_paths_scipy(mutant=0):
    _, idx, d2 = _graph(seed=4)
    idx = idx.copy()
    idx[::7, -1] = -1  # absent entries carry no edge
    seeds = np.array([0, 222])
    dist = RO.path_lengths(idx, d2, seeds, mutant=mutant)
    ref = dijkstra(_csr(idx, np.sqrt(d2)), directed=True, indices=seeds, min_only=True)
    assert np.allclose(dist, ref, rtol=1e-12, atol=0) and np.array_equal(np.isinf(dist), np.isinf(ref))


def pin_paths_invariants(mutant=0):
    _, idx, d2 = _graph(seed=5)
    seeds = [9]
    dist = RO.path_lengths(idx, d2, seeds, mutant=mutant)
    N, k = idx.shape
    for i in range(N):
        if not np.isfinite(dist[i]):
            continue
        for s in range(k):
            j = idx[i, s]
            assert dist[j] <= dist[i] + math.sqrt(d2[i, s]) * (1 + 1e-12)  # no edge relaxes further
    for j in range(N):
        if j in seeds or not np.isfinite(dist[j]):
            continue
        tight = [abs(dist[i] + math.sqrt(d2[i, s]) - dist[j]) <= 1e-12 * dist[j]
                 for i in range(N) for s in range(k) if idx[i, s] == j and np.isfinite(dist[i])]
        assert any(tight), "point %d has no tight predecessor" % j


def pin_density_hand(mutant=0):
    # points on a line: a dense run of 12 and three isolated points; the
    # isolated points have the widest Gaussians and come first
    X = np.concatenate([np.arange(12) * 0.1, [5.0, 9.0, 14.0]]).reshape(-1, 1).astype(np.float32)
    idx, d2, _ = O.get().knn(X, 6)
    _, beta, _, _ = O.get().calibrate(d2, 2.0)
    order = RO.density_order(beta, mutant=mutant)
    assert set(order[:3].tolist()) == {12, 13, 14}
    sig = 1.0 / np.sqrt(2.0 * beta[order])
    assert np.all(np.diff(sig) <= 0)


def pin_density_ties_and_selection(mutant=0):
    beta = np.array([2.0, 1.0, 2.0, 0.5, 1.0, np.inf, 0.0])
    assert RO.density_order(beta, mutant=mutant).tolist() == [6, 3, 1, 4, 0, 2, 5]
    assert RO.density_order(beta, ids=[5, 4, 2, 1], mutant=mutant).tolist() == [1, 4, 2, 5]


PINS = [pin_bfs_scipy, pin_bfs_hand, pin_paths_scipy, pin_paths_invariants, pin_density_hand,
        pin_density_ties_and_selection]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_refine_order_pin(pin):
    pin()


@pytest.mark.parametrize("mutant", [1, 2, 3])
def test_planted_order_mistakes_fail_a_pin(mutant):
    caught = []
    for pin in PINS:
        try:
            pin(mutant)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, "mutant %d slipped past every pin" % mutant
