"""Pins of the cluster-pruned search's definition (oracle/ivf.py) and of the
candidate-restricted kNN in the C oracle."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import ivf as IV
from oracle import oracle as O
from paper_1512_01655_amd import datagen
from tests import ivf_reading as RD


def test_candidates_all_rows_is_plain_knn():
    X = datagen.mixture_isotropic(n=300, d=7, seed=71)
    N = X.shape[0]
    q = np.arange(N, dtype=np.int32)
    ptr = np.arange(0, N * N + 1, N, dtype=np.int64)
    cand = np.tile(np.arange(N, dtype=np.int32), N)
    a = O.get().knn_candidates(X, 9, q, ptr, cand)
    b = O.get().knn(X, 9)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_candidates_brute_force_subsets():
    rng = np.random.default_rng(2)
    X = rng.integers(-3, 4, size=(60, 3)).astype(np.float32)  # integer coordinates: exact ties
    q = rng.choice(60, size=20, replace=False).astype(np.int32)
    ptr, cand = [0], []
    for i in q:
        c = rng.choice(60, size=int(rng.integers(3, 40)), replace=False)
        cand += c.tolist()
        ptr.append(len(cand))
    K = 5
    idx, d2, nxt = O.get().knn_candidates(X, K, q, np.array(ptr), np.array(cand, np.int32))
    for m, i in enumerate(q):
        c = [j for j in cand[ptr[m]:ptr[m + 1]] if j != i]
        d = [int(((X[i].astype(int) - X[j].astype(int)) ** 2).sum()) for j in c]
        keys = sorted(zip(d, c))
        want = [j for _, j in keys[:K]] + [-1] * max(0, K - len(keys))
        assert idx[m].tolist() == want
        assert np.all(np.isinf(d2[m][len(keys):]))
        assert nxt[m] == (keys[K][0] if len(keys) > K else np.inf)


def test_nearest_centroid_against_scipy():
    X = datagen.mixture_isotropic(n=500, d=12, seed=72)
    cent = X[np.random.default_rng(1).choice(500, size=17, replace=False)].astype(np.float64)
    a = IV.nearest_centroid(X, cent)
    D = cdist(X.astype(np.float64), cent, "sqeuclidean")
    assert np.array_equal(a, np.argmin(D, axis=1))
    # ties go to the lower centroid index
    Xt = np.array([[0.0, 0.0]], np.float32)
    assert IV.nearest_centroid(Xt, np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])).tolist() == [0]


def test_lloyd_update_hand_and_objective():
    X = np.array([[0, 0], [2, 0], [0, 2], [10, 10], [12, 10]], np.float32)
    cent = IV.lloyd_update(X, np.array([0, 0, 0, 1, 1]), np.zeros((3, 2)) + 7.0)
    assert np.allclose(cent, [[2 / 3, 2 / 3], [11, 10], [7, 7]])  # empty cluster 2 keeps its centroid
    # Lloyd's alternation never increases the objective
    X = datagen.mixture_isotropic(n=800, d=10, seed=73)
    cent = X[:20].astype(np.float64)
    prev = np.inf
    for _ in range(6):
        a = IV.nearest_centroid(X, cent)
        obj = ((X.astype(np.float64) - cent[a]) ** 2).sum()
        assert obj <= prev * (1 + 1e-12)
        prev = obj
        cent = IV.lloyd_update(X, a, cent)


def test_cluster_order_and_probe_order():
    assign = np.array([2, 0, 2, 1, 0, 2])
    perm, start = IV.cluster_order(assign, 4)
    assert perm.tolist() == [1, 4, 3, 0, 2, 5] and start.tolist() == [0, 2, 3, 6, 6]
    cent = np.array([[0.0], [1.0], [5.0], [-1.0]])
    po = IV.probe_order(cent)
    assert po[0].tolist() == [0, 1, 3, 2]  # ties (1 and 3 at distance 1) by index
    assert po[2].tolist() == [2, 1, 0, 3]


def test_candidate_clusters_hand():
    start = np.array([0, 100, 300, 700, 700, 1000])
    probe = np.array([[0, 1, 2, 3, 4], [1, 0, 2, 3, 4], [2, 4, 1, 0, 3], [3, 2, 4, 1, 0], [4, 3, 2, 1, 0]])
    c = IV.candidate_clusters(start, probe, 1, 10)
    assert c == [[0], [1], [2], [3, 2], [4]]  # cluster 3 is empty: probing extends to cluster 2
    # the K + 1 rule counts cluster rows: 100 and 100 + 200 rows are short of 301
    assert IV.candidate_clusters(start, probe, 1, 300)[0] == [0, 1, 2]
    assert IV.candidate_clusters(start, probe, 2, 10)[0] == [0, 1]
    assert IV.candidate_clusters(start, probe, 5, 10)[2] == [2, 4, 1, 0, 3]


def test_tile_rounding_is_a_superset():
    # the library's reading (whole 256-row tiles) covers every candidate row
    start = np.array([0, 100, 300, 700, 700, 1000])
    probe = np.array([[0, 1, 2, 3, 4], [1, 0, 2, 3, 4], [2, 4, 1, 0, 3], [3, 2, 4, 1, 0], [4, 3, 2, 1, 0]])
    cover = RD.tile_rounded_rows(start, IV.candidate_clusters(start, probe, 1, 10), 1000)
    assert cover[0].tolist() == list(range(256)) and cover[4].tolist() == list(range(512, 1000))
    rng = np.random.default_rng(9)
    for trial in range(20):
        C = int(rng.integers(2, 40))
        N = int(rng.integers(C, 3000))
        assign = rng.integers(0, C, size=N)
        _, st = IV.cluster_order(assign, C)
        pr = np.array([np.concatenate([[c], rng.permutation(np.delete(np.arange(C), c))]) for c in range(C)])
        for n_probe in (1, 2, C):
            cl = IV.candidate_clusters(st, pr, n_probe, 10)
            cov = RD.tile_rounded_rows(st, cl, N)
            for c in range(C):
                rows = np.concatenate([np.arange(st[p], st[p + 1]) for p in cl[c]])
                assert set(rows.tolist()) <= set(cov[c].tolist())
                assert len(rows) >= min(11, N)


def test_precision_grows_with_candidates():
    # a superset of candidates gives each row at least the hits of a subset
    # (Eq. 9 counts exact neighbours found; an exact neighbour among the
    # candidates is always among their K nearest)
    X = datagen.mixture_isotropic(n=600, d=8, seed=75)
    rng = np.random.default_rng(6)
    C = 8
    cent = X[rng.choice(600, size=C, replace=False)].astype(np.float64)
    a = IV.nearest_centroid(X, cent)
    probe = IV.probe_order(cent)
    e_idx, _, _ = O.get().knn(X, 10)
    sub = IV.search(X, 10, a, C, cent, 1)[0]
    sup = RD.search_tile_rounded(X, 10, a, C, probe, 1)[0]
    for r in range(600):
        hs = len(set(sub[r].tolist()) & set(e_idx[r].tolist()))
        hp = len(set(sup[r].tolist()) & set(e_idx[r].tolist()))
        assert hp >= hs


def test_search_reduces_to_exact_with_all_probes():
    X = datagen.mixture_isotropic(n=700, d=9, seed=74)
    rng = np.random.default_rng(5)
    C = 6
    cent = X[rng.choice(700, size=C, replace=False)].astype(np.float64)
    a = IV.nearest_centroid(X, cent)
    idx, d2, nxt, ncand = IV.search(X, 10, a, C, cent, C)
    e_idx, e_d2, _ = O.get().knn(X, 10)
    assert np.array_equal(idx, e_idx) and IV.precision(idx, e_idx) == 1.0
    idx1, _, _, n1 = IV.search(X, 10, a, C, cent, 1)
    assert np.all(n1 <= ncand) and IV.precision(idx1, e_idx) <= 1.0
    # Eq. 9 by hand
    assert IV.precision(np.array([[1, 2, 3], [4, 5, -1]]), np.array([[3, 2, 9], [6, 5, 4]])) == pytest.approx(4 / 6)
    with pytest.raises(ValueError):
        IV.precision(np.array([[1, 1, 3]]), np.array([[1, 2, 3]]))
