"""Pins of the FP64 model of Sec. 5.3 (insertion by Eq. 13, deletion without
replacement) and of calibration over listed neighbours only.

Each pin checks the model against something other than itself: brute-force
kNN of the grown corpus, set algebra on the initial lists, or a from-scratch
recomputation of every row's list after each operation ("the nearest c_i of
everything the row has been offered and that is still alive", which the
incremental rules of Sec. 5.3 must reproduce).  Planted mistakes in the model
must fail at least one pin.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import serve_model as SM
from paper_1512_01655_amd import datagen


def _data(n=360, d=6, seed=5):
    return datagen.mixture_isotropic(n=n, d=d, seed=seed)


def _bruteforce_lists(X, alive, rows, K):
    """Exact K nearest live points of each row (FP64, key (d, j))."""
    live = np.flatnonzero(alive)
    D = SM.sqdist(X[rows], X[live])
    out = []
    for t, i in enumerate(rows):
        keys = sorted((D[t, s], int(j)) for s, j in enumerate(live) if j != i)
        out.append([j for _, j in keys[:K]])
    return out


def _recompute(X, K, ops, n0):
    """Replay ops from scratch: per row, the offered set S_i and the count c_i.

    A row is created with its exact K nearest live points; an insert offers
    the batch to every live row; a delete lowers c_i by the number of deleted
    points among the row's current nearest c_i of S_i and removes them from
    S_i.  The row's list is then the nearest c_i of S_i by (d, j)."""
    Xall = X
    n = n0
    alive = np.zeros(X.shape[0], bool)
    alive[:n0] = True
    S = {}
    c = {}

    def nearest(i, cnt):
        if cnt == 0 or not S[i]:
            return []
        js = np.array(sorted(S[i]), np.int64)
        d = SM.sqdist(Xall[i:i + 1], Xall[js])[0]
        keys = sorted(zip(d.tolist(), js.tolist()))
        return [j for _, j in keys[:cnt]]

    for i, lst in zip(range(n0), _bruteforce_lists(Xall[:n0], alive[:n0], np.arange(n0), K)):
        S[i] = set(lst)
        c[i] = K
    for op in ops:
        if op[0] == "i":
            B = op[1]
            new = list(range(n, n + B))
            alive[n:n + B] = True
            for i in list(S):
                if alive[i]:
                    S[i] |= set(new)
            lists = _bruteforce_lists(Xall[:n + B], alive[:n + B], np.array(new), K)
            for i, lst in zip(new, lists):
                S[i] = set(lst)
                c[i] = K
            n += B
        else:
            ids = set(int(v) for v in op[1])
            for i in list(S):
                if not alive[i] or i in ids:
                    continue
                cur = nearest(i, c[i])
                c[i] -= len(ids.intersection(cur))
                S[i] -= ids
            for v in ids:
                alive[v] = False
                S[v] = set()
                c[v] = 0
    return {i: nearest(i, c[i]) for i in S}, c, alive[:n]


def _sequence(X0, seed, mutant=0, n_new=160):
    """A mixed insert/delete sequence on the model; returns (model, ops, Xall)."""
    rng = np.random.default_rng(seed)
    pts = datagen.mixture_isotropic(n=n_new, d=X0.shape[1], seed=seed + 100)
    m = SM.ResidentModel(X0, 4.0, mutant=mutant)
    ops = []
    off = 0
    for B, n_del in [(5, 12), (40, 3), (1, 30), (0, 25), (70, 0), (20, 40), (24, 9)]:
        if B:
            m.insert(pts[off:off + B])
            ops.append(("i", B))
            off += B
        if n_del:
            live = np.flatnonzero(m.alive)
            ids = rng.choice(live, size=n_del, replace=False).astype(np.int32)
            m.delete(ids)
            ops.append(("d", ids))
    return m, ops, np.concatenate([X0, pts[:off]])


def _assert_matches_recompute(m, ops, Xall, n0):
    lists, c, alive = _recompute(Xall, m.K, ops, n0)
    assert np.array_equal(m.alive, alive), "alive flags differ"
    for i in range(m.n_rows()):
        if i in m.tie_rows:
            continue
        got = [int(j) for j in m.idx[i] if j >= 0]
        assert got == lists[i], "row %d: %s vs recomputed %s" % (i, got[:6], lists[i][:6])
        assert m.present()[i] == c[i]
    assert np.allclose(m.rho(), np.array([c[i] for i in range(m.n_rows())]) / m.K)


def test_insert_only_is_exact_knn_of_grown_corpus():
    X0 = _data()
    m = SM.ResidentModel(X0, 4.0)
    pts = datagen.mixture_isotropic(n=120, d=6, seed=9)
    off = 0
    for B in (1, 7, 40, 72):
        m.insert(pts[off:off + B])
        off += B
    Xall = np.concatenate([X0, pts[:off]])
    o_idx, o_d2, o_nx = O.get().knn(Xall, m.K)
    assert m.present().min() == m.K
    bad = [i for i in range(m.n_rows()) if i not in m.tie_rows and not np.array_equal(m.idx[i], o_idx[i])]
    assert not bad, "rows differ from brute force: %s" % bad[:10]
    assert np.allclose(m.d2, o_d2, rtol=1e-13, atol=0)  # summation order differs


def test_delete_only_removes_without_replacement():
    X0 = _data(seed=6)
    m = SM.ResidentModel(X0, 4.0)
    init = m.idx.copy()
    rng = np.random.default_rng(1)
    dead = set()
    for n_del in (1, 17, 60):
        ids = rng.choice(np.flatnonzero(m.alive), size=n_del, replace=False).astype(np.int32)
        changed = m.delete(ids)
        dead |= set(ids.tolist())
        exp_changed = [i for i in range(m.n_rows()) if i not in dead and set(ids.tolist()) & set(init[i].tolist())]
        assert changed.tolist() == sorted(exp_changed)
    for i in range(m.n_rows()):
        if i in dead:
            assert np.all(m.idx[i] == -1) and np.all(np.isinf(m.d2[i])) and m.rho()[i] == 0.0
            continue
        want = [j for j in init[i].tolist() if j not in dead]
        got = m.idx[i][m.idx[i] >= 0].tolist()
        assert got == want
        assert m.rho()[i] == pytest.approx(1.0 - (m.K - len(want)) / m.K)
        assert np.all(m.idx[i][len(want):] == -1) and np.all(np.isinf(m.d2[i][len(want):]))


def test_mixed_sequence_matches_recomputation():
    X0 = _data(seed=7)
    m, ops, Xall = _sequence(X0, 3)
    assert m.present().min() < m.K  # holes exist, some of them were offered new points
    _assert_matches_recompute(m, ops, Xall, X0.shape[0])


@pytest.mark.parametrize("mutant", [1, 2, 3, 4])
def test_planted_model_mistakes_fail_a_pin(mutant):
    X0 = _data(seed=7)
    m, ops, Xall = _sequence(X0, 3, mutant=mutant)
    with pytest.raises(AssertionError):
        _assert_matches_recompute(m, ops, Xall, X0.shape[0])


def test_calibrate_absent_rows():
    rng = np.random.default_rng(4)
    K, mu = 30, 6.0
    d2 = np.sort(rng.gamma(2.0, 1.0, size=(40, K)), axis=1)
    holes = [0, 1, 5, 6, 24, 29, 30]  # present entries per row for the first rows
    for r, c in enumerate(holes):
        d2[r, c:] = np.inf
    P, beta, flags = SM.calibrate_absent(d2, mu)
    present = np.isfinite(d2)
    assert np.all(P[~present] == 0.0)
    for r in range(d2.shape[0]):
        c = int(present[r].sum())
        if c == 0:
            assert flags[r] & SM.FLAG_DEGENERATE and np.all(P[r] == 0)
            continue
        p = P[r][present[r]]
        assert abs(p.sum() - 1.0) < 1e-12
        if c <= mu:
            assert flags[r] & SM.FLAG_DEGENERATE and np.allclose(p, 1.0 / c)
            continue
        # closed form of the returned beta: p_j = exp(-beta d_j) / Z, e^H = mu
        d = d2[r][present[r]]
        w = np.exp(-beta[r] * (d - d.min()))
        assert np.allclose(p, w / w.sum(), rtol=1e-12, atol=0)
        H = -(p * np.log(p)).sum()
        assert abs(math.exp(H) - mu) < 1e-8
    # absent entries anywhere in the row give the same calibration
    r = 3
    perm = rng.permutation(K)
    P2, b2, _ = SM.calibrate_absent(d2[r:r + 1, perm], mu)
    assert np.allclose(P2[0], P[r, perm], rtol=1e-13, atol=0) and b2[0] == pytest.approx(beta[r], rel=1e-13)
