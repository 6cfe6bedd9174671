"""Pins for the FP64 oracle: checks against what the paper and mathematics fix.

Each pin takes an ``oracle.Oracle`` handle and raises AssertionError on a
mismatch.  They are run against the real oracle (tests/test_oracle_*.py) and
against builds with a planted mistake (tests/test_oracle_mutants.py), which
every mutant must fail.  None of them re-types the oracle's code: they use
exact rational brute force, closed forms solved by mpmath, an independent
library (scikit-learn), invariants and metamorphic relations.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath as mp
import numpy as np

# --------------------------------------------------------------------------
# kNN  (Eq. 3 squared Euclidean distance; Eq. 8 neighbour set; tie rule (d, j))
# --------------------------------------------------------------------------


def pin_knn_exact_rational(o, seed: int = 5):
    """Brute force in exact rationals on tiny inputs with many exact ties."""
    rng = np.random.default_rng(seed)
    for N, D, K in [(12, 2, 3), (25, 3, 7), (40, 1, 10), (33, 4, 32), (9, 5, 8)]:
        Xq = rng.integers(-6, 7, size=(N, D))  # quarters: exactly representable
        X = (Xq / 4.0).astype(np.float32)
        idx, d2, nxt = o.knn(X, K)
        for i in range(N):
            keys = []
            for j in range(N):
                if j == i:
                    continue
                s = sum((Fraction(int(Xq[i, d]), 4) - Fraction(int(Xq[j, d]), 4)) ** 2 for d in range(D))
                keys.append((s, j))
            keys.sort()
            assert [j for _, j in keys[:K]] == idx[i].tolist(), (N, D, K, i)
            for t in range(K):
                assert Fraction(float(d2[i, t])) == keys[t][0]
            if K < N - 1:
                assert Fraction(float(nxt[i])) == keys[K][0]
            else:
                assert np.isinf(nxt[i])


def pin_knn_line(o):
    """Points at 0,1,...,N-1 on a line: the neighbour order is i-1, i+1, i-2, i+2, ...
    (lower index first on equal distance), clipped at the ends."""
    N, K = 50, 9
    X = np.arange(N, dtype=np.float32)[:, None]
    idx, d2, _ = o.knn(X, K)
    for i in range(N):
        exp = []
        r = 1
        while len(exp) < K:
            for j in (i - r, i + r):
                if 0 <= j < N and len(exp) < K:
                    exp.append(j)
            r += 1
        assert idx[i].tolist() == exp, (i, idx[i], exp)
        assert np.array_equal(d2[i], (np.array(exp) - i) ** 2.0)


def pin_knn_sklearn(o, seed: int = 6):
    """Continuous data (no ties): scikit-learn's brute-force search agrees."""
    from sklearn.neighbors import NearestNeighbors

    rng = np.random.default_rng(seed)
    for N, D, K in [(300, 7, 20), (500, 50, 90)]:
        X = rng.normal(size=(N, D)).astype(np.float32)
        idx, d2, _ = o.knn(X, K)
        nn = NearestNeighbors(n_neighbors=K + 1, algorithm="brute").fit(X.astype(np.float64))
        dist, ind = nn.kneighbors(X.astype(np.float64))
        for i in range(N):
            sk = [j for j in ind[i] if j != i][:K]
            assert idx[i].tolist() == sk
        dd = ((X[:, None, :].astype(np.float64) - X[idx].astype(np.float64)) ** 2).sum(-1)
        assert np.allclose(d2, dd, rtol=1e-12, atol=0)


def pin_knn_metamorphic(o, seed: int = 7):
    """Translation leaves the sets unchanged; a row permutation permutes them
    (sets compared where no tie straddles the K-th place)."""
    rng = np.random.default_rng(seed)
    N, D, K = 200, 6, 15
    Xq = rng.integers(-40, 41, size=(N, D))
    X = Xq.astype(np.float32)
    idx, d2, nxt = o.knn(X, K)
    idx_t, d2_t, _ = o.knn((Xq + 1000).astype(np.float32), K)
    assert np.array_equal(idx, idx_t) and np.array_equal(d2, d2_t)
    perm = rng.permutation(N)
    idx_p, d2_p, _ = o.knn(X[perm], K)
    # row r of the permuted problem is original row perm[r]; index s maps to perm[s].
    for r in range(N):
        i = perm[r]
        assert np.array_equal(d2_p[r], d2[i])
        if d2[i, -1] < nxt[i]:
            assert set(perm[idx_p[r]].tolist()) == set(idx[i].tolist())


def pin_knn_subset(o, seed: int = 8):
    """A query subset gives the same rows as the full problem."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(150, 9)).astype(np.float32)
    idx, d2, nxt = o.knn(X, 12)
    q = rng.choice(150, size=40, replace=False).astype(np.int32)
    idx_s, d2_s, nxt_s = o.knn(X, 12, query_ids=q)
    assert np.array_equal(idx_s, idx[q]) and np.array_equal(d2_s, d2[q]) and np.array_equal(nxt_s, nxt[q])


# --------------------------------------------------------------------------
# Calibration (Eq. 3, Eq. 4 on the neighbour set of Eq. 8)
# --------------------------------------------------------------------------

mp.mp.dps = 50


def _solve_beta(H, mu, lo, hi):
    target = mp.log(mp.mpf(mu))
    f = lambda b: H(b) - target  # noqa: E731
    a, b = mp.mpf(lo), mp.mpf(hi)
    fa = f(a)
    for _ in range(400):  # exact-arithmetic bisection at 50 digits
        m = (a + b) / 2
        fm = f(m)
        if (fm > 0) == (fa > 0):
            a, fa = m, fm
        else:
            b = m
    return (a + b) / 2


def pin_calibrate_two_level(o):
    """m neighbours at delta=0 and K-m at delta=Delta: p0 = 1/(m + (K-m) e^{-beta Delta}),
    p1 = p0 e^{-beta Delta}, H = -m p0 ln p0 - (K-m) p1 ln p1."""
    for K, m, Delta, mu, off in [(90, 1, 2.5, 30.0, 7.0), (30, 3, 0.125, 10.0, 100.0), (12, 2, 40.0, 5.5, 0.0),
                                 (150, 1, 1.0, 50.0, 3.0)]:
        def H(b, K=K, m=m, Delta=Delta):
            e = mp.e ** (-b * Delta)
            p0 = 1 / (m + (K - m) * e)
            p1 = p0 * e
            return -m * p0 * mp.log(p0) - (K - m) * p1 * mp.log(p1)

        beta = _solve_beta(H, mu, 0, 1e4 / Delta)
        d2 = np.array([[off] * m + [off + Delta] * (K - m)], np.float64)
        P, b, perp, flags = o.calibrate(d2, mu)
        assert flags[0] == 0
        assert abs(b[0] - float(beta)) <= 1e-9 * float(beta), (K, m, b[0], float(beta))
        e = mp.e ** (-beta * Delta)
        p0 = float(1 / (m + (K - m) * e))
        p1 = float(e / (m + (K - m) * e))
        assert np.allclose(P[0, :m], p0, rtol=1e-10, atol=0) and np.allclose(P[0, m:], p1, rtol=1e-9, atol=1e-300)
        assert abs(perp[0] - mu) <= 1e-9 * mu


def pin_calibrate_progression(o):
    """delta_j = j*Delta (j = 0..K-1): with r = e^{-beta Delta},
    Z = (1 - r^K)/(1 - r),  E[j] = r/(1-r) - K r^K/(1 - r^K),  H = ln Z + beta Delta E[j]."""
    for K, Delta, mu in [(90, 0.05, 30.0), (30, 1.0, 10.0), (150, 0.01, 50.0), (7, 3.0, 2.0)]:
        def H(b, K=K, Delta=Delta):
            r = mp.e ** (-b * Delta)
            Z = (1 - r ** K) / (1 - r)
            Ej = r / (1 - r) - K * r ** K / (1 - r ** K)
            return mp.log(Z) + b * Delta * Ej

        beta = _solve_beta(H, mu, 1e-30, 1e4 / Delta)
        d2 = (np.arange(K, dtype=np.float64) * Delta + 11.0)[None, :]
        # shuffle the row: calibration must not depend on neighbour order
        perm = np.random.default_rng(K).permutation(K)
        P, b, perp, flags = o.calibrate(d2[:, perm], mu)
        assert flags[0] == 0
        assert abs(b[0] - float(beta)) <= 1e-9 * float(beta), (K, b[0], float(beta))
        r = mp.e ** (-beta * Delta)
        Z = (1 - r ** K) / (1 - r)
        pexp = np.array([float(r ** j / Z) for j in range(K)])[perm]
        assert np.allclose(P[0], pexp, rtol=1e-9, atol=1e-300)


def pin_calibrate_invariants(o, seed: int = 9):
    """Rows sum to one, achieved perplexity equals mu, beta decreases as mu grows."""
    rng = np.random.default_rng(seed)
    d2 = np.sort(rng.gamma(5.0, 3.0, size=(200, 90)), axis=1)
    P30, b30, perp30, f30 = o.calibrate(d2, 30.0)
    P45, b45, perp45, f45 = o.calibrate(d2, 45.0)
    assert not f30.any() and not f45.any()
    assert np.allclose(P30.sum(1), 1.0, atol=1e-12)
    assert np.allclose(perp30, 30.0, rtol=1e-10)
    assert np.allclose(perp45, 45.0, rtol=1e-10)
    H = -(P30 * np.log(P30)).sum(1)
    assert np.allclose(np.exp(H), 30.0, rtol=1e-10)
    assert np.all(b45 < b30)
    # weights follow the Gaussian of Eq. 3: p_j / p_0 = exp(-beta (d_j - d_0))
    ratio = P30 / P30[:, :1]
    assert np.allclose(ratio, np.exp(-b30[:, None] * (d2 - d2[:, :1])), rtol=1e-9)


def pin_calibrate_scaling(o, seed: int = 10):
    """Scaling X by c scales squared distances by c^2: beta -> beta/c^2, P unchanged
    (c = 2 keeps every value exact); duplicating every coordinate doubles d^2: beta/2."""
    rng = np.random.default_rng(seed)
    d2 = rng.uniform(1.0, 9.0, size=(50, 60))
    P, b, _, _ = o.calibrate(d2, 20.0)
    P4, b4, _, _ = o.calibrate(d2 * 4.0, 20.0)
    P2, b2, _, _ = o.calibrate(d2 * 2.0, 20.0)
    assert np.allclose(b4, b / 4.0, rtol=1e-12) and np.allclose(P4, P, rtol=1e-11, atol=1e-300)
    assert np.allclose(b2, b / 2.0, rtol=1e-12) and np.allclose(P2, P, rtol=1e-11, atol=1e-300)


def pin_calibrate_degenerate(o):
    """m >= mu zero-shift neighbours: the limit beta -> inf, uniform over those m.
    All neighbours equidistant: uniform 1/K, flagged."""
    d2 = np.array([[1.0] * 12 + [2.0] * 18, [3.0] * 30], np.float64)
    P, b, perp, flags = o.calibrate(d2, 10.0)
    assert flags[0] & 4 and flags[1] & 4
    assert np.allclose(P[0, :12], 1 / 12) and np.all(P[0, 12:] == 0) and np.isinf(b[0])
    assert np.allclose(P[1], 1 / 30) and abs(perp[1] - 30) < 1e-9
    assert abs(perp[0] - 12) < 1e-9


def pin_calibrate_brentq(o, seed: int = 11):
    """scipy's Brent root finder on an independently written H(beta) agrees."""
    from scipy.optimize import brentq

    rng = np.random.default_rng(seed)
    d2 = rng.uniform(0.0, 50.0, size=(20, 45))
    P, b, _, _ = o.calibrate(d2, 12.0)
    for i in range(20):
        dl = d2[i] - d2[i].min()

        def f(beta):
            lw = -beta * dl
            lZ = np.log(np.exp(lw).sum())
            p = np.exp(lw - lZ)
            return -(p * np.log(np.where(p > 0, p, 1.0))).sum() - np.log(12.0)

        r = brentq(f, 1e-12, 1e3, xtol=1e-16, rtol=1e-14, maxiter=500)
        assert abs(r - b[i]) <= 1e-9 * r


# --------------------------------------------------------------------------
# Symmetrisation (Eq. 2 / Eq. 10)
# --------------------------------------------------------------------------


def pin_symmetrize_hand(o):
    """Worked by hand from Eq. 2 for N=4, K=2 (2N = 8):
      rows (neighbours: p):  0: {1: 3/4, 2: 1/4}   1: {0: 1/2, 2: 1/2}
                             2: {3: 5/8, 1: 3/8}   3: {2: 7/8, 0: 1/8}
      p01 = (3/4 + 1/2)/8 = 5/32    p02 = (1/4 + 0)/8 = 1/32    p03 = (0 + 1/8)/8 = 1/64
      p12 = (1/2 + 3/8)/8 = 7/64    p23 = (5/8 + 7/8)/8 = 3/16  p13 = 0 (absent)
    """
    idx = np.array([[1, 2], [0, 2], [3, 1], [2, 0]], np.int32)
    P = np.array([[0.75, 0.25], [0.5, 0.5], [0.625, 0.375], [0.875, 0.125]])
    ptr, col, val = o.symmetrize(idx, P)
    assert ptr.tolist() == [0, 3, 5, 8, 10]
    assert col.tolist() == [1, 2, 3, 0, 2, 0, 1, 3, 0, 2]
    exp = [5 / 32, 1 / 32, 1 / 64, 5 / 32, 7 / 64, 1 / 32, 7 / 64, 3 / 16, 1 / 64, 3 / 16]
    assert val.tolist() == exp


def pin_symmetrize_dense(o, seed: int = 12):
    """Against the dense matrix (P_cond + P_cond^T) / 2N, plus symmetry, total 1,
    sorted columns, no diagonal and N*K <= nnz <= 2*N*K."""
    rng = np.random.default_rng(seed)
    N, K = 300, 20
    X = rng.normal(size=(N, 5)).astype(np.float32)
    idx, d2, _ = o.knn(X, K)
    P, _, _, _ = o.calibrate(d2, 6.0)
    ptr, col, val = o.symmetrize(idx, P)
    dense = np.zeros((N, N))
    dense[np.repeat(np.arange(N), K), idx.reshape(-1)] = P.reshape(-1)
    J = (dense + dense.T) / (2 * N)
    S = np.zeros((N, N))
    for i in range(N):
        cols = col[ptr[i]:ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i not in cols
        S[i, cols] = val[ptr[i]:ptr[i + 1]]
    assert np.allclose(S, J, rtol=1e-15, atol=0)
    assert np.array_equal(S != 0, J != 0)
    assert np.allclose(S, S.T, rtol=0, atol=0)
    assert abs(val.sum() - 1.0) < 1e-12
    assert N * K <= len(val) <= 2 * N * K


def pin_pipeline_small(o):
    """End to end on a 3-point line with K = 2 (mu in (1, 2)): every row has both
    other points, so P_sym is dense off the diagonal and sums to one."""
    X = np.array([[0.0], [1.0], [3.0]], np.float32)
    r = o.similarity(X, mu=1.5, K=2)
    assert r["idx"].tolist() == [[1, 2], [0, 2], [1, 0]]
    # row 0: distances 1 and 9, delta = (0, 8); p0 solves binary entropy = ln 1.5
    a, b = mp.mpf("0.5"), mp.mpf(1) - mp.mpf(10) ** -40  # binary entropy falls on (1/2, 1)
    for _ in range(300):
        m = (a + b) / 2
        if -m * mp.log(m) - (1 - m) * mp.log(1 - m) > mp.log(mp.mpf("1.5")):
            a = m
        else:
            b = m
    p0 = float((a + b) / 2)
    assert abs(r["P"][0, 0] - p0) < 1e-11
    assert abs(r["beta"][0] - float(mp.log(p0 / (1 - p0)) / 8)) < 1e-10
    assert abs(r["val"].sum() - 1.0) < 1e-14


# --------------------------------------------------------------------------
# Attractive forces (Eq. 5-7) and selective exaggeration (Sec. 4.3)
# --------------------------------------------------------------------------


def _sym_csr(rng, N, deg):
    """A random symmetric sparse pattern with positive values, as CSR."""
    rows, cols = [], []
    for i in range(N):
        for j in rng.choice(N, size=deg, replace=False):
            if j != i:
                rows += [i, j]
                cols += [j, i]
    key = sorted(set(zip(rows, cols)))
    vals = {}
    for (i, j) in key:
        if (j, i) in vals:
            vals[(i, j)] = vals[(j, i)]
        else:
            vals[(i, j)] = float(rng.uniform(0.1, 1.0))
    ptr = np.zeros(N + 1, np.int64)
    for (i, _) in key:
        ptr[i + 1] += 1
    ptr = np.cumsum(ptr)
    col = np.array([j for (_, j) in key], np.int32)
    val = np.array([vals[k] for k in key], np.float64)
    return ptr, col, val


def pin_attr_two_points(o):
    """Two points at distance 5: F_0 = p (y_0 - y_1) / (1 + 25), F_1 = -F_0."""
    ptr = np.array([0, 1, 2], np.int64)
    col = np.array([1, 0], np.int32)
    val = np.array([0.5, 0.5])
    Y = np.array([[0.0, 0.0], [3.0, 4.0]])
    F = o.attractive(ptr, col, val, Y)
    assert np.allclose(F, [[-1.5 / 26, -2.0 / 26], [1.5 / 26, 2.0 / 26]], rtol=1e-15, atol=0)


def pin_attr_exact_rational(o):
    """Four points with integer coordinates and rational p, summed exactly."""
    Yq = [(0, 0), (1, 2), (-2, 1), (3, -1)]
    P = {(0, 1): Fraction(1, 8), (0, 2): Fraction(1, 16), (1, 2): Fraction(3, 16), (1, 3): Fraction(1, 8),
         (2, 3): Fraction(1, 32)}
    P.update({(j, i): v for (i, j), v in list(P.items())})
    key = sorted(P)
    ptr = np.zeros(5, np.int64)
    for (i, _) in key:
        ptr[i + 1] += 1
    ptr = np.cumsum(ptr)
    F = o.attractive(ptr, np.array([j for _, j in key], np.int32), np.array([float(P[k]) for k in key]),
                     np.array(Yq, np.float64))
    for i in range(4):
        for d in range(2):
            exact = Fraction(0)
            for (a, b), p in P.items():
                if a != i:
                    continue
                d2 = sum((Yq[a][t] - Yq[b][t]) ** 2 for t in range(2))
                exact += p * (Yq[a][d] - Yq[b][d]) / (1 + d2)
            assert abs(F[i, d] - float(exact)) <= 1e-16 * max(1.0, abs(float(exact)))


def pin_attr_invariants(o, seed: int = 13):
    """Pairwise forces cancel (P symmetric), translation invariance, rotation
    equivariance, linearity in P."""
    rng = np.random.default_rng(seed)
    ptr, col, val = _sym_csr(rng, 60, 5)
    Y = rng.normal(size=(60, 2)) * 3
    F = o.attractive(ptr, col, val, Y)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() <= 1e-13 * scale
    assert np.allclose(o.attractive(ptr, col, val, Y + np.array([5.0, -7.0])), F, rtol=1e-11, atol=1e-14)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    assert np.allclose(o.attractive(ptr, col, val, Y @ R), F @ R, rtol=1e-10, atol=1e-13)
    assert np.allclose(o.attractive(ptr, col, 3.0 * val, Y), 3.0 * F, rtol=1e-14, atol=0)


def pin_attr_exaggeration(o):
    """Multiplier tau at the refine iteration, 1 + (tau - 1)/2 after decay ln 2
    iterations, 1 when never refined or refined later; the global factor multiplies."""
    ptr = np.array([0, 1, 2, 3, 4, 4], np.int64)
    col = np.array([1, 0, 3, 2], np.int32)
    val = np.full(4, 0.25)
    Y = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0], [0.0, 0.0], [9.0, 9.0]])
    base = o.attractive(ptr, col, val, Y)
    t_now = 100
    decay = 20.0 / np.log(2.0)
    t_ref = np.array([100, 80, -1, 150, 3], np.int32)
    F = o.attractive(ptr, col, val, Y, t_ref=t_ref, tau=12.0, decay=decay, t_now=t_now, global_exag=2.0)
    m = np.array([12.0, 1.0 + 11.0 / 2.0, 1.0, 1.0, 1.0]) * 2.0
    assert np.allclose(F, base * m[:, None], rtol=1e-14, atol=0)
    assert np.all(F[4] == 0.0)  # an isolated point feels no attraction


# --------------------------------------------------------------------------
# Precision rho (Eq. 9): mean over rows of |N^A_i & N_i| / |N_i|
# --------------------------------------------------------------------------


def pin_recall(o, recall=None):
    """Eq. 9 on hand-counted rows; invalid lists are refused, not scored."""
    from oracle import oracle as O

    rec = recall or O.recall
    # rows share 2 of 3 and 3 of 3 ids: (2 + 3) / 6
    assert rec(np.array([[1, 2, 3], [4, 5, 6]]), np.array([[3, 2, 9], [6, 5, 4]])) == 5 / 6
    # order inside a row does not matter; identical lists score 1, disjoint 0
    e = np.array([[7, 8, 9, 10]])
    assert rec(e[:, ::-1], e) == 1.0
    assert rec(np.array([[0, 1, 2, 3]]), e) == 0.0
    # an absent entry (-1, a deleted neighbour) is a miss: 1 of 3
    assert rec(np.array([[1, -1, -1]]), np.array([[1, 2, 3]])) == 1 / 3
    # a repeated id must not count twice: the list is refused
    for bad, kw in [(np.array([[1, 1, 1]]), {}),            # duplicates
                    (np.array([[4, 2, 3]]), {"query_ids": [4]}),  # the row's own id
                    (np.array([[1, 2, 9]]), {"n": 5}),          # outside [0, n)
                    (np.array([[1, -1, 2]]), {})]:              # a listed id after an absent one
        try:
            rec(bad, np.array([[1, 2, 3]]), **kw)
        except ValueError:
            continue
        raise AssertionError("recall scored an invalid list %s" % bad.tolist())


KNN_PINS = [pin_knn_exact_rational, pin_knn_line, pin_knn_sklearn, pin_knn_metamorphic, pin_knn_subset]
CAL_PINS = [pin_calibrate_two_level, pin_calibrate_progression, pin_calibrate_invariants,
            pin_calibrate_scaling, pin_calibrate_degenerate, pin_calibrate_brentq]
SYM_PINS = [pin_symmetrize_hand, pin_symmetrize_dense, pin_pipeline_small]
ATTR_PINS = [pin_attr_two_points, pin_attr_exact_rational, pin_attr_invariants, pin_attr_exaggeration]
METRIC_PINS = [pin_recall]
ALL_PINS = KNN_PINS + CAL_PINS + SYM_PINS + ATTR_PINS + METRIC_PINS
