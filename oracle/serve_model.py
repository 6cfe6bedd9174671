"""Sequential FP64 model of the data-manipulation operations of Sec. 5.3 --
TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module; the GPU library never does, and
the two share no code.  It keeps, for every point, the neighbour list that
the operations of Sec. 5.3 define, applied one at a time in submission order:

  * creation (Sec. 3.1): a point's list is its exact K nearest live points,
    K = floor(3 mu), by the key (squared distance, index);
  * insertion (Eq. 13): for every live point x_i with a non-empty list, each
    new point strictly closer than x_i's farthest listed neighbour enters
    the list and that farthest neighbour leaves, so the list keeps its
    length.  A batch of new points is inserted at once; one point after the
    other gives the same lists, since each step keeps the nearest entries of
    the union by (d, j);
  * deletion (Sec. 5.3): the deleted point leaves every list without a
    replacement, and the list's precision rho_i drops by 1/K.

Readings taken (the paper is silent on them):
  * a list shortened by deletions stays short: Eq. 13 compares with and
    evicts the farthest neighbour that is still listed, so a hole is never
    refilled, and rho_i = (listed neighbours) / K;
  * a row's conditional P is calibrated over its listed neighbours only
    (absent entries get p = 0); a row with no more listed neighbours than mu
    cannot reach the target perplexity and is uniform over them, flagged
    degenerate;
  * a deleted point's own list is empty (rho = 0, P = 0).

Distances are FP64 direct differences of the FP32 inputs, as in the C oracle.
``mutant`` > 0 plants one deliberate mistake so the pins can show they catch
it (see the CPU tests); 0 is the model.

Parity status: pinned by ``tests/test_oracle_serve_model.py`` (insert-only
sequences reduce to brute-force kNN of the grown corpus, delete-only
sequences to the initial lists minus the deleted points, and a from-scratch
recomputation of every row over a mixed sequence; planted mistakes fail).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

FLAG_NOT_CONVERGED = O.FLAG_NOT_CONVERGED
FLAG_DEGENERATE = O.FLAG_DEGENERATE
TIE_REL = 1e-5


def sqdist(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """FP64 squared distances by direct difference, rows of A against rows of B."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    out = np.empty((A.shape[0], B.shape[0]), np.float64)
    step = max(1, (1 << 22) // max(1, B.shape[0] * A.shape[1]))
    for s in range(0, A.shape[0], step):
        diff = A[s:s + step, None, :] - B[None, :, :]
        out[s:s + step] = np.einsum("rbd,rbd->rb", diff, diff)
    return out


def calibrate_absent(d2: np.ndarray, mu: float, oracle: O.Oracle | None = None):
    """Calibrate rows whose +inf entries are absent (Eq. 3, Eq. 4, Eq. 8 over
    the listed neighbours).  Returns (P, beta, flags) like the C oracle."""
    ora = oracle or O.get()
    d2 = np.asarray(d2, np.float64)
    M, K = d2.shape
    P = np.zeros((M, K), np.float64)
    beta = np.zeros((M,), np.float64)
    flags = np.zeros((M,), np.uint8)
    present = np.isfinite(d2)
    cnt = present.sum(axis=1)
    for c in np.unique(cnt):
        rows = np.flatnonzero(cnt == c)
        if c == 0:
            flags[rows] = FLAG_DEGENERATE
            continue
        sub = np.stack([d2[r][present[r]] for r in rows])
        if not (mu < c):
            Pc = np.full(sub.shape, 1.0 / c)
            bc = np.zeros(len(rows))
            fc = np.full(len(rows), FLAG_DEGENERATE, np.uint8)
        else:
            Pc, bc, _, fc = ora.calibrate(sub, mu)
        for t, r in enumerate(rows):
            P[r][present[r]] = Pc[t]
        beta[rows] = bc
        flags[rows] = fc
    return P, beta, flags


class ResidentModel:
    """Neighbour lists of a growing and shrinking corpus (Sec. 5.3)."""

    def __init__(self, X0: np.ndarray, mu: float, oracle: O.Oracle | None = None, mutant: int = 0):
        self.ora = oracle or O.get()
        self.mu = float(mu)
        self.K = int(math.floor(3.0 * mu))
        self.mutant = int(mutant)
        self.X = np.ascontiguousarray(X0, np.float32).copy()
        n = self.X.shape[0]
        self.alive = np.ones(n, bool)
        idx, d2, nxt = self.ora.knn(self.X, self.K)
        self.idx = idx.astype(np.int32)
        self.d2 = d2.astype(np.float64)
        # rows where a decision of the model sat within TIE_REL of its boundary
        self.tie_rows = set(np.flatnonzero(nxt <= d2[:, -1] * (1 + TIE_REL)).tolist())
        self.history = []  # ("i", first_row, count) / ("d", ids)

    # -- queries ---------------------------------------------------------
    def n_rows(self) -> int:
        return self.X.shape[0]

    def present(self) -> np.ndarray:
        return (self.idx >= 0).sum(axis=1)

    def rho(self) -> np.ndarray:
        """Precision rho_i = listed neighbours / K; 0 for deleted points."""
        r = self.present() / float(self.K)
        r[~self.alive] = 0.0
        return r

    def calibrated(self):
        return calibrate_absent(self.d2, self.mu, self.ora)

    # -- operations --------------------------------------------------------
    def insert(self, Xnew: np.ndarray) -> np.ndarray:
        """Insert a batch; returns the ids of resident rows whose list changed."""
        Xnew = np.ascontiguousarray(Xnew, np.float32)
        B = Xnew.shape[0]
        r0 = self.n_rows()
        self.X = np.concatenate([self.X, Xnew])
        self.alive = np.concatenate([self.alive, np.ones(B, bool)])
        live = np.flatnonzero(self.alive)
        if self.mutant == 4:  # planted: new rows also see deleted points
            live = np.arange(self.n_rows())
        # new rows: exact K nearest live points (the batch included)
        qpos = np.arange(len(live) - B, len(live), dtype=np.int32)
        li, ld, lnext = self.ora.knn(self.X[live], self.K, query_ids=qpos)
        new_idx = live[li].astype(np.int32)
        for t in np.flatnonzero(lnext <= ld[:, -1] * (1 + TIE_REL)):
            self.tie_rows.add(r0 + int(t))
        # Eq. 13 over the live residents that existed before the batch
        res = live[(live < r0) & self.alive[live]]
        dist = sqdist(self.X[res], Xnew)
        # rows that a new point can reach (or nearly reach): the others keep their list
        npv = (self.idx[res] >= 0).sum(axis=1)
        dmv = np.where(npv > 0, self.d2[res, np.maximum(npv - 1, 0)], -np.inf)
        if self.mutant == 1:
            dmv = np.where((npv > 0) & (npv < self.K), np.inf, dmv)
        reach = np.flatnonzero((dist <= (dmv * (1 + TIE_REL))[:, None]).any(axis=1))
        changed = []
        for t in reach:
            i = res[t]
            npres = int((self.idx[i] >= 0).sum())
            if npres == 0:
                continue
            if self.mutant == 1:  # planted: holes are refilled by any new point
                dmax = math.inf if npres < self.K else self.d2[i, self.K - 1]
                npres = self.K if npres < self.K else npres
            else:
                dmax = self.d2[i, npres - 1]
            dj = dist[t]
            cand = np.flatnonzero(dj < dmax)
            near = np.abs(dj - dmax) <= TIE_REL * dmax
            if np.any(near):
                self.tie_rows.add(int(i))
            if cand.size == 0:
                continue
            keys = [(self.d2[i, s], int(self.idx[i, s])) for s in range(self.K) if self.idx[i, s] >= 0]
            keys += [(float(dj[c]), r0 + int(c)) for c in cand]
            keys.sort()
            if len(keys) > npres and keys[npres][0] <= keys[npres - 1][0] * (1 + TIE_REL):
                self.tie_rows.add(int(i))
            if self.mutant == 2:  # planted: the nearest neighbour is evicted instead of the farthest
                keep = keys[1:npres + 1] if len(keys) > npres else keys
            else:
                keep = keys[:npres]
            row_i = np.full(self.K, -1, np.int32)
            row_d = np.full(self.K, math.inf)
            for s, (d, j) in enumerate(keep):
                row_i[s], row_d[s] = j, d
            if not np.array_equal(row_i, self.idx[i]):
                changed.append(int(i))
            self.idx[i], self.d2[i] = row_i, row_d
        self.idx = np.concatenate([self.idx, new_idx])
        self.d2 = np.concatenate([self.d2, ld])
        self.history.append(("i", r0, B))
        return np.asarray(sorted(changed), np.int32)

    def delete(self, ids) -> np.ndarray:
        """Delete live points; returns the ids of live rows whose list changed."""
        ids = np.asarray(ids, np.int32)
        assert np.all(self.alive[ids]) and len(np.unique(ids)) == len(ids)
        self.alive[ids] = False
        if self.mutant == 3:  # planted: lists keep the deleted points
            hit = np.zeros(self.idx.shape, bool)
        else:
            hit = np.isin(self.idx, ids)
        changed = []
        for i in np.flatnonzero(hit.any(axis=1)):
            if not self.alive[i]:
                continue
            keep = (self.idx[i] >= 0) & ~hit[i]
            n = int(keep.sum())
            row_i = np.full(self.K, -1, np.int32)
            row_d = np.full(self.K, math.inf)
            row_i[:n] = self.idx[i][keep]
            row_d[:n] = self.d2[i][keep]
            self.idx[i], self.d2[i] = row_i, row_d
            changed.append(int(i))
        self.idx[ids] = -1
        self.d2[ids] = math.inf
        self.history.append(("d", ids.copy()))
        return np.asarray(sorted(changed), np.int32)
