"""GPU precision-controlled approximate kNN (cluster-pruned search) against
its oracle definition (oracle/ivf.py).

The partition is checked step by step: the assignment against the FP64
nearest centroid (the GPU's assigned centroid must be nearest within the
FP32 tie rule), the update against the FP64 mean of the members (FP32 sum of
n terms: relative error below (n + 2) u of the sum of magnitudes), and the
probe order against FP64 centroid distances.  The search is checked against
the exact kNN over each point's tile-rounded candidates (the library's
reading: whole 256-row tiles covering the candidate clusters), computed by
the oracle from the GPU's partition (the partition is an input of the
search), with the same neighbour-set tie rule as the exact path; and against
the oracle's definition over the candidate clusters' rows, which that
superset can only match or beat at every rank.
"""
import numpy as np
import pytest
import torch

from oracle import ivf as IV
from oracle import oracle as O
from paper_1512_01655_amd import datagen
from tests import ivf_reading as RD
from tests import parity
from tests.gpu_common import lib, say

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def A():
    return lib()


def _assign_ok(X, cent, assign):
    D = IV.sqdist(X, np.asarray(cent, np.float64))
    best = D.min(axis=1)
    got = D[np.arange(X.shape[0]), assign]
    assert np.all(got <= best * (1 + parity.TIE_REL) + 1e-30), "a point is not at its nearest centroid"


def test_partition_steps(A):
    X = datagen.mixture_isotropic(n=3000, d=30, seed=81)
    C = 24
    init = np.random.default_rng(3).choice(3000, size=C, replace=False).astype(np.int32)
    Xt = torch.from_numpy(X).cuda()
    ix0 = A.IVF(Xt, C, iters=0, init_ids=init)
    a0, c0, s0, p0 = ix0.partition()
    a0 = a0.cpu().numpy()
    assert np.array_equal(c0.cpu().numpy(), X[init])
    _assign_ok(X, X[init], a0)
    ix0.close()
    ix1 = A.IVF(Xt, C, iters=1, init_ids=init)
    a1, c1, s1, p1 = ix1.partition()
    a1, c1 = a1.cpu().numpy(), c1.cpu().numpy().astype(np.float64)
    ref = IV.lloyd_update(X, a0, X[init])
    for c in range(C):
        mem = X[a0 == c].astype(np.float64)
        bound = (len(mem) + 2) * U * np.abs(mem).sum(axis=0) / max(len(mem), 1) + 1e-30
        assert np.all(np.abs(c1[c] - ref[c]) <= 2 * bound)
    _assign_ok(X, c1, a1)
    perm, start = IV.cluster_order(a1, C)
    assert np.array_equal(s1, start)
    Dc = IV.sqdist(c1, c1)
    for c in range(C):
        assert p1[c, 0] == c and sorted(p1[c].tolist()) == list(range(C))
        d = Dc[c, p1[c, 1:]]
        assert np.all(np.diff(d) >= -parity.TIE_REL * d[1:])
    ix1.close()


@pytest.mark.parametrize("n_probe", [1, 3, 24])
def test_search_matches_definition(A, n_probe):
    X = datagen.mixture_isotropic(n=3000, d=30, seed=82)
    C, k = 24, 30
    init = np.random.default_rng(4).choice(3000, size=C, replace=False).astype(np.int32)
    ix = A.IVF(torch.from_numpy(X).cuda(), C, iters=4, init_ids=init)
    assign, cent, start, probe = ix.partition()
    assign = assign.cpu().numpy()
    idx, d2, fl, frac = ix.knn(k, n_probe)
    g_idx, g_d2 = idx.cpu().numpy(), d2.cpu().numpy()
    probe = np.asarray(probe)
    o_idx, o_d2, o_nx, ncand = RD.search_tile_rounded(X, k, assign, C, probe, n_probe)
    rows = np.arange(3000)
    ties, exact = parity.check_knn(X, rows, g_idx, g_d2, o_idx, o_d2, o_nx)
    assert abs(frac - ncand.sum() / 3000.0 ** 2) < 1e-9
    # the oracle's definition: candidates are the candidate clusters' rows;
    # the tile-rounded superset is as close or closer at every rank
    d_idx, d_d2, _, dcand = IV.search(X, k, assign, C, cent.cpu().numpy(), n_probe, probe=probe)
    assert np.all(dcand <= ncand)
    td = np.sort(parity.true_d2(X, rows, g_idx), axis=1)
    assert np.all(td <= d_d2 * (1 + parity.TIE_REL) + 1e-30)
    e_idx, _, _ = O.get().knn(X, k)
    rho = IV.precision(g_idx, e_idx)
    rho_def = IV.precision(d_idx, e_idx)
    say("    n_probe %d: candidates %.3f of N, precision %.4f (definition's %.4f), %d tie-rule rows" % (
        n_probe, frac, rho, rho_def, ties))
    assert rho >= rho_def - 1e-3
    if n_probe == C:
        assert frac == 1.0 and rho == 1.0
        # every tile probed: the exact search's rows bit for bit (the index
        # searches a cluster-sorted copy on its own contraction)
        x_idx, x_d2, _ = A.knn(torch.from_numpy(X).cuda(), k)
        assert np.array_equal(idx.cpu().numpy(), x_idx.cpu().numpy())
        assert np.array_equal(d2.cpu().numpy(), x_d2.cpu().numpy())
    ix.close()


def test_fit_and_full_size(A):
    """The image-like workload (N = 70000, D = 784): fit n_probe to rho = 0.9
    on a sample of clusters, search all points, measure Eq. 9 against the
    exact GPU path, and check sampled rows against the oracle definition."""
    X = datagen.image_like()
    N, C, k, rho = X.shape[0], 256, 90, 0.9
    Xt = torch.from_numpy(X).cuda()
    rng = np.random.default_rng(5)
    ix = A.IVF(Xt, C, iters=8, init_ids=rng.choice(N, size=C, replace=False))
    sample = rng.choice(C, size=16, replace=False)
    n_probe, rho_s = ix.fit(k, rho, sample)
    idx, d2, fl, frac = ix.knn(k, n_probe)
    e_idx, e_d2, e_fl = A.knn(Xt, k)
    rho_all = IV.precision(idx.cpu().numpy(), e_idx.cpu().numpy())
    say("    fit: n_probe %d (sample precision %.4f), all rows %.4f, candidates %.4f of N" % (
        n_probe, rho_s, rho_all, frac))
    assert rho_s >= rho and rho_all >= rho - 0.03
    assign, cent, start, probe = ix.partition()
    rows = rng.choice(N, size=200, replace=False).astype(np.int32)
    o_idx, o_d2, o_nx, _ = RD.search_tile_rounded(X, k, assign.cpu().numpy(), C, np.asarray(probe), n_probe,
                                                  rows=rows)
    parity.check_knn(X, rows, idx.cpu().numpy()[rows], d2.cpu().numpy()[rows], o_idx, o_d2, o_nx)
    ix.close()


def test_ivf_errors(A):
    X = torch.from_numpy(datagen.mixture_isotropic(n=500, d=8, seed=83)).cuda()
    with pytest.raises(A.AtsneError):
        A.IVF(X, 1)  # at least two clusters
    with pytest.raises(A.AtsneError):
        A.IVF(X, 4, init_ids=[0, 1, 1, 2])  # initial points must be distinct
    ix = A.IVF(X, 8, iters=2)
    with pytest.raises(A.AtsneError):
        ix.knn(500, 2)  # k above N - 1
    with pytest.raises(A.AtsneError):
        ix.fit(10, 1.5, [0])
    ix.close()
