"""GPU refinement orderings (Sec. 5.1) against the oracle.

Density order and hop counts are exact (integer or identical FP32 keys).
Path lengths are FP32 sums along paths: with h hops each of the h additions
and the h square roots rounds once, so a path length is within (2h + 2) u of
its FP64 value (u = 2^-24); the test applies that bound with h the hop count
of the oracle's shortest path tree.  At the full image-like size the visit is
checked by the properties that define it at any size: seeds at 0, no edge
relaxes any further, every reached point has a tight predecessor, and no
unreached point has a reached predecessor.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import refine_order as RO
from paper_1512_01655_amd import datagen
from tests.gpu_common import lib, say

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def A():
    return lib()


def _graph(A, X, k):
    idx, d2, fl = A.knn(torch.from_numpy(X).cuda(), k)
    return idx, d2


def test_density_order(A):
    X = datagen.mixture_isotropic(n=3000, d=20, seed=61)
    idx, d2 = _graph(A, X, 30)
    P, beta, perp, fl = A.calibrate_p(d2, 10.0)
    b = beta.cpu().numpy()
    got = A.order_density(beta).cpu().numpy()
    assert np.array_equal(got, RO.density_order(b))
    rng = np.random.default_rng(2)
    sel = rng.choice(3000, size=700, replace=False).astype(np.int32)
    got = A.order_density(beta, torch.from_numpy(sel).cuda()).cpu().numpy()
    assert np.array_equal(got, RO.density_order(b, sel))
    # ties, beta = 0 (all neighbours equidistant) and beta = +inf (degenerate limit)
    bb = np.array([2.0, 1.0, 2.0, 0.5, 1.0, np.inf, 0.0], np.float32)
    got = A.order_density(torch.from_numpy(bb).cuda()).cpu().numpy()
    assert got.tolist() == RO.density_order(bb).tolist() == [6, 3, 1, 4, 0, 2, 5]
    with pytest.raises(A.AtsneError):
        A.order_density(beta, torch.tensor([0, 3000], dtype=torch.int32, device="cuda"))


def _hops(idx, d2, dist, seeds):
    """Hop count along the oracle's shortest path tree (for the FP32 bound)."""
    N, k = idx.shape
    order = np.argsort(dist, kind="stable")
    hops = np.full(N, np.inf)
    hops[seeds] = 0
    for i in order:
        if not np.isfinite(dist[i]):
            break
        for s in range(k):
            j = idx[i, s]
            if j >= 0 and abs(dist[i] + math.sqrt(d2[i, s]) - dist[j]) <= 1e-12 * max(dist[j], 1e-300):
                hops[j] = min(hops[j], hops[i] + 1)
    return np.where(np.isinf(hops), N, hops)  # zero-length edges: fall back to the N-hop bound


@pytest.mark.parametrize("absent", [False, True])
def test_neighbourhood_small(A, absent):
    X = datagen.mixture_isotropic(n=2500, d=8, seed=62)
    idx, d2 = _graph(A, X, 6)
    if absent:
        idx[::5, -2:] = -1  # deleted neighbours carry no edge
        d2[::5, -2:] = float("inf")
    ih, dh = idx.cpu().numpy(), d2.cpu().numpy().astype(np.float64)
    seeds = np.array([3, 1700, 42, 3], np.int32)  # a repeated seed is one seed
    st = torch.from_numpy(seeds).cuda()
    for depth in (-1, 0, 3):
        order, key = A.order_neighbourhood(idx, None, st, weighted=False, max_depth=depth)
        lv = RO.bfs_levels(ih, seeds, max_depth=depth)
        k = key.cpu().numpy()
        assert np.array_equal(np.where(np.isinf(k), -1, k).astype(np.int64), lv)
        assert np.array_equal(order.cpu().numpy(), RO.order_by_key(np.where(lv < 0, np.inf, lv)))
    order, key = A.order_neighbourhood(idx, d2, st, weighted=True)
    ref = RO.path_lengths(ih, dh, seeds)
    k = key.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isinf(k), np.isinf(ref))
    fin = np.isfinite(ref)
    h = _hops(ih, dh, ref, seeds)
    bound = (2 * h[fin] + 2) * U * ref[fin]
    err = np.abs(k[fin] - ref[fin])
    say("    weighted: %d reached, max hops %d, max err/bound %.3f" % (fin.sum(), h[fin].max(),
                                                                     (err / np.maximum(bound, 1e-300)).max()))
    assert np.all(err <= bound)
    o = order.cpu().numpy()
    assert sorted(o.tolist()) == np.flatnonzero(fin).tolist()
    assert np.all(np.diff(k[o]) >= 0)  # sorted by the GPU's own keys
    assert np.all(np.diff(ref[o]) >= -2 * bound.max())


def test_neighbourhood_errors(A):
    idx = torch.zeros((10, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(A.AtsneError):
        A.order_neighbourhood(idx, None, torch.tensor([10], dtype=torch.int32, device="cuda"))
    order, key = A.order_neighbourhood(idx, None, torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert order.numel() == 0 and torch.all(torch.isinf(key))


def test_neighbourhood_full_size_properties(A):
    X = datagen.image_like()
    idx, d2 = _graph(A, X, 90)
    ih = idx.cpu().numpy()
    w = np.sqrt(d2.cpu().numpy())  # FP32 square roots, as the kernel takes them
    seeds = np.array([0, 12345, 69999, 500, 31337], np.int32)
    st = torch.from_numpy(seeds).cuda()
    N, k = ih.shape
    src = np.repeat(np.arange(N), k)
    dst = ih.reshape(-1)
    for weighted in (False, True):
        order, key = A.order_neighbourhood(idx, d2 if weighted else None, st, weighted=weighted)
        key = key.cpu().numpy()
        o = order.cpu().numpy()
        reached = np.isfinite(key)
        assert np.all(key[seeds] == 0)
        assert sorted(o.tolist()) == np.flatnonzero(reached).tolist()
        assert np.all(np.diff(key[o]) >= 0)
        r = reached[src]
        if weighted:
            cand = (key[src] + w.reshape(-1)).astype(np.float32)  # fl(key_i + w_ij)
        else:
            cand = key[src] + 1
        # no edge from a reached point relaxes further, and none leads to an unreached point
        assert np.all(key[dst[r]] <= cand[r])
        # every reached non-seed point has a tight predecessor
        tight = np.zeros(N, bool)
        tight[dst[r & (cand == key[dst])]] = True
        tight[seeds] = True
        assert np.array_equal(tight, reached)
        say("    %s: %d reached, max key %.4g" % ("weighted" if weighted else "hops", reached.sum(),
                                                  key[reached].max()))
