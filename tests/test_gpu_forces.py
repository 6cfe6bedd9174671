"""GPU attractive forces (Eq. 5-7 over the sparse symmetric P, selective
exaggeration of Sec. 4.3) against the FP64 oracle.

Tolerance, from the FP32 arithmetic of one term t_j = w_j (y_i - y_j)_d with
w_j = p_ij / (1 + d_ij^2): the difference, the dims-term squared norm, the
add, the divide and the accumulate each round once, and the row sum of n_i
terms adds at most n_i roundings, so
    |F_gpu - F_oracle| <= m_i (n_i + dims + 8) u sum_j |t_j| + 8 u |F_i|,
u = 2^-24; the second term covers the exaggeration factor's own rounding
(exp and two products).  The test applies this bound with a factor 2.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1512_01655_amd import datagen
from tests.gpu_common import lib, say

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def A():
    return lib()


def _sim(A, Xt, mu):
    k = int(np.floor(3 * mu))
    idx, d2, fl = A.knn(Xt, k)
    P, beta, perp, fl = A.calibrate_p(d2, mu, flags=fl)
    return A.symmetrize(idx, P)


def _check(A, rp, col, val, Y, dims, t_ref=None, tau=1.0, decay=1.0, t_now=0, g=1.0, label=""):
    N = Y.shape[0]
    Yt = torch.from_numpy(Y.astype(np.float32)).cuda()
    tr = None if t_ref is None else torch.from_numpy(t_ref.astype(np.int32)).cuda()
    F = A.attractive_forces(rp, col, val, Yt, t_ref=tr, tau=tau, decay=decay, t_now=t_now,
                            global_exaggeration=g)
    torch.cuda.synchronize()
    F = F.cpu().numpy().astype(np.float64)
    rp_h, col_h, val_h = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    Y32 = Y.astype(np.float32).astype(np.float64)
    ref = O.get().attractive(rp_h, col_h, val_h.astype(np.float64), Y32, t_ref=t_ref, tau=tau, decay=decay,
                             t_now=t_now, global_exag=g)
    # the bound's ingredients, in FP64
    m = np.full(N, g)
    if t_ref is not None:
        ok = (t_ref >= 0) & (t_ref <= t_now)
        m = m * np.where(ok, 1.0 + (tau - 1.0) * np.exp(-(t_now - t_ref) / decay), 1.0)
    rows = np.repeat(np.arange(N), np.diff(rp_h))
    cv = col_h[: len(rows)]
    valid = (cv >= 0) & (cv < N)
    diff = Y32[rows] - Y32[np.where(valid, cv, 0)]
    w = val_h[: len(rows)] / (1.0 + (diff ** 2).sum(axis=1))
    absterm = np.zeros((N, dims))
    np.add.at(absterm, rows[valid], np.abs(w[valid, None] * diff[valid]))
    n_i = np.diff(rp_h)
    bound = 2.0 * (m[:, None] * (n_i[:, None] + dims + 8) * U * absterm + 8 * U * np.abs(ref))
    err = np.abs(F - ref)
    worst = (err / np.maximum(bound, 1e-300)).max()
    say("    %s: N=%d nnz=%d max err %.3g, max err/bound %.3f" % (label, N, len(col_h), err.max(), worst))
    assert np.all(err <= bound), "attractive forces outside the FP32 bound"
    return F


def test_forces_small_with_exaggeration(A):
    X = datagen.mixture_isotropic(n=2000, d=50, seed=51)
    rp, col, val = _sim(A, torch.from_numpy(X).cuda(), 30.0)
    rng = np.random.default_rng(3)
    Y = rng.normal(size=(2000, 2)) * 8.0
    _check(A, rp, col, val, Y, 2, label="dims 2")
    t_ref = rng.integers(-5, 300, size=2000)
    _check(A, rp, col, val, Y, 2, t_ref=t_ref, tau=12.0, decay=30.0, t_now=250, g=4.0, label="exaggerated")
    _check(A, rp, col, val, rng.normal(size=(2000, 3)) * 5.0, 3, label="dims 3")


def test_forces_edges(A):
    # one point, a row without entries, and a malformed column that is skipped
    Y = np.array([[0.0, 0.0], [3.0, 4.0], [1.0, 1.0]])
    rp = torch.tensor([0, 1, 2, 4], dtype=torch.int64, device="cuda")
    col = torch.tensor([1, 0, 0, 7], dtype=torch.int32, device="cuda")
    val = torch.tensor([0.5, 0.5, 0.25, 0.25], dtype=torch.float32, device="cuda")
    F = A.attractive_forces(rp, col, val, torch.from_numpy(Y.astype(np.float32)).cuda()).cpu().numpy()
    assert np.allclose(F[0], [-1.5 / 26, -2.0 / 26], rtol=1e-6)
    assert np.allclose(F[2], [0.25 / 3, 0.25 / 3], rtol=1e-6)  # the entry with column 7 is ignored
    one = A.attractive_forces(torch.zeros(2, dtype=torch.int64, device="cuda"),
                              torch.zeros(0, dtype=torch.int32, device="cuda"),
                              torch.zeros(0, dtype=torch.float32, device="cuda"),
                              torch.ones((1, 2), device="cuda"))
    assert torch.all(one == 0)
    with pytest.raises(A.AtsneError):
        A.attractive_forces(rp, col, val, torch.ones((3, 4), device="cuda"))


def test_forces_full_size(A):
    """The image-like workload's P (N = 70000) at the size the benchmark times."""
    X = datagen.image_like()
    rp, col, val = _sim(A, torch.from_numpy(X).cuda(), 30.0)
    rng = np.random.default_rng(4)
    Y = rng.normal(size=(X.shape[0], 2)) * 20.0
    t_ref = np.where(rng.random(X.shape[0]) < 0.1, rng.integers(0, 100, X.shape[0]), -1)
    _check(A, rp, col, val, Y, 2, t_ref=t_ref, tau=12.0, decay=25.0, t_now=100, g=1.0, label="image-like")
