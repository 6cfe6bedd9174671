"""GPU calibration (atsne_calibrate_p) and symmetrisation (atsne_symmetrize*)
against the FP64 oracle, stage by stage and end to end."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1512_01655_amd import datagen
from tests import parity
from tests.gpu_common import lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    return lib()


@pytest.fixture(scope="module")
def ora():
    return O.get()


def _cal(A, d2: np.ndarray, mu, **kw):
    say("  calibrate M=%d k=%d mu=%g" % (d2.shape[0], d2.shape[1], mu))
    P, beta, perp, fl = A.calibrate_p(torch.from_numpy(d2.astype(np.float32)).cuda(), mu, **kw)
    torch.cuda.synchronize()
    return P.cpu().numpy(), beta.cpu().numpy(), perp.cpu().numpy(), fl.cpu().numpy()


def _check_cal(A, ora, d2, mu):
    d2f = d2.astype(np.float32)
    gP, gb, gperp, gfl = _cal(A, d2f, mu)
    oP, ob, operp, ofl = ora.calibrate(d2f.astype(np.float64), mu)
    ok = ofl == 0
    dP = np.abs(gP - oP)[ok].max()
    perp = parity.perplexity_of_rows(gP)[ok]
    say("    max|dP| %.3g  max|perp-mu| %.3g  max rel dbeta %.3g" % (
        dP, np.abs(perp - mu).max(), (np.abs(gb - ob) / ob)[ok].max()))
    assert dP <= parity.P_TOL
    # the FP32 entropy resolves the perplexity to about 1e-6 mu: the 1e-4
    # contract holds up to mu = 100, 2e-6 mu above (the bound the entry
    # states); rows whose bracket collapsed before tol carry TOL_LIMITED
    lim = (gfl[ok] & A.FLAG_TOL_LIMITED) != 0
    say("    TOL_LIMITED rows %d / %d" % (int(lim.sum()), int(ok.sum())))
    assert np.abs(perp - mu).max() <= (parity.PERP_TOL if mu <= 100 else 2e-6 * mu)
    assert np.abs(gP.astype(np.float64).sum(1) - 1.0).max() <= 1e-6
    assert np.all((gfl[ok] | A.FLAG_TOL_LIMITED) == A.FLAG_TOL_LIMITED)
    return gP, gb


def test_calibrate_on_oracle_neighbours_config1(A, ora):
    X = datagen.mixture_isotropic()
    _, d2, _ = ora.knn(X, 90)
    _check_cal(A, ora, d2, 30.0)


@pytest.mark.parametrize("k,mu", [(2, 1.5), (30, 10.0), (64, 21.0), (65, 21.5), (150, 50.0), (300, 100.0),
                                  (1000, 333.0)])
def test_calibrate_k_range(A, ora, k, mu):
    rng = np.random.default_rng(k)
    d2 = np.sort(rng.gamma(4.0, 2.0, size=(257, k)), axis=1) + rng.uniform(0, 50, size=(257, 1))
    _check_cal(A, ora, d2, mu)


def test_calibrate_scale_range(A, ora):
    # distances from 1e-6 to 1e6 scale: beta spans 12 decades
    rng = np.random.default_rng(11)
    for s in [1e-6, 1e-3, 1.0, 1e3, 1e6]:
        d2 = np.sort(rng.uniform(1.0, 3.0, size=(100, 90)), axis=1) * s
        _check_cal(A, ora, d2, 30.0)


def test_calibrate_degenerate(A, ora):
    d2 = np.array([[1.0] * 12 + [2.0] * 18, [3.0] * 30, [0.0] * 30], np.float32)
    gP, gb, gperp, gfl = _cal(A, d2, 10.0)
    assert np.all(gfl & 4)
    assert np.allclose(gP[0, :12], 1 / 12) and np.all(gP[0, 12:] == 0) and np.isinf(gb[0])
    assert np.allclose(gP[1], 1 / 30) and np.allclose(gP[2], 1 / 30)


def test_calibrate_strict_not_converged(A):
    d2 = torch.from_numpy(np.sort(np.random.default_rng(1).uniform(1, 2, size=(50, 30)), 1).astype(np.float32)).cuda()
    with pytest.raises(A.AtsneError) as e:
        A.calibrate_p(d2, 10.0, max_iter=1, strict=True)
    assert e.value.status == A.E_NOT_CONVERGED
    with pytest.raises(A.AtsneError) as e:
        A.calibrate_p(d2, 30.0)
    assert e.value.status == A.E_K_RANGE


def _sym(A, idx, P):
    say("  symmetrize N=%d k=%d" % idx.shape)
    rp, col, val = A.symmetrize(torch.from_numpy(idx.astype(np.int32)).cuda(),
                                torch.from_numpy(P.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()


def _check_sym_equal(N, g, o):
    grp, gcol, gval = g
    orp, ocol, oval = o
    assert np.array_equal(grp, orp)
    assert np.array_equal(gcol, ocol)
    err = np.abs(gval.astype(np.float64) - oval).max() * 2 * N
    say("    max |2N dP_sym| = %.3g" % err)
    assert err <= parity.P_TOL


def test_symmetrize_hand_example(A):
    idx = np.array([[1, 2], [0, 2], [3, 1], [2, 0]], np.int32)
    P = np.array([[0.75, 0.25], [0.5, 0.5], [0.625, 0.375], [0.875, 0.125]])
    rp, col, val = _sym(A, idx, P)
    assert rp.tolist() == [0, 3, 5, 8, 10]
    assert col.tolist() == [1, 2, 3, 0, 2, 0, 1, 3, 0, 2]
    assert val.tolist() == [5 / 32, 1 / 32, 1 / 64, 5 / 32, 7 / 64, 1 / 32, 7 / 64, 3 / 16, 1 / 64, 3 / 16]


def test_symmetrize_two_points(A):
    rp, col, val = _sym(A, np.array([[1], [0]], np.int32), np.array([[1.0], [1.0]]))
    assert rp.tolist() == [0, 1, 2] and col.tolist() == [1, 0]
    assert val.tolist() == [0.5, 0.5]


def test_symmetrize_complete_graph(A, ora):
    # k = N - 1: every pair is both an own and a mirrored entry, so the union
    # is the complete graph and nnz = N (N - 1)
    rng = np.random.default_rng(15)
    N = 50
    idx = np.array([rng.permutation(np.delete(np.arange(N), i)) for i in range(N)], np.int32)
    P = rng.dirichlet(np.ones(N - 1), size=N)
    Pf = P.astype(np.float32)
    g = _sym(A, idx, Pf)
    assert g[0][-1] == N * (N - 1)
    _check_sym_equal(N, g, ora.symmetrize(idx, Pf.astype(np.float64)))


def test_symmetrize_csr_form_equals_fixed_k(A):
    # the same conditional rows given as fixed-k and as CSR: identical output
    rng = np.random.default_rng(17)
    N, k = 1200, 25
    idx = np.array([rng.choice(np.delete(np.arange(N), i), size=k, replace=False) for i in range(N)], np.int32)
    P = rng.dirichlet(np.ones(k), size=N).astype(np.float32)
    a = _sym(A, idx, P)
    ptr = torch.arange(0, N * k + 1, k, dtype=torch.int64, device="cuda")
    rp, c, v = A.symmetrize_csr(ptr, torch.from_numpy(idx.reshape(-1)).cuda(), torch.from_numpy(P.reshape(-1)).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(a[0], rp.cpu().numpy()) and np.array_equal(a[1], c.cpu().numpy())
    assert np.array_equal(a[2], v.cpu().numpy())


def test_symmetrize_on_oracle_rows_config1(A, ora):
    X = datagen.mixture_isotropic()
    idx, d2, _ = ora.knn(X, 90)
    P, _, _, _ = ora.calibrate(d2, 30.0)
    Pf = P.astype(np.float32)
    g = _sym(A, idx, Pf)
    o = ora.symmetrize(idx, Pf.astype(np.float64))
    _check_sym_equal(2000, g, o)
    assert abs(g[2].astype(np.float64).sum() - 1.0) < 1e-5


def test_symmetrize_hub_rows(A, ora):
    # every row points at node 0 and node 1: rows 0 and 1 collect N entries
    # (beyond the LDS path), exercising the in-place global sort
    rng = np.random.default_rng(12)
    N, k = 6000, 8
    idx = np.empty((N, k), np.int32)
    for i in range(N):
        others = rng.choice(N, size=k + 2, replace=False)
        others = [j for j in others if j not in (i, 0, 1)][: k - 2]
        row = [0, 1] + others if i > 1 else ([1 - i] + [j for j in rng.choice(np.arange(2, N), size=k - 1,
                                                                               replace=False)])
        idx[i] = row
    P = rng.dirichlet(np.ones(k), size=N)
    Pf = P.astype(np.float32)
    g = _sym(A, idx, Pf)
    o = ora.symmetrize(idx, Pf.astype(np.float64))
    _check_sym_equal(N, g, o)


@pytest.mark.parametrize("k,form", [(100, "fixed"), (200, "fixed"), (100, "csr")])
def test_symmetrize_heavy_tailed_in_degree(A, ora, k, form):
    # neighbour lists drawn with power-law popularity, as kNN graphs of
    # image-like data have (median in-degree far below k, a few rows listed
    # by thousands): many mirrored runs exceed the row caches (256 entries
    # for k <= 128, 1024 for k <= 256 and 512 for CSR input when emitting,
    # 1024 when counting), and a workgroup's rows share their mirrored runs
    rng = np.random.default_rng(14)
    N = 8000
    logw = -0.9 * np.log(np.arange(1, N + 1))[rng.permutation(N)]
    idx = np.empty((N, k), np.int32)
    for s in range(0, N, 1000):
        key = logw[None, :] + rng.gumbel(size=(min(1000, N - s), N))  # Gumbel top-k: sampling without replacement
        key[np.arange(key.shape[0]), np.arange(s, s + key.shape[0])] = -np.inf  # no self
        idx[s:s + key.shape[0]] = np.argpartition(-key, k, axis=1)[:, :k]
    deg = np.bincount(idx.ravel(), minlength=N)
    assert deg.max() > 1024 and ((deg > 256) & (deg <= 1024)).sum() >= 50
    P = rng.dirichlet(np.ones(k), size=N)
    Pf = P.astype(np.float32)
    if form == "fixed":
        g = _sym(A, idx, Pf)
    else:
        ptr = np.arange(0, N * k + 1, k, dtype=np.int64)
        rp, c, v = A.symmetrize_csr(torch.from_numpy(ptr).cuda(), torch.from_numpy(idx.ravel()).cuda(),
                                    torch.from_numpy(Pf.ravel()).cuda())
        torch.cuda.synchronize()
        g = (rp.cpu().numpy(), c.cpu().numpy(), v.cpu().numpy())
    o = ora.symmetrize(idx, Pf.astype(np.float64))
    _check_sym_equal(N, g, o)


def test_symmetrize_many_entries(A, ora):
    # 18 M conditional entries: past 4096 x 4096 keys the sort's tiles hold
    # several 4096-key chunks each (the staged scatter carries each digit's
    # position from chunk to chunk); the CSR is compared with the oracle's
    rng = np.random.default_rng(16)
    N, k = 200000, 90
    # row i lists (i + 1 + (a_i j + b_i) mod (N - 1)) mod N, j < k: distinct,
    # never i (a_i coprime to N - 1)
    a = rng.integers(1, N - 1, size=N)
    while True:
        bad = np.gcd(a, N - 1) != 1
        if not bad.any():
            break
        a[bad] = rng.integers(1, N - 1, size=bad.sum())
    b = rng.integers(0, N - 1, size=N)
    j = np.arange(k)
    idx = ((np.arange(N)[:, None] + 1 + (a[:, None] * j[None, :] + b[:, None]) % (N - 1)) % N).astype(np.int32)
    assert N * k > 4096 * 4096
    P = rng.dirichlet(np.ones(k), size=N)
    Pf = P.astype(np.float32)
    g = _sym(A, idx, Pf)
    o = ora.symmetrize(idx, Pf.astype(np.float64))
    _check_sym_equal(N, g, o)


def test_symmetrize_csr_variable_rows(A, ora):
    rng = np.random.default_rng(13)
    N = 3000
    lens = rng.integers(1, 40, size=N)
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([rng.choice(np.delete(np.arange(N), i), size=lens[i], replace=False)
                          for i in range(N)]).astype(np.int32)
    val = rng.uniform(0.01, 1.0, size=ptr[-1]).astype(np.float32)
    rp, c, v = A.symmetrize_csr(torch.from_numpy(ptr).cuda(), torch.from_numpy(col).cuda(),
                                torch.from_numpy(val).cuda())
    torch.cuda.synchronize()
    o = ora.symmetrize_csr(ptr, col, val.astype(np.float64), N)
    _check_sym_equal(N, (rp.cpu().numpy(), c.cpu().numpy(), v.cpu().numpy()), o)


def test_symmetrize_csr_empty_rows(A, ora):
    # empty rows at both ends and in runs, rows that only receive mirrored
    # entries, and rows that neither own nor receive any (row_ptr gaps)
    rng = np.random.default_rng(14)
    N = 2500
    lens = rng.integers(0, 12, size=N)
    lens[:3] = 0
    lens[-5:] = 0
    lens[700:900] = 0
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pool = np.arange(N // 2)  # columns only in the first half: the rest receive nothing
    col = np.concatenate([rng.choice(pool[pool != i], size=lens[i], replace=False)
                          for i in range(N)]).astype(np.int32)
    val = rng.uniform(0.01, 1.0, size=ptr[-1]).astype(np.float32)
    say("  symmetrize_csr N=%d nnz=%d" % (N, ptr[-1]))
    rp, c, v = A.symmetrize_csr(torch.from_numpy(ptr).cuda(), torch.from_numpy(col).cuda(),
                                torch.from_numpy(val).cuda())
    torch.cuda.synchronize()
    o = ora.symmetrize_csr(ptr, col, val.astype(np.float64), N)
    _check_sym_equal(N, (rp.cpu().numpy(), c.cpu().numpy(), v.cpu().numpy()), o)


def test_symmetrize_csr_no_entries(A):
    N = 40
    ptr = torch.zeros(N + 1, dtype=torch.int64, device="cuda")
    dummy_c = torch.zeros(1, dtype=torch.int32, device="cuda")
    dummy_v = torch.zeros(1, dtype=torch.float32, device="cuda")
    rp, c, v = A.symmetrize_csr(ptr, dummy_c, dummy_v)
    torch.cuda.synchronize()
    assert rp.cpu().tolist() == [0] * (N + 1)
    assert c.numel() == 0 and v.numel() == 0


def _pipeline_check(A, ora, X, mu, rows=None):
    N = X.shape[0]
    K = int(math.floor(3 * mu))
    Xt = torch.from_numpy(X).cuda()
    say("  pipeline N=%d D=%d mu=%g" % (N, X.shape[1], mu))
    r = A.similarity(Xt, mu)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in r.items()}
    # global properties at full size
    perp = parity.perplexity_of_rows(g["P"])
    ok = (g["flags"] & 4) == 0
    assert np.abs(perp[ok] - mu).max() <= parity.PERP_TOL
    assert np.abs(g["P"].astype(np.float64).sum(1) - 1).max() <= 1e-6
    assert abs(g["val"].astype(np.float64).sum() - 1.0) < 1e-4
    assert N * K <= len(g["val"]) <= 2 * N * K
    # oracle rows
    if rows is None:
        rows = np.arange(N, dtype=np.int32)
    o_idx, o_d2, o_nx = ora.knn(X, K, query_ids=rows)
    oP, ob, operp, ofl = ora.calibrate(o_d2, mu)
    ties, _ = parity.check_knn(X, rows, g["idx"][rows], g["d2"][rows], o_idx, o_d2, o_nx)
    dP = parity.check_p_rows(g["idx"][rows], g["P"][rows], o_idx, oP, o_d2, o_nx)
    say("    rows %d: ties %d, max|dP| %.3g, max|perp-mu| %.3g" % (len(rows), ties, dP, np.abs(perp - mu).max()))
    return g, (o_idx, o_d2, o_nx, oP)


def test_pipeline_config1_full(A, ora):
    X = datagen.mixture_isotropic()
    g, (o_idx, o_d2, o_nx, oP) = _pipeline_check(A, ora, X, 30.0)
    # symmetric P, compared as 2N * p_ij over the union, except entries whose
    # pair sits in a row's tie band (both sets are correct there)
    N, K = o_idx.shape
    band = set()
    dK = o_d2[:, K - 1]
    for i in range(N):
        if o_nx[i] <= dK[i] * (1 + parity.TIE_REL):
            for j in o_idx[i][o_d2[i] >= dK[i] * (1 - parity.TIE_REL)]:
                band.add((i, int(j)))
                band.add((int(j), i))
            for j in g["idx"][i]:
                band.add((i, int(j)))
                band.add((int(j), i))
    orp, ocol, oval = ora.symmetrize(o_idx, oP)
    gd = parity.csr_to_dict(g["row_ptr"], g["col"], g["val"])
    od = parity.csr_to_dict(orp, ocol, oval)
    worst = 0.0
    for key in set(gd) | set(od):
        if key in band:
            continue
        worst = max(worst, abs(gd.get(key, 0.0) - od.get(key, 0.0)) * 2 * N)
    say("    max |2N dP_sym| off the tie bands: %.3g (%d band pairs)" % (worst, len(band)))
    assert worst <= parity.P_TOL
