"""GPU kNN (atsne_knn / atsne_knn_subset) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1512_01655_amd import datagen
from tests import parity
from tests.gpu_common import lib, run_knn, say

pytestmark = pytest.mark.gpu
# the two exact contractions: FP32 MFMA and the BF16 hi/lo split (FP32X3)
EXACT = ["fp32", "fp32x3"]


@pytest.fixture(scope="module")
def A():
    return lib()


@pytest.fixture(scope="module")
def ora():
    return O.get()


def _compare(A, ora, X, k, prec="fp32", kc=0, qids=None, exact=False):
    g_idx, g_d2, g_fl = run_knn(A, X, k, prec, kc, qids)
    o_idx, o_d2, o_nx = ora.knn(X, k, query_ids=qids)
    rows = np.arange(X.shape[0]) if qids is None else np.asarray(qids)
    if exact:
        assert np.array_equal(g_idx, o_idx)
        assert np.array_equal(g_d2.astype(np.float64), o_d2)
        return g_fl
    ties, _ = parity.check_knn(X, rows, g_idx, g_d2, o_idx, o_d2, o_nx)
    say("    tie-rule rows %d / %d, fp64-reranked %d, exact-scan %d" % (
        ties, len(rows), int((g_fl & 1).sum()), int((g_fl & 8).sum() // 8)))
    return g_fl


@pytest.mark.parametrize("prec", EXACT)
@pytest.mark.parametrize("case", range(7))
def test_knn_small_ragged(A, ora, case, prec):
    X = datagen.small_cases()[case]
    N = X.shape[0]
    for k in sorted({1, 7, min(90, N - 1), N - 1}):
        _compare(A, ora, X, k, prec=prec)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_config1_full(A, ora, prec):
    X = datagen.mixture_isotropic()
    _compare(A, ora, X, 90, prec=prec)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_balanced_schedule_ragged(A, ora, prec):
    # 24 x 24 (query block, key tile) units of 256 rows, more than two per CU:
    # the balanced schedule, whose workgroups cross query blocks (segments run
    # by first tile), with a ragged last block and D off the chunk size
    X = datagen.mixture_isotropic(n=6001, d=37)
    _compare(A, ora, X, 90, prec=prec)


def test_knn_balanced_schedule_ragged_bf16(A, ora):
    X = datagen.mixture_isotropic(n=6001, d=37)
    g_idx, g_d2, g_fl = run_knn(A, X, 90, "bf16")
    o_idx, o_d2, o_nx = ora.knn(X, 90)
    rows = np.arange(X.shape[0])
    td = parity.check_rows_valid(X, rows, g_idx, g_d2)
    rec = O.recall(g_idx, o_idx, query_ids=rows, n=X.shape[0])
    say("    bf16 recall %.6f (tie-aware %.6f)" % (rec, parity.recall_tie_aware(td, o_d2, o_idx, g_idx)))
    assert rec >= 0.999


@pytest.mark.parametrize("prec", EXACT)
def test_knn_config1_kcand_equals_k(A, ora, prec):
    # no candidate margin: the certificate must route uncertain rows to the exact scan
    X = datagen.mixture_isotropic()
    _compare(A, ora, X, 90, prec=prec, kc=90)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_exact_scan_equals_certified(A, prec):
    # k_cand = k leaves no candidate margin, so most rows are redone by the
    # exact scan; the scan keeps the near-tie band past the k-th, so every
    # row (neighbours, distances, FP64 re-rank) ends bit for bit as with the
    # default margin, where rows are certified
    X = datagen.mixture_isotropic()
    a_idx, a_d2, a_fl = run_knn(A, X, 90, prec, 0)
    b_idx, b_d2, b_fl = run_knn(A, X, 90, prec, 90)
    n_scan = int(((b_fl & 8) > 0).sum())
    say("    exact-scan rows %d (margin 0) vs %d (default); fp64 rows %d / %d" % (
        n_scan, int(((a_fl & 8) > 0).sum()), int((a_fl & 1).sum()), int((b_fl & 1).sum())))
    assert n_scan > 100
    assert np.array_equal(a_idx, b_idx) and np.array_equal(a_d2, b_d2)
    assert np.array_equal(a_fl & 1, b_fl & 1)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_integer_ties_exact(A, ora, prec):
    # small integers: every distance is exact in FP32, so the (d, j) ranking,
    # ties included, must match bit for bit
    rng = np.random.default_rng(3)
    for N, D, k in [(300, 4, 20), (1000, 3, 50), (600, 40, 90)]:
        X = rng.integers(-3, 4, size=(N, D)).astype(np.float32)
        _compare(A, ora, X, k, prec=prec, exact=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "fp32x3"])
def test_knn_representable_exact_all_precisions(A, ora, prec):
    # integers in [-7, 7] with a 7 in every row are exact in FP32, BF16 and
    # (scale 7/448 = 2^-6) FP8 e4m3, so all three contractions are exact
    rng = np.random.default_rng(4)
    for N, D, k in [(700, 50, 30), (1300, 128, 90), (520, 200, 10)]:
        X = rng.integers(-7, 8, size=(N, D)).astype(np.float32)
        X[:, 0] = 7.0
        _compare(A, ora, X, k, prec=prec, exact=True)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_duplicates(A, ora, prec):
    rng = np.random.default_rng(5)
    base = rng.normal(size=(300, 16)).astype(np.float32)
    X = np.concatenate([base, base, base])[rng.permutation(900)]
    _compare(A, ora, X, 10, prec=prec, exact=False)
    g_idx, g_d2, _ = run_knn(A, X, 10, prec)
    o_idx, o_d2, _ = ora.knn(X, 10)
    assert np.array_equal(g_idx[:, :2], o_idx[:, :2])  # the two exact copies, lower index first
    assert np.all(g_d2[:, :2] == 0)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_all_equal(A, ora, prec):
    X = np.ones((600, 33), np.float32)
    g_idx, g_d2, g_fl = run_knn(A, X, 25, prec)
    for i in range(600):
        exp = [j for j in range(27) if j != i][:25]
        assert g_idx[i].tolist() == exp
    assert np.all(g_d2 == 0)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_subset(A, ora, prec):
    X = datagen.mixture_isotropic()
    q = np.random.default_rng(6).choice(2000, size=333, replace=False).astype(np.int32)
    _compare(A, ora, X, 90, prec=prec, qids=q)


@pytest.mark.parametrize("prec", EXACT + ["bf16", "fp8"])
def test_knn_subset_rows_equal_full_search(A, prec):
    # a row's result does not depend on the rows searched with it: the
    # subset search (few query blocks, small geometry, task grid) and the
    # full search (balanced schedule) give the same rows bit for bit
    X = datagen.mixture_isotropic(n=6001, d=37)
    q = np.random.default_rng(16).choice(6001, size=500, replace=False).astype(np.int32)
    f_idx, f_d2, f_fl = run_knn(A, X, 90, prec)
    s_idx, s_d2, s_fl = run_knn(A, X, 90, prec, qids=q)
    assert np.array_equal(s_idx, f_idx[q]) and np.array_equal(s_d2, f_d2[q])
    assert np.array_equal(s_fl & 1, f_fl[q] & 1)


def test_knn_fp32x3_equals_fp32_small_and_ragged(A):
    # the two exact contractions give the same rows bit for bit on the small
    # geometry (N = 2000) and the balanced schedule (N = 6001, D = 37)
    for X in (datagen.mixture_isotropic(), datagen.mixture_isotropic(n=6001, d=37)):
        a = run_knn(A, X, 90, "fp32")
        b = run_knn(A, X, 90, "fp32x3")
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("prec", EXACT + ["bf16"])
def test_knn_strided_rows_equal_contiguous(A, prec):
    # X as a view with row stride ld = D + 8 = 53 floats (odd, so rows start
    # off 16-byte boundaries) gives the rows of the contiguous copy bit for bit
    import torch

    X = datagen.mixture_isotropic(n=1500, d=45)
    big = torch.zeros((1500, 53), dtype=torch.float32, device="cuda")
    big[:, :45] = torch.from_numpy(X).cuda()
    view = big[:, :45]
    assert view.stride(0) == 53
    a = A.knn(view, 40, prec=prec)
    b = A.knn(torch.from_numpy(X).cuda(), 40, prec=prec)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_knn_all_candidates_equal_exact(A, prec):
    # with every key a candidate (k_cand = N - 1) the low-precision
    # contraction only orders the candidates, and the FP32 re-rank (FP64 for
    # near ties) returns the exact path's rows bit for bit
    X = datagen.mixture_isotropic(n=1000, d=40)
    a_idx, a_d2, a_fl = run_knn(A, X, 30, "fp32")
    b_idx, b_d2, b_fl = run_knn(A, X, 30, prec, kc=999)
    assert np.array_equal(a_idx, b_idx) and np.array_equal(a_d2, b_d2)
    assert np.array_equal(a_fl & 1, b_fl & 1)


@pytest.mark.parametrize("prec", EXACT)
def test_knn_subset_repeated_ids(A, prec):
    # a query id listed several times gets the same row each time
    X = datagen.mixture_isotropic()
    q = np.array([5, 5, 17, 5, 1999, 17, 0], np.int32)
    idx, d2, fl = run_knn(A, X, 90, prec, qids=q)
    f_idx, f_d2, f_fl = run_knn(A, X, 90, prec)
    assert np.array_equal(idx, f_idx[q]) and np.array_equal(d2, f_d2[q])


@pytest.mark.parametrize("prec", EXACT)
@pytest.mark.parametrize("N,D,k,kc", [(2, 5, 1, 0), (3, 2, 2, 0), (500, 1, 90, 0), (260, 65536, 10, 0),
                                      (1100, 16, 1000, 1024)])
def test_knn_extremes(A, ora, N, D, k, kc, prec):
    # the entry's limits: the fewest rows (N = 2, 3), one dimension (D = 1:
    # near ties everywhere), the largest D (65536: 2048 chunks per tile), the
    # largest k (1000) with the largest candidate count (1024)
    X = np.random.default_rng(N + D).normal(size=(N, D)).astype(np.float32)
    _compare(A, ora, X, k, prec=prec, kc=kc)


@pytest.mark.parametrize("prec", EXACT + ["bf16", "fp8"])
def test_knn_subset_empty(A, prec):
    # no query rows: empty outputs, nothing launched that reads them
    X = datagen.mixture_isotropic(n=600, d=20)
    idx, d2, fl = run_knn(A, X, 10, prec, qids=np.zeros(0, np.int32))
    assert idx.shape == (0, 10) and d2.shape == (0, 10) and fl.shape == (0,)


def run_knn_seed_count(A, X, seeded):
    # with kernel timing on, the seeding pass shows as one "seed_total"
    # record, plus an empty "seed_declined" one when it stepped aside (its
    # results unused), which would make the comparison vacuous
    A.profile_enable(True)
    try:
        out = run_knn(A, X, 150, "fp8", 300)
        assert A.profile_read("seed_total")[1] - A.profile_read("seed_declined")[1] == seeded
    finally:
        A.profile_enable(False)
    return out


def test_knn_fp8_seeded_equals_unseeded(A, monkeypatch):
    # a full FP8 search of at least 2^18 rows first bounds each row's k'-th
    # key code from the keys near it; rows, distances and flags are those of
    # the search without that pass, bit for bit
    X = datagen.mixture_anisotropic(n=300000)
    a = run_knn_seed_count(A, X, 1)
    monkeypatch.setenv("ATSNE_FP8_SEED", "0")
    b = run_knn_seed_count(A, X, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_knn_fp8_seeded_equals_unseeded_with_ties(A, monkeypatch):
    # 2^18 rows drawn from 2000 prototypes: every row has ~130 exact
    # duplicates, so many keys share the k'-th key code exactly; the seeded
    # threshold keeps every key at or below it and the rows stay bit-identical
    rng = np.random.default_rng(21)
    proto = rng.normal(size=(2000, 64)).astype(np.float32)
    X = proto[rng.integers(0, 2000, size=1 << 18)]
    a = run_knn_seed_count(A, X, 1)
    monkeypatch.setenv("ATSNE_FP8_SEED", "0")
    b = run_knn_seed_count(A, X, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_knn_fp8_seeding_declines_on_one_cell(A, monkeypatch):
    # the seeding partition starts from the rows c N / C (C = N / 1000
    # cells); when they all hold the same point every row joins one cell,
    # the lists would cover every row pair, and the pass steps aside: the
    # search runs unseeded, with the unseeded results
    N = 1 << 18
    C = N // 1000
    X = np.random.default_rng(23).normal(size=(N, 32)).astype(np.float32)
    X[(np.arange(C) * N) // C] = X[0]
    A.profile_enable(True)
    try:
        a = run_knn(A, X, 30, "fp8", 60)
        assert A.profile_read("seed_total")[1] == 1
        assert A.profile_read("seed_declined")[1] == 1
    finally:
        A.profile_enable(False)
    monkeypatch.setenv("ATSNE_FP8_SEED", "0")
    b = run_knn(A, X, 30, "fp8", 60)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_knn_errors(A):
    import torch

    X = torch.zeros((10, 4), device="cuda")
    with pytest.raises(A.AtsneError) as e:
        A.knn(X, 10)
    assert e.value.status == A.E_K_RANGE
    with pytest.raises(A.AtsneError) as e:
        A.knn(X, 3, k_cand=2)
    assert e.value.status == A.E_K_RANGE
