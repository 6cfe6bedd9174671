"""GPU serving loop (atsne_serve_*): continuous batching of inserts and
refines against a device-resident corpus."""
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


def _corpus(n=3000, d=50, seed=31):
    return datagen.mixture_isotropic(n=n, d=d, seed=seed)


def _standalone(A, X, ids, mu):
    """Same rows computed by the plain entry points on the same corpus prefix."""
    k = int(math.floor(3 * mu))
    Xt = torch.from_numpy(X).cuda()
    q = torch.from_numpy(np.asarray(ids, np.int32)).cuda()
    lo = torch.empty((len(ids), k), dtype=torch.float32, device="cuda")
    idx, d2, fl = A.knn(Xt, k, query_ids=q, d2_lo=lo)
    P, beta, perp, fl = A.calibrate_p(d2, mu, flags=fl, d2_lo=lo)
    torch.cuda.synchronize()
    return dict(idx=idx.cpu().numpy(), d2=d2.cpu().numpy(), P=P.cpu().numpy(), beta=beta.cpu().numpy())


def _same(a, b, keys=("idx", "d2", "P", "beta")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), "field %s differs" % k


def test_serve_refine_matches_standalone(A):
    X = _corpus()
    say("  serve: create N=%d" % X.shape[0])
    s = A.Server(torch.from_numpy(X).cuda(), 30.0)
    rng = np.random.default_rng(1)
    reqs = []
    for n, mu in [(1000, 10.0), (20, 30.0), (2500, 50.0), (333, 30.0), (1, 10.0), (1777, 50.0)]:
        ids = rng.choice(X.shape[0], size=n, replace=False).astype(np.int32)
        reqs.append((s.refine(ids, mu), ids, mu))
    for rid, ids, mu in reqs:
        r = s.wait(rid)
        assert r["status"] == 0 and r["kind"] == "refine"
        assert np.array_equal(r["row_ids"], ids)
        _same(r, _standalone(A, X, ids, mu))
        s.release(rid)
    st = s.stats()
    say("    stats %s" % st)
    assert st["completed"] == len(reqs) and st["max_requests_per_launch"] >= 2
    s.close()


def _run_sequence(A, X0, seq, mu0, wait_each):
    """Submit the sequence ('i', points) / ('r', ids, mu); returns results in order."""
    s = A.Server(torch.from_numpy(X0).cuda(), mu0, capacity_rows=X0.shape[0] + 5000)
    rids = []
    out = []
    for item in seq:
        if item[0] == "i":
            rid = s.insert(torch.from_numpy(item[1]).cuda())
        else:
            rid = s.refine(item[1], item[2])
        if wait_each:
            out.append(s.wait(rid))
            s.release(rid)
        else:
            rids.append(rid)
    for rid in rids:
        out.append(s.wait(rid))
        s.release(rid)
    snap = s.snapshot()
    st = s.stats()
    s.close()
    return out, snap, st


def _sequence(X0, rng, n_new):
    pts = datagen.mixture_isotropic(n=n_new, d=X0.shape[1], seed=77)
    seq = []
    off = 0
    n = X0.shape[0]
    for B, (m, mu) in zip([64, 400, 17, 1000, 250], [(500, 10.0), (1200, 30.0), (50, 50.0), (900, 30.0), (7, 10.0)]):
        seq.append(("r", rng.choice(n, size=m, replace=False).astype(np.int32), mu))
        seq.append(("i", pts[off:off + B]))
        off += B
        n += B
    return seq, np.concatenate([X0, pts[:off]])


def test_serve_alone_vs_mix_and_exact_state(A):
    X0 = _corpus(n=2500, seed=32)
    rng = np.random.default_rng(2)
    seq, Xfull = _sequence(X0, rng, 2000)
    say("  serve: %d requests, alone (one at a time)" % len(seq))
    alone, snap_a, st_a = _run_sequence(A, X0, seq, 30.0, wait_each=True)
    say("  serve: same requests in the mix")
    mix, snap_m, st_m = _run_sequence(A, X0, seq, 30.0, wait_each=False)
    say("    mix stats %s" % st_m)
    assert st_m["max_concurrent"] >= 2
    for a, b in zip(alone, mix):
        assert a["status"] == 0 and b["status"] == 0 and a["epoch"] == b["epoch"]
        _same(a, b, keys=("row_ids", "idx", "d2", "P", "beta", "flags"))
        if a["kind"] == "insert":
            assert sorted(a["changed"].tolist()) == sorted(b["changed"].tolist())
    assert np.array_equal(snap_a[1], snap_m[1]) and np.array_equal(snap_a[2], snap_m[2])
    # each request equals the plain entry points on its epoch's corpus prefix
    n = X0.shape[0]
    for item, r in zip(seq, alone):
        if item[0] == "r":
            _same(r, _standalone(A, Xfull[:n], item[1], item[2]))
        else:
            B = item[1].shape[0]
            ids = np.arange(n, n + B, dtype=np.int32)
            ref = _standalone(A, Xfull[:n + B], ids, 30.0)
            _same(r, ref, keys=("idx", "d2"))
            assert np.abs(r["P"] - ref["P"]).max() <= parity.P_TOL
            n += B
    # after the inserts, the resident lists are the exact kNN of the grown corpus
    assert np.array_equal(snap_a[0], Xfull)
    o_idx, o_d2, o_nx = O.get().knn(Xfull, 90)
    ties, _ = parity.check_knn(Xfull, np.arange(Xfull.shape[0]), snap_a[1], snap_a[2], o_idx, o_d2, o_nx)
    say("    final state vs oracle: %d tie-rule rows of %d" % (ties, Xfull.shape[0]))


def test_serve_budget_backpressure(A):
    X = _corpus(n=4000, seed=33)
    budget = 6 << 20
    s = A.Server(torch.from_numpy(X).cuda(), 30.0, hbm_budget_bytes=budget, max_slots=3)
    rng = np.random.default_rng(3)
    with pytest.raises(A.AtsneError) as e:
        s.refine(np.arange(4000, dtype=np.int32), 50.0)  # needs ~7 MB of results
    assert e.value.status == A.E_NOMEM
    rids = [s.refine(rng.choice(4000, size=1500, replace=False).astype(np.int32), 30.0) for _ in range(8)]
    for rid in rids:
        r = s.wait(rid)
        assert r["status"] == 0
        s.release(rid)
    st = s.stats()
    say("    budget stats %s" % st)
    assert st["peak_bytes_in_flight"] <= budget and st["max_concurrent"] <= 3
    s.close()


def test_serve_errors(A):
    X = _corpus(n=500, seed=34)
    s = A.Server(torch.from_numpy(X).cuda(), 10.0, capacity_rows=600)
    with pytest.raises(A.AtsneError):
        s.refine(np.array([0, 600], np.int32), 10.0)  # id outside the corpus
    with pytest.raises(A.AtsneError):
        s.refine(np.array([0], np.int32), 80.0)  # perplexity above the serving maximum
    with pytest.raises(A.AtsneError) as e:
        s.insert(torch.zeros((200, 50), device="cuda"))  # capacity 600 rows
    assert e.value.status == A.E_NOMEM
    s.close()


# ---------------------------------------------------------------------------
# Deletion and the sliding window (Sec. 5.3, Sec. 8) against the FP64 model
# ---------------------------------------------------------------------------
from oracle import serve_model as SM  # noqa: E402


def _run_ops(A, X0, mu0, ops, wait_each, capacity):
    """ops: ('i', points) / ('d', ids) / ('r', ids, mu).  Returns (results, snapshot, stats)."""
    s = A.Server(torch.from_numpy(X0).cuda(), mu0, capacity_rows=capacity)
    rids, out = [], []
    for op in ops:
        if op[0] == "i":
            rid = s.insert(torch.from_numpy(op[1]).cuda())
        elif op[0] == "d":
            rid = s.delete(op[1])
        else:
            rid = s.refine(op[1], op[2])
        if wait_each:
            out.append(s.wait(rid))
            s.release(rid)
        else:
            rids.append(rid)
    for rid in rids:
        out.append(s.wait(rid))
        s.release(rid)
    snap = s.snapshot()
    st = s.stats()
    s.close()
    return out, snap, st


def _check_against_model(m, snap, results, ops, label):
    X, idx, d2, P, beta, rho, alive = snap
    n = m.n_rows()
    assert X.shape[0] == n and np.array_equal(X, m.X)
    assert np.array_equal(alive.astype(bool), m.alive), "%s: alive flags" % label
    tie = np.zeros(n, bool)
    tie[list(m.tie_rows)] = True
    ok = ~tie
    # same listed set per row (the order of near-equal distances inside a list
    # may differ between FP32 and FP64), absent entries at the tail
    gs, ms = np.sort(idx, axis=1), np.sort(m.idx, axis=1)
    bad = np.flatnonzero(ok & (gs != ms).any(axis=1))
    for i in bad[:3]:
        say("    row %d: gpu %s / %s  model %s / %s" % (i, idx[i].tolist(), d2[i].tolist(), m.idx[i].tolist(),
                                                     m.d2[i].tolist()))
    assert bad.size == 0, "%s: listed sets differ in %d rows" % (label, bad.size)
    assert np.array_equal(rho[ok], m.rho()[ok].astype(np.float32))
    pres = idx >= 0
    assert np.all(pres[:, :-1] >= pres[:, 1:]), "absent entries must trail"
    dd = np.where(pres, d2, np.inf)
    with np.errstate(invalid="ignore"):
        assert np.all(np.diff(dd, axis=1)[pres[:, 1:]] >= 0), "listed distances not ascending"
    # FP32 direct-difference distances of the listed points
    td = parity.true_d2(m.X, np.arange(n), np.maximum(idx, 0))
    e = np.abs(d2[pres].astype(np.float64) - td[pres])
    assert np.all(e <= parity.D2_REL * td[pres] + 1e-30)
    assert np.all(np.isinf(d2[~pres]))
    # calibration over the listed neighbours, from the GPU's own distances
    o_P, o_beta, o_fl = SM.calibrate_absent(d2.astype(np.float64), m.mu)
    assert np.abs(P - o_P).max() <= parity.P_TOL, "%s: max |dP| %g" % (label, np.abs(P - o_P).max())
    few = np.isfinite(d2).sum(axis=1) <= m.mu  # uniform over the listed neighbours (or empty)
    assert np.all(beta[few] == 0.0)
    say("    %s: %d rows (%d alive, %d with removed neighbours, %d tie rows)" % (
        label, n, int(alive.sum()), int(((rho < 1) & (alive > 0)).sum()), int(tie.sum())))


def _mixed_ops(X0, seed):
    rng = np.random.default_rng(seed)
    pts = datagen.mixture_isotropic(n=1200, d=X0.shape[1], seed=seed + 1)
    ops, off = [], 0
    n, alive = X0.shape[0], np.ones(X0.shape[0], bool)
    for B, n_del, n_ref in [(64, 40, 300), (0, 400, 50), (300, 17, 0), (1, 1, 999), (500, 250, 20),
                            (100, 0, 700), (0, 60, 0)]:
        if B:
            ops.append(("i", pts[off:off + B]))
            off += B
            alive = np.concatenate([alive, np.ones(B, bool)])
        if n_del:
            # a mix of old points and points of the last insert
            ids = rng.choice(np.flatnonzero(alive), size=n_del, replace=False).astype(np.int32)
            ops.append(("d", ids))
            alive[ids] = False
        if n_ref:
            ids = rng.choice(np.flatnonzero(alive), size=n_ref, replace=False).astype(np.int32)
            ops.append(("r", ids, [10.0, 30.0, 50.0][n_ref % 3]))
    return ops


def test_serve_delete_alone_vs_mix_and_model(A):
    X0 = _corpus(n=2500, seed=35)
    mu0 = 10.0
    ops = _mixed_ops(X0, 8)
    cap = X0.shape[0] + 1200
    say("  serve+delete: %d requests, alone" % len(ops))
    alone, snap_a, _ = _run_ops(A, X0, mu0, ops, True, cap)
    say("  serve+delete: same requests in the mix")
    mix, snap_m, st = _run_ops(A, X0, mu0, ops, False, cap)
    say("    mix stats %s" % st)
    for op, a, b in zip(ops, alone, mix):
        assert a["status"] == 0 and b["status"] == 0 and a["epoch"] == b["epoch"]
        if op[0] == "d":
            assert a["kind"] == "delete" and sorted(a["changed"].tolist()) == sorted(b["changed"].tolist())
        else:
            _same(a, b, keys=("row_ids", "idx", "d2", "P", "beta", "flags"))
    for x, y in zip(snap_a, snap_m):
        assert np.array_equal(x, y)
    # the FP64 model replays the commits; refines are checked on the live subset
    m = SM.ResidentModel(X0, mu0)
    for op, r in zip(ops, alone):
        if op[0] == "i":
            ch = m.insert(op[1])
            got = np.sort(r["changed"])
            tie = np.array([i in m.tie_rows for i in range(m.n_rows())])
            assert np.array_equal(got[~tie[got]], ch[~tie[ch]]), "insert changed rows differ"
        elif op[0] == "d":
            ch = m.delete(op[1])
            assert np.array_equal(np.sort(r["changed"]), ch), "delete changed rows differ"
        else:
            live = np.flatnonzero(m.alive)
            pos = np.searchsorted(live, op[1]).astype(np.int32)
            ref = _standalone(A, m.X[live], pos, op[2])
            ref["idx"] = live[ref["idx"]].astype(np.int32)
            _same(r, ref)
    _check_against_model(m, snap_a, alone, ops, "final state")


def test_serve_sliding_window(A):
    """Stream readings through a window: each tick inserts the new readings
    and deletes the ones that left the window (Sec. 8)."""
    W, D, T, per_tick = 1500, 52, 120, 3
    stream = datagen.activity_stream(n=W + T * per_tick, d=D, seed=41)
    X0 = stream[:W]
    ops = []
    for t in range(T):
        a = W + t * per_tick
        ops.append(("i", stream[a:a + per_tick]))
        ops.append(("d", np.arange(t * per_tick, (t + 1) * per_tick, dtype=np.int32)))
    say("  sliding window W=%d, %d ticks of %d readings" % (W, T, per_tick))
    res, snap, st = _run_ops(A, X0, 10.0, ops, False, stream.shape[0])
    assert all(r["status"] == 0 for r in res)
    m = SM.ResidentModel(X0, 10.0)
    for op in ops:
        (m.insert if op[0] == "i" else m.delete)(op[1])
    assert int(m.alive.sum()) == W
    _check_against_model(m, snap, res, ops, "window")
    lat = np.array([r["t_complete_ms"] - r["t_submit_ms"] for r in res])
    say("    commit latency p50 %.2f ms p99 %.2f ms" % (np.percentile(lat, 50), np.percentile(lat, 99)))


def test_serve_delete_errors(A):
    X = _corpus(n=300, seed=36)
    s = A.Server(torch.from_numpy(X).cuda(), 10.0, capacity_rows=400)
    rid = s.delete(np.array([3, 7], np.int32))
    s.wait(rid)
    s.release(rid)
    for bad in ([3], [300], [-1], [5, 5]):  # deleted, outside, negative, duplicate
        with pytest.raises(A.AtsneError):
            s.delete(np.array(bad, np.int32))
    with pytest.raises(A.AtsneError):
        s.refine(np.array([0, 7], np.int32), 10.0)  # 7 was deleted
    with pytest.raises(A.AtsneError) as e:
        s.delete(np.arange(10, 280, dtype=np.int32))  # would leave fewer than K+1 live points
    assert e.value.status == A.E_K_RANGE
    r = s.wait(s.refine(np.array([0, 1], np.int32), 10.0))
    assert r["status"] == 0 and not np.isin(r["idx"], [3, 7]).any()
    s.release(r["req_id"])
    s.close()


# ---------------------------------------------------------------------------
# Operating size: requests split across launches, refine rows against the
# FP64 oracle, image-like corpus, failure of a batched launch
# ---------------------------------------------------------------------------
def _vs_oracle(X, r, ids, mu, sample=None, seed=0):
    """Refine rows against the oracle's exact kNN and calibration at mu on the
    request's corpus (all rows, or a seeded sample of them)."""
    ids = np.asarray(ids, np.int32)
    pos = np.arange(len(ids))
    if sample is not None and sample < len(ids):
        pos = np.sort(np.random.default_rng(seed).choice(len(ids), size=sample, replace=False))
    k = int(math.floor(3 * mu))
    o_idx, o_d2, o_nx = O.get().knn(X, k, query_ids=ids[pos])
    o_P, _, _, _ = O.get().calibrate(o_d2, mu)
    ties, _ = parity.check_knn(X, ids[pos], r["idx"][pos], r["d2"][pos], o_idx, o_d2, o_nx)
    dP = parity.check_p_rows(r["idx"][pos], r["P"][pos], o_idx, o_P, o_d2, o_nx)
    perp = parity.perplexity_of_rows(r["P"][pos])
    assert np.abs(perp - mu).max() <= parity.PERP_TOL
    return ties, dP


def test_serve_split_launches_vs_oracle(A):
    # 300-row launches: every request but the smallest spans several
    # launches on both batch slots; each result equals the plain entry
    # points bit for bit and the oracle within the parity rules
    X = _corpus(n=3000, seed=37)
    s = A.Server(torch.from_numpy(X).cuda(), 30.0, max_batch_rows=300)
    rng = np.random.default_rng(4)
    reqs = []
    for n, mu in [(1000, 10.0), (2500, 50.0), (299, 30.0), (300, 30.0), (301, 10.0), (7, 50.0), (1777, 30.0)]:
        ids = rng.choice(X.shape[0], size=n, replace=False).astype(np.int32)
        reqs.append((s.refine(ids, mu), ids, mu))
    for rid, ids, mu in reqs:
        r = s.wait(rid)
        assert r["status"] == 0 and np.array_equal(r["row_ids"], ids)
        _same(r, _standalone(A, X, ids, mu))
        ties, dP = _vs_oracle(X, r, ids, mu)
        say("    refine %d rows mu %g: tie-rule rows %d, max|dP| %.2g" % (len(ids), mu, ties, dP))
        s.release(rid)
    st = s.stats()
    say("    stats %s" % st)
    assert st["launches"] >= sum(len(x[1]) for x in reqs) // 300 and st["max_requests_per_launch"] >= 2
    s.close()


def test_serve_imagelike_alone_vs_mix(A):
    # an image-like corpus (D = 784) with refines larger than one launch
    # (8192 rows by default): the same requests alone and in the mix give the
    # same bits, and every refine matches the oracle on its corpus version
    X0 = datagen.image_like(n=20000, noise_seed=91)
    pts = datagen.image_like(n=2200, noise_seed=92)
    rng = np.random.default_rng(5)
    seq, n = [], X0.shape[0]
    for B, (m, mu) in zip([1500, 700, 0], [(10000, 30.0), (9000, 10.0), (12000, 50.0)]):
        seq.append(("r", rng.choice(n, size=m, replace=False).astype(np.int32), mu))
        if B:
            off = n - X0.shape[0]
            seq.append(("i", pts[off:off + B]))
            n += B
    say("  serve image-like: %d requests, alone" % len(seq))
    alone, snap_a, _ = _run_sequence_cap(A, X0, seq, 30.0, True, X0.shape[0] + 2300)
    say("  serve image-like: same requests in the mix")
    mix, snap_m, st = _run_sequence_cap(A, X0, seq, 30.0, False, X0.shape[0] + 2300)
    say("    mix stats %s" % st)
    assert st["max_concurrent"] >= 2 and st["launches"] >= 5
    for a, b in zip(alone, mix):
        assert a["status"] == 0 and b["status"] == 0 and a["epoch"] == b["epoch"]
        _same(a, b, keys=("row_ids", "idx", "d2", "P", "beta", "flags"))
    assert np.array_equal(snap_a[1], snap_m[1]) and np.array_equal(snap_a[3], snap_m[3])
    Xfull = np.concatenate([X0, pts[:n - X0.shape[0]]])
    n = X0.shape[0]
    for i, (item, r) in enumerate(zip(seq, alone)):
        if item[0] == "r":
            ties, dP = _vs_oracle(Xfull[:n], r, item[1], item[2], sample=300, seed=i)
            say("    refine %d rows mu %g vs oracle (300 sampled): tie-rule rows %d, max|dP| %.2g" % (
                len(item[1]), item[2], ties, dP))
        else:
            n += item[1].shape[0]


def _run_sequence_cap(A, X0, seq, mu0, wait_each, cap):
    s = A.Server(torch.from_numpy(X0).cuda(), mu0, capacity_rows=cap)
    rids, out = [], []
    for item in seq:
        rid = s.insert(torch.from_numpy(item[1]).cuda()) if item[0] == "i" else s.refine(item[1], item[2])
        if wait_each:
            out.append(s.wait(rid))
            s.release(rid)
        else:
            rids.append(rid)
    for rid in rids:
        out.append(s.wait(rid))
        s.release(rid)
    snap = s.snapshot()
    st = s.stats()
    s.close()
    return out, snap, st


def test_serve_failed_launch_fails_every_request(A, monkeypatch):
    # the second batched launch fails on the host before touching the device
    # (a forced E_NOMEM): every request in flight or queued completes with
    # that status once the streams have drained, later submissions and
    # snapshots are refused, and the server still shuts down
    import time

    X = _corpus(n=3000, seed=38)
    monkeypatch.setenv("ATSNE_SERVE_FAIL_LAUNCH", "2")
    s = A.Server(torch.from_numpy(X).cuda(), 30.0, max_batch_rows=300, capacity_rows=4000)
    monkeypatch.delenv("ATSNE_SERVE_FAIL_LAUNCH")
    rng = np.random.default_rng(6)
    # the failure can come before every submission is in: from then on a
    # submission is refused with the failure's status
    subs = [lambda: s.refine(rng.choice(3000, size=1000, replace=False).astype(np.int32), 30.0)] * 3
    subs += [lambda: s.insert(torch.from_numpy(_corpus(n=200, seed=39)).cuda()),
             lambda: s.refine(rng.choice(3000, size=50, replace=False).astype(np.int32), 10.0)]
    rids, refused = [], 0
    for sub in subs:
        try:
            rids.append(sub())
        except A.AtsneError as e:
            assert e.status == A.E_NOMEM
            refused += 1
    say("    accepted %d, refused %d" % (len(rids), refused))
    assert rids, "the first submission comes before any launch"
    deadline = time.time() + 60
    res = {}
    while len(res) < len(rids) and time.time() < deadline:
        for rid in rids:
            if rid not in res:
                r = s.poll(rid, fetch=False)
                if r is not None:
                    res[rid] = r
        time.sleep(0.01)
    assert len(res) == len(rids), "requests did not complete after a failed launch"
    st = [res[r]["status"] for r in rids]
    say("    statuses after the failed launch: %s" % st)
    assert all(x == A.E_NOMEM for x in st)
    with pytest.raises(A.AtsneError) as e:
        s.refine(np.array([0, 1], np.int32), 10.0)
    assert e.value.status == A.E_NOMEM
    with pytest.raises(A.AtsneError):
        s.snapshot()
    for rid in rids:
        s.release(rid)
    s.close(force=False)
