"""Benchmark of the A-tSNE high-dimensional similarity path on one MI355X.

A step is one pass of the whole path over the image-shaped workload
(N = 70000 points, D = 784, perplexity 30, K = 90): exact kNN
(atsne_knn, FP32 contraction) -> perplexity calibration (atsne_calibrate_p)
-> symmetrisation (atsne_symmetrize), inputs resident in HBM.  The metric is
points per second of the whole step.  The same line carries the BF16
contraction + FP32 re-rank variant, the roofline of the dominant kernel
(knn_tile, timed with HIP events on its own stream inside the timed
region), per-stage times, and the FP64 CPU oracle timed on a bounded sample
of the same workload on the host cores.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload imagelike|mixture]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}  # dense MFMA TFLOP/s, MI355X
PEAK_HBM_GBS = 8000.0  # HBM3E, MI355X


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="imagelike", choices=["imagelike", "mixture", "aniso"])
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 precision-at-scale leg (N = 10^6)")
    ap.add_argument("--path-only", action="store_true",
                    help="only the FP32 and BF16 steps (no approximate, attractive, ordering, serving legs): the "
                         "command the kernel-trace profile runs")
    ap.add_argument("--profile-kernel", default=None, choices=["fp32", "bf16", "fp8", "fp32x3"],
                    help="profiling mode: one warm-up and one timed kNN at this precision, then a 1 GiB device "
                         "copy (the reference kernel for scaling HBM byte counters); prints the launch shapes")
    ap.add_argument("--serve-rate", type=float, default=25.0, help="Poisson request rate (req/s)")
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-sweep", default=None,
                    help="comma-separated rates (req/s): only the serving sweep, one JSON line per rate "
                         "(--sweep-requests measured after --sweep-warmup)")
    ap.add_argument("--sweep-requests", type=int, default=2000)
    ap.add_argument("--sweep-warmup", type=int, default=100)
    ap.add_argument("--sweep-insert-points", default="64,4096",
                    help="inclusive range of points per insert request in the sweep (the survey's mix: 64,4096)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target length of the oracle sample")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_1512_01655_amd/csrc/knn.hip", "paper_1512_01655_amd/csrc/wave.h",
                  "paper_1512_01655_amd/csrc/knn_internal.h", "paper_1512_01655_amd/csrc/common.h"]
TRAFFIC_FILE = "profiles/knn_tile_traffic.txt"
TRAFFIC_NOTE = ("rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, measured by the builder on these kernel sources "
                "(profiles/knn_tile_traffic.txt, keyed by source hash); null when the sources changed since")


def kernel_source_hash():
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec):
    """HBM bytes per knn_tile launch from the committed counter summary, or
    None when it was taken on other kernel sources or another workload."""
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    key = "%s_%s_bytes_per_launch" % (workload, prec)
    return int(float(rec[key])) if key in rec else None


def run_path(A, torch, Xt, mu, k, prec, steps, warmup):
    """Warm up, then time `steps` whole-path steps; returns timing dict and last outputs."""
    N, D = Xt.shape
    ws = torch.empty(A.knn_workspace_size(N, N, D, k, prec), dtype=torch.uint8, device="cuda")
    lo = torch.empty((N, k), dtype=torch.float32, device="cuda")
    out = None
    for _ in range(warmup):
        idx, d2, fl = A.knn(Xt, k, prec=prec, workspace=ws, d2_lo=lo)
        P, beta, perp, fl = A.calibrate_p(d2, mu, flags=fl, d2_lo=lo)
        out = A.symmetrize(idx, P)
    torch.cuda.synchronize()
    A.profile_enable(True)
    t0 = time.perf_counter()
    for s in range(steps):
        idx, d2, fl = A.knn(Xt, k, prec=prec, workspace=ws, d2_lo=lo)
        P, beta, perp, fl = A.calibrate_p(d2, mu, flags=fl, d2_lo=lo)
        rp, col, val = A.symmetrize(idx, P)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = {}
    for name in ["seed_total", "knn_prep", "knn_tile", "knn_select", "knn_scan", "calibrate_rows", "sym_total"]:
        ms, n = A.profile_read(name)
        if n or name != "seed_total":  # the FP8 seeding pass runs only on large FP8 searches
            stages[name] = (ms, n)
    A.profile_enable(False)
    flags = fl.cpu().numpy()
    return dict(wall=wall, stages=stages, idx=idx, d2=d2, P=P, beta=beta, rp=rp, col=col, val=val, flags=flags)


def attractive_leg(A, torch, rp, col, val, reps=50, warm=5, seed=7):
    """Attractive forces (Eq. 7) over the step's symmetric P with a random 2-D
    embedding and 10% of points under selective exaggeration.  HBM bytes per
    launch: the CSR stream (8 B per entry + 8 B per row pointer), the
    embedding read once and the forces written (8 B per point each), and the
    refinement iterations (4 B per point)."""
    N = rp.shape[0] - 1
    nnz = int(col.shape[0])
    rng = np.random.default_rng(seed)
    Y = torch.from_numpy((rng.normal(size=(N, 2)) * 20.0).astype(np.float32)).cuda()
    t_ref = torch.from_numpy(np.where(rng.random(N) < 0.1, rng.integers(0, 100, N), -1).astype(np.int32)).cuda()
    F = torch.empty((N, 2), dtype=torch.float32, device="cuda")
    for _ in range(warm):
        A.attractive_forces(rp, col, val, Y, t_ref=t_ref, tau=12.0, decay=25.0, t_now=100, out=F)
    torch.cuda.synchronize()
    A.profile_enable(True)
    for _ in range(reps):
        A.attractive_forces(rp, col, val, Y, t_ref=t_ref, tau=12.0, decay=25.0, t_now=100, out=F)
    torch.cuda.synchronize()
    ms, n = A.profile_read("attractive_rows")
    A.profile_enable(False)
    avg_s = ms / max(n, 1) * 1e-3
    nbytes = nnz * 8 + (N + 1) * 8 + N * 8 * 2 + N * 4
    gbs = nbytes / avg_s / 1e9
    return {"N": N, "nnz": nnz, "avg_launch_ms": round(avg_s * 1e3, 4), "points_per_s": round(N / avg_s, 1),
            "roofline": {"bound": "hbm", "kernel": "attractive_rows", "achieved": round(gbs, 1),
                         "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                         "traffic": None, "algorithmic_bytes": nbytes}}


def order_leg(A, torch, idx, d2, beta, reps=5, seed=9):
    """Refinement orderings (Sec. 5.1) on the step's kNN graph: density order of
    all points, and the breadth-first visit (hops and path length) from 16
    seeds.  Wall time per call, synchronisations included."""
    rng = np.random.default_rng(seed)
    seeds = torch.from_numpy(rng.choice(idx.shape[0], size=16, replace=False).astype(np.int32)).cuda()
    out = {}
    for name, fn in [("density_ms", lambda: A.order_density(beta)),
                     ("bfs_hops_ms", lambda: A.order_neighbourhood(idx, None, seeds)),
                     ("bfs_path_length_ms", lambda: A.order_neighbourhood(idx, d2, seeds, weighted=True))]:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        out[name] = round((time.perf_counter() - t0) / reps * 1e3, 3)
    out["reached_from_16_seeds"] = int(r[0].shape[0])
    return out


def rows_valid(torch, idx, d2, n):
    """Every row lists distinct ids in [0, n), never its own row (rows are
    queries 0..M-1 of the corpus), with distances ascending."""
    M = idx.shape[0]
    own = torch.arange(M, device=idx.device, dtype=idx.dtype)[:, None]
    srt = idx.sort(dim=1).values
    ok = bool(((idx >= 0) & (idx < n)).all().item()) and not bool((idx == own).any().item())
    ok = ok and not bool((srt[:, 1:] == srt[:, :-1]).any().item())
    return ok and bool((d2[:, 1:] >= d2[:, :-1]).all().item())


def precision_eq9(torch, approx, exact, chunk=4096):
    """Eq. 9: mean over rows of |N^A_i & N_i| / K; each listed id counts once
    (a repeated id of an approximate row is not a second hit)."""
    hits = 0
    for s in range(0, exact.shape[0], chunk):
        a, e = approx[s:s + chunk], exact[s:s + chunk]
        a_s = a.sort(dim=1).values
        first = torch.ones_like(a_s, dtype=torch.bool)
        first[:, 1:] = a_s[:, 1:] != a_s[:, :-1]
        hit = ((a_s[:, :, None] == e[:, None, :]) & (a_s[:, :, None] >= 0)).any(dim=2) & first
        hits += int(hit.sum().item())
    return hits / float(exact.numel())


def host_recall(g_idx, o_idx):
    """Eq. 9 on host arrays whose rows are already validated (distinct ids)."""
    return sum(len(set(a) & set(b)) for a, b in zip(g_idx.tolist(), o_idx.tolist())) / float(o_idx.size)


def union_dP(g_idx, g_P, o_idx, o_P):
    """max over rows of |p_gpu - p_oracle| over the union of the two rows'
    supports, an entry missing from one side counting as 0."""
    M, K = o_idx.shape
    r = np.repeat(np.arange(M, dtype=np.int64), K)
    n = int(max(g_idx.max(), o_idx.max())) + 1
    gk = r * n + g_idx.reshape(-1).astype(np.int64)
    ok = r * n + o_idx.reshape(-1).astype(np.int64)
    keys = np.union1d(gk, ok)
    gv = np.zeros(keys.shape)
    ov = np.zeros(keys.shape)
    gv[np.searchsorted(keys, gk)] = g_P.reshape(-1)
    ov[np.searchsorted(keys, ok)] = o_P.reshape(-1)
    return float(np.abs(gv - ov).max())


def vs_oracle(g_idx, g_P, o):
    """a8 metrics of GPU rows against the oracle's rows of the same queries."""
    same = sum(set(a) == set(b) for a, b in zip(g_idx.tolist(), o["idx"].tolist()))
    return {"oracle_rows": int(o["idx"].shape[0]), "recall_vs_oracle": round(host_recall(g_idx, o["idx"]), 6),
            "rows_with_oracle_set": int(same),
            "max_abs_dP_cond_vs_oracle": float("%.4g" % union_dP(g_idx, g_P.astype(np.float64), o["idx"], o["P"]))}


def fp8_scale_leg(A, torch, datagen, steps=2, warmup=1, sample=10000, seed=13):
    """Precision at scale: N = 10^6, D = 128 anisotropic mixture, mu = 50, k = 150, FP8 e4m3 contraction with
    per-row scales and an FP32 re-rank of 2k = 300 candidates.  Whole-path points/s and the tile against the FP8
    matrix-core peak; the rows of a seeded sample are kept for the comparison with the FP64 oracle."""
    X = datagen.mixture_anisotropic()
    N, D = X.shape
    mu, k = 50.0, 150
    Xt = torch.from_numpy(X).cuda()
    r = run_path(A, torch, Xt, mu, k, "fp8", steps, warmup)
    value = N * steps / r["wall"]
    t_ms, t_n = r["stages"]["knn_tile"]
    t_avg = t_ms / max(t_n, 1) * 1e-3
    ach = 2.0 * N * N * D * steps / max(t_n, 1) / t_avg / 1e12
    rows = np.sort(np.random.default_rng(seed).choice(N, size=sample, replace=False)).astype(np.int32)
    q = torch.from_numpy(rows.astype(np.int64)).cuda()
    valid = rows_valid(torch, r["idx"], r["d2"], N)
    kept = {"X": X, "rows": rows, "idx": r["idx"][q].cpu().numpy(), "P": r["P"][q].cpu().numpy()}
    out = {
        "workload": "aniso50_N1000000_D128_mu50_k150", "k_cand": 2 * k, "value": round(value, 1),
        "ms_per_step": round(1e3 * r["wall"] / steps, 3),
        "stages_ms": {kname: round(v[0] / steps, 3) for kname, v in r["stages"].items()},
        "roofline": {"bound": "mfma", "kernel": "knn_tile", "achieved": round(ach, 2), "peak": PEAK["fp8"],
                     "unit": "TFLOP/s", "frac": round(ach / PEAK["fp8"], 4),
                     "traffic": measured_traffic("aniso", "fp8"),
                     "traffic_source": TRAFFIC_NOTE,
                     "algorithmic": "2*N*D FLOP per query point x N queries per step, N=%d, D=%d" % (N, D)},
        "rows_valid": valid,
    }
    del r, Xt
    torch.cuda.empty_cache()
    return out, kept


def approx_leg(A, torch, Xt, mu, k, exact_idx, exact_value, rho=0.9, C=256, iters=8, steps=5, seed=11):
    """Precision-controlled path: cluster-pruned kNN with n_probe fitted to rho
    on 16 sample clusters, then calibration and symmetrisation.  Precision
    (Eq. 9) is measured on every row against the exact path's neighbours."""
    N = Xt.shape[0]
    rng = np.random.default_rng(seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = A.IVF(Xt, C, iters=iters, init_ids=rng.choice(N, size=C, replace=False))
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    n_probe, rho_s = ix.fit(k, rho, rng.choice(C, size=16, replace=False))
    t_fit = time.perf_counter() - t0
    idx, d2, fl, frac = ix.knn(k, n_probe)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        idx, d2, fl, frac = ix.knn(k, n_probe)
        P, beta, perp, fl = A.calibrate_p(d2, mu, flags=fl)
        A.symmetrize(idx, P)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    rho_all = precision_eq9(torch, idx, exact_idx)
    ix.close()
    return {"rho_target": rho, "n_clusters": C, "kmeans_iters": iters, "n_probe": n_probe,
            "rho_sample": round(rho_s, 4), "rho_all_rows": round(rho_all, 4),
            "candidate_fraction": round(frac, 4), "build_ms": round(t_build * 1e3, 2), "fit_ms": round(t_fit * 1e3, 2),
            "ms_per_step": round(t_step * 1e3, 3), "value": round(N / t_step, 1),
            "speedup_vs_exact": round(N / t_step / exact_value, 3),
            "step": "cluster-pruned kNN + calibrate + symmetrize (build and fit excluded, reported apart)"}


def serve_load(A, torch, X, rate, n_req, n_warm, seed=5, pool_cache=None, progress=0, insert_points=(64, 4096)):
    """Poisson stream against a server holding X: half inserts of 64-4096 new
    points (same generator, fresh noise), half refines of 1000-20000 resident
    ids at perplexity 10, 30 or 50.  Latency = completion - the client's call.
    The request sequence depends on the seed only, so runs at several rates
    share it (and the insert pool, through pool_cache)."""
    import threading

    from paper_1512_01655_amd import datagen

    rng = np.random.default_rng(seed)
    kinds = rng.random(n_req) < 0.5
    sizes = np.where(kinds, rng.integers(insert_points[0], insert_points[1] + 1, n_req),
                     rng.integers(1000, 20001, n_req))
    mus = rng.choice([10.0, 30.0, 50.0], n_req)
    gaps = rng.exponential(1.0 / rate, n_req)
    n_new = int(sizes[kinds].sum())
    key = (seed, n_req, tuple(insert_points))
    if pool_cache is not None and key in pool_cache:
        pool = pool_cache[key]
    else:
        pool = torch.from_numpy(datagen.image_like(n=max(n_new, 1), noise_seed=seed + 1000)).cuda()
        if pool_cache is not None:
            pool_cache[key] = pool
    srv = A.Server(torch.from_numpy(X).cuda(), 30.0, capacity_rows=X.shape[0] + n_new + 1)
    rids, lat, rows = [], [], []
    done = threading.Event()
    t0 = time.perf_counter()

    def collect():
        i = 0
        while i < n_req:
            while i >= len(rids):
                time.sleep(0.0005)
            r = srv.wait(rids[i], fetch=False)
            if r["status"] != 0:
                raise RuntimeError("request failed: %s" % r)
            lat.append(r["t_complete_ms"] - r["t_submit_ms"])
            rows.append(r["n_rows"])
            srv.release(rids[i])
            i += 1
            if progress and i % progress == 0:
                log("  serve %.0f req/s: %d / %d complete, %.0f s, last latency %.0f ms" % (
                    rate, i, n_req, time.perf_counter() - t0, lat[-1]))
        done.set()

    th = threading.Thread(target=collect)
    th.start()
    off = 0
    corpus_n = X.shape[0]
    t_start = time.perf_counter()
    t_next = t_start
    t_first = None
    for i in range(n_req):
        t_next += gaps[i]
        while time.perf_counter() < t_next:
            time.sleep(0.0002)
        if i == n_warm:
            t_first = time.perf_counter()
        if kinds[i]:
            B = int(sizes[i])
            rids.append(srv.insert(pool[off:off + B]))
            off += B
            corpus_n += B
        else:
            ids = rng.choice(corpus_n, size=int(sizes[i]), replace=False).astype(np.int32)
            rids.append(srv.refine(ids, float(mus[i])))
    done.wait()
    th.join()
    t_end = time.perf_counter()
    st = srv.stats()
    srv.close()
    lat_m = np.array(lat[n_warm:])
    rows_m = np.array(rows[n_warm:])
    kind_m = kinds[n_warm:]
    span = t_end - t_first

    def pct(a, q):
        return round(float(np.percentile(a, q)), 2) if len(a) else None

    return {
        "rate_req_s": rate, "requests": n_req - n_warm, "warmup_requests": n_warm,
        "p50_ms": pct(lat_m, 50), "p99_ms": pct(lat_m, 99),
        "insert_p50_ms": pct(lat_m[kind_m], 50), "insert_p99_ms": pct(lat_m[kind_m], 99),
        "refine_p50_ms": pct(lat_m[~kind_m], 50), "refine_p99_ms": pct(lat_m[~kind_m], 99),
        "mean_ms": round(float(lat_m.mean()), 2), "throughput_req_s": round((n_req - n_warm) / span, 2),
        "arrival_span_s": round(float(gaps[n_warm:].sum()), 1), "measured_span_s": round(span, 1),
        "rows_per_s": round(float(rows_m.sum()) / span, 1),
        "mix": "0.5 insert (%d-%d points) / 0.5 refine (1000-20000 ids, mu in {10,30,50})" % tuple(insert_points),
        "corpus_rows_start": int(X.shape[0]), "corpus_rows_end": int(st["corpus_rows"]),
        "launches": int(st["launches"]), "max_requests_per_launch": int(st["max_requests_per_launch"]),
        "max_concurrent": int(st["max_concurrent"]),
    }


def window_stream(A, torch, W=6000, D=52, ticks=400, warm=40, mu=30.0, seed=41):
    """Sliding window of Sec. 8 on a synthetic activity stream: the window
    keeps the last W readings; each tick inserts the new reading and deletes
    the one that left the window.  Ticks run closed-loop (submit insert and
    delete, wait for both); tick latency = delete completion - insert
    submission, against the stream's 100 ms reading period."""
    from paper_1512_01655_amd import datagen

    stream = datagen.activity_stream(n=W + ticks, d=D, seed=seed)
    dev = torch.from_numpy(stream).cuda()
    srv = A.Server(dev[:W].contiguous(), mu, capacity_rows=W + ticks + 1)
    lat = []
    t_first = None
    for t in range(ticks):
        if t == warm:
            t_first = time.perf_counter()
        ri = srv.insert(dev[W + t:W + t + 1])
        rd = srv.delete(np.array([t], np.int32))
        r1 = srv.wait(ri, fetch=False)
        r2 = srv.wait(rd, fetch=False)
        if r1["status"] != 0 or r2["status"] != 0:
            raise RuntimeError("window tick %d failed" % t)
        lat.append(r2["t_complete_ms"] - r1["t_submit_ms"])
        srv.release(ri)
        srv.release(rd)
    span = time.perf_counter() - t_first
    srv.close()
    lm = np.array(lat[warm:])
    return {
        "window": W, "dims": D, "perplexity": mu, "ticks": ticks - warm, "warmup_ticks": warm,
        "tick_p50_ms": round(float(np.percentile(lm, 50)), 3), "tick_p99_ms": round(float(np.percentile(lm, 99)), 3),
        "ticks_per_s": round((ticks - warm) / span, 1), "reading_period_ms": 100.0,
        "data": "synthetic activity stream (24 activities, AR(1) drift), 1 insert + 1 delete per tick",
    }


def cpu_baseline(X, mu, k, target_s):
    """The FP64 oracle (exact kNN against the full corpus + bisection) timed on
    a seeded sample of query rows sized to about target_s seconds on the host
    cores.  Returns the baseline record and the oracle's rows (the precision
    metrics compare the GPU paths with them)."""
    from oracle import oracle as O

    o = O.get()
    cores = o.max_threads()
    rng = np.random.default_rng(12345)
    probe = rng.choice(X.shape[0], size=64, replace=False).astype(np.int32)
    t0 = time.perf_counter()
    _, d2, _ = o.knn(X, k, query_ids=probe)
    o.calibrate(d2, mu)
    rate = 64 / (time.perf_counter() - t0)
    m = int(min(X.shape[0], max(64, rate * target_s)))
    rows = np.sort(rng.choice(X.shape[0], size=m, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    idx, d2, nx = o.knn(X, k, query_ids=rows)
    t1 = time.perf_counter()
    P, _, _, _ = o.calibrate(d2, mu)
    dt = time.perf_counter() - t0
    rec = {"value": m / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
           "sample": "%d of %d query rows: FP64 exact kNN against the full corpus + bisection, %.1f s" % (
               m, X.shape[0], dt),
           "stages_s": {"knn": round(t1 - t0, 3), "calibrate": round(dt - (t1 - t0), 3)},
           "cpu_model": host_cpu_model()}
    return rec, {"rows": rows, "idx": idx, "d2": d2, "nx": nx, "P": P}


def host_cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or null where unreadable."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_rows(X, k, mu, rows):
    """The FP64 oracle's rows for the sampled queries of the FP8 leg (timed)."""
    from oracle import oracle as O

    o = O.get()
    t0 = time.perf_counter()
    idx, d2, nx = o.knn(X, k, query_ids=rows)
    P, _, _, _ = o.calibrate(d2, mu)
    dt = time.perf_counter() - t0
    return {"rows": rows, "idx": idx, "d2": d2, "nx": nx, "P": P, "seconds": dt, "cores": o.max_threads()}


def exact_vs_oracle(g_idx, g_d2, g_P, o, rel=1e-5):
    """The exact path on the oracle's sample rows: rows outside the tie rule
    must have the oracle's set; P compared entry by entry where the sets agree."""
    K = o["idx"].shape[1]
    dK = o["d2"][:, K - 1]
    tie = o["nx"] <= dK * (1 + rel)
    mism = 0
    worst = 0.0
    for r in range(g_idx.shape[0]):
        a, b = g_idx[r].tolist(), o["idx"][r].tolist()
        if set(a) != set(b):
            mism += 0 if tie[r] else 1
            continue
        gm = dict(zip(a, g_P[r].tolist()))
        worst = max(worst, max(abs(gm[j] - p) for j, p in zip(b, o["P"][r].tolist())))
    return {"oracle_rows": int(g_idx.shape[0]), "tie_rule_rows": int(tie.sum()), "set_mismatch_rows": mism,
            "max_abs_dP_cond_vs_oracle": float("%.4g" % worst)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (the path would shard by "
              "query rows)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1512_01655_amd import atsne as A
    from paper_1512_01655_amd import datagen

    A.load()
    if a.serve_sweep:
        X = datagen.image_like()
        cache = {}
        for rate in [float(v) for v in a.serve_sweep.split(",")]:
            log("serve sweep: %.0f req/s, %d requests after %d warm-up ..." % (rate, a.sweep_requests,
                                                                             a.sweep_warmup))
            ins = tuple(int(v) for v in a.sweep_insert_points.split(","))
            rec = serve_load(A, torch, X, rate, a.sweep_requests + a.sweep_warmup, a.sweep_warmup, pool_cache=cache,
                             progress=100, insert_points=ins)
            rec["scheduler"] = "launch-batched (host worker, continuous batching)"
            print(json.dumps({"serve_sweep": rec}), flush=True)
        return
    if a.workload == "imagelike":
        X = datagen.image_like()
        name = "imagelike_N70000_D784_mu30_k90"
    elif a.workload == "mixture":
        X = datagen.mixture_isotropic()
        name = "mixture10_N2000_D50_mu30_k90"
    else:
        X = datagen.mixture_anisotropic()
        name = "aniso50_N1000000_D128_mu50_k150"
    mu, k = (50.0, 150) if a.workload == "aniso" else (30.0, 90)
    N, D = X.shape
    Xt = torch.from_numpy(X).cuda()
    log("bench: %s on %s" % (name, torch.cuda.get_device_name(0)))
    if a.profile_kernel:
        for _ in range(2):
            idx, d2, fl = A.knn(Xt, k, prec=a.profile_kernel)
            torch.cuda.synchronize()
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = src.clone()
        torch.cuda.synchronize()
        log("profile: knn %s N=%d D=%d k=%d; copy kernel moved %d bytes read + %d bytes written; "
            "kernel sources %s" % (a.profile_kernel, N, D, k, src.numel() * 4, dst.numel() * 4, kernel_source_hash()))
        return

    r = run_path(A, torch, Xt, mu, k, "fp32", a.steps, a.warmup)
    ms_step = 1e3 * r["wall"] / a.steps
    value = N * a.steps / r["wall"]
    tile_ms, tile_n = r["stages"]["knn_tile"]
    tile_avg_s = tile_ms / max(tile_n, 1) * 1e-3
    # algorithmic work: 2*N*D FLOP per query point (full distance row), N
    # queries per step, spread over tile_n / steps launches per step
    flop_step = 2.0 * N * N * D
    flop = flop_step * a.steps / max(tile_n, 1)  # per launch
    achieved = flop / tile_avg_s / 1e12
    stages_ms = {kname: round(v[0] / a.steps, 3) for kname, v in r["stages"].items()}
    log("fp32: %.1f points/s, %.2f ms/step, stages %s" % (value, ms_step, stages_ms))
    line = {
        "metric": "kNN+P points/s at N=70k,D=784 (FP32 vs BF16+rerank); serve p50/p99 ms",
        "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "N": N, "D": D, "perplexity": mu, "k": k, "precision": "fp32",
                   "k_cand": k + max(32, k // 2)},
        "roofline": {"bound": "mfma", "kernel": "knn_tile", "achieved": round(achieved, 2),
                     "peak": PEAK["fp32"], "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp32"], 4),
                     "traffic": measured_traffic(a.workload, "fp32"), "avg_launch_ms": round(tile_avg_s * 1e3, 3),
                     "launches_per_step": tile_n / a.steps,
                     "algorithmic": "2*N*D FLOP per query point x N queries per step, N=%d, D=%d" % (N, D)},
        "stages_ms": stages_ms,
        "rows_fp64_reranked": int((r["flags"] & 1).sum()), "rows_exact_scan": int(((r["flags"] & 8) > 0).sum()),
    }
    if not a.no_bf16:
        rb = run_path(A, torch, Xt, mu, k, "bf16", a.steps, a.warmup)
        vb = N * a.steps / rb["wall"]
        tb_ms, tb_n = rb["stages"]["knn_tile"]
        tb_avg = tb_ms / max(tb_n, 1) * 1e-3
        ach_b = flop_step * a.steps / max(tb_n, 1) / tb_avg / 1e12
        line["bf16_rerank"] = {
            "value": round(vb, 1), "ms_per_step": round(1e3 * rb["wall"] / a.steps, 3),
            "speedup_vs_fp32": round(vb / value, 3), "k_cand": 2 * k,
            "stages_ms": {kname: round(v[0] / a.steps, 3) for kname, v in rb["stages"].items()},
            "roofline": {"bound": "mfma", "kernel": "knn_tile", "achieved": round(ach_b, 2), "peak": PEAK["bf16"],
                         "unit": "TFLOP/s", "frac": round(ach_b / PEAK["bf16"], 4),
                         "traffic": measured_traffic(a.workload, "bf16"), "traffic_source": TRAFFIC_NOTE},
            "rows_valid": rows_valid(torch, rb["idx"], rb["d2"], N),
            "agree_with_fp32_rows": float((rb["idx"] == r["idx"]).all(1).float().mean().item()),
        }
        keep_b = {"idx": rb["idx"].cpu().numpy(), "P": rb["P"].cpu().numpy()}
        log("bf16: %.1f points/s (x%.2f)" % (vb, vb / value))
    keep_e = {"idx": r["idx"].cpu().numpy(), "d2": r["d2"].cpu().numpy(), "P": r["P"].cpu().numpy()}
    # The second exact contraction: each FP32 value split into BF16 hi + lo,
    # three BF16 MFMA products per element pair.  Same certificate (with its
    # own bound), same FP32 re-rank: its outputs must equal the FP32 path's.
    rx = run_path(A, torch, Xt, mu, k, "fp32x3", a.steps, a.warmup)
    vx = N * a.steps / rx["wall"]
    tx_ms, tx_n = rx["stages"]["knn_tile"]
    tx_avg = tx_ms / max(tx_n, 1) * 1e-3
    # the method's work is the FP32 contraction's 2*N*D per query; the matrix
    # cores run three BF16 products per element pair (mfma_ops_frac)
    ach_x = flop_step * a.steps / max(tx_n, 1) / tx_avg / 1e12
    same = bool(torch.equal(rx["idx"], r["idx"]) and torch.equal(rx["d2"], r["d2"])
                and np.array_equal(rx["flags"], r["flags"]))
    line["exact_fp32x3"] = {
        "value": round(vx, 1), "ms_per_step": round(1e3 * rx["wall"] / a.steps, 3),
        "speedup_vs_fp32": round(vx / value, 3), "k_cand": k + max(32, k // 2),
        "stages_ms": {kname: round(v[0] / a.steps, 3) for kname, v in rx["stages"].items()},
        "roofline": {"bound": "mfma", "kernel": "knn_tile", "achieved": round(ach_x, 2), "peak": PEAK["bf16"],
                     "unit": "TFLOP/s", "frac": round(ach_x / PEAK["bf16"], 4),
                     "mfma_ops_frac": round(3.0 * ach_x / PEAK["bf16"], 4),
                     "traffic": measured_traffic(a.workload, "fp32x3"), "traffic_source": TRAFFIC_NOTE,
                     "algorithmic": "2*N*D FLOP per query point (the method's contraction) against the BF16 peak; "
                                    "mfma_ops_frac counts the three BF16 products (hi*hi + hi*lo + lo*hi) issued"},
        "outputs_identical_to_fp32": same,
        "rows_exact_scan": int(((rx["flags"] & 8) > 0).sum()),
    }
    del rx
    log("fp32x3: %.1f points/s (x%.2f), identical to fp32: %s" % (vx, vx / value, same))
    if not (a.no_serve or a.path_only) and a.workload == "imagelike":
        log("serve: Poisson stream at %.0f req/s ..." % a.serve_rate)
        line["serve"] = serve_load(A, torch, X, a.serve_rate, a.serve_requests + 10, 10)
        log("serve: p50 %.1f ms, p99 %.1f ms" % (line["serve"]["p50_ms"], line["serve"]["p99_ms"]))
    if a.path_only:
        print(json.dumps(line), flush=True)
        return
    if a.workload == "imagelike":
        log("precision-controlled path (rho = 0.9) ...")
        line["approx_rho"] = approx_leg(A, torch, Xt, mu, k, r["idx"], value)
        log("approx: %s" % line["approx_rho"])
    fp8_kept = None
    if a.workload == "imagelike" and not a.no_fp8:
        log("precision at scale: FP8, N = 10^6 ...")
        line["fp8_scale"], fp8_kept = fp8_scale_leg(A, torch, datagen)
        log("fp8: %s" % line["fp8_scale"])
    log("attractive forces over the step's P ...")
    line["attractive"] = attractive_leg(A, torch, r["rp"], r["col"], r["val"])
    log("attractive: %.4f ms/launch, %.0f GB/s" % (line["attractive"]["avg_launch_ms"],
                                                   line["attractive"]["roofline"]["achieved"]))
    log("refinement orderings ...")
    line["order"] = order_leg(A, torch, r["idx"], r["d2"], r["beta"])
    log("order: %s" % line["order"])
    if not a.no_serve:
        log("window: sliding-window stream ...")
        line["window"] = window_stream(A, torch)
        log("window: tick p50 %.2f ms, p99 %.2f ms" % (line["window"]["tick_p50_ms"], line["window"]["tick_p99_ms"]))
    if not a.no_cpu_baseline:
        log("cpu baseline: timing the FP64 oracle on a bounded sample ...")
        line["cpu_baseline"], ora = cpu_baseline(X, mu, k, a.cpu_seconds)
        # precision metrics (Eq. 9 recall, max |dP| over the union support)
        # of each GPU path against the FP64 oracle on the sampled rows
        rows = ora["rows"]
        line["exact_vs_oracle"] = exact_vs_oracle(keep_e["idx"][rows], keep_e["d2"][rows],
                                                  keep_e["P"][rows].astype(np.float64), ora)
        if not a.no_bf16:
            line["bf16_rerank"].update(vs_oracle(keep_b["idx"][rows], keep_b["P"][rows], ora))
        log("vs oracle: exact %s" % line["exact_vs_oracle"])
        if fp8_kept is not None:
            log("fp8 vs oracle: %d sampled rows of 10^6 ..." % len(fp8_kept["rows"]))
            o8 = oracle_rows(fp8_kept["X"], 150, 50.0, fp8_kept["rows"])
            line["fp8_scale"].update(vs_oracle(fp8_kept["idx"], fp8_kept["P"], o8))
            line["fp8_scale"]["oracle_seconds"] = round(o8["seconds"], 1)
            log("fp8 vs oracle: %s" % {kk: line["fp8_scale"][kk] for kk in ("recall_vs_oracle",
                                                                          "max_abs_dP_cond_vs_oracle")})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
