"""Shared fixtures for the GPU tests (HIP path through the C ABI)."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch


def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1512_01655_amd import atsne

    atsne.load()  # raises if libatsne.so is missing: no fallback
    return atsne


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_knn(A, X: np.ndarray, k: int, prec: str = "fp32", kc: int = 0, qids=None):
    say("  knn N=%d D=%d k=%d prec=%s kc=%d M=%s" % (X.shape[0], X.shape[1], k, prec, kc,
                                                     "all" if qids is None else len(qids)))
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    q = None if qids is None else torch.from_numpy(np.asarray(qids, np.int32)).cuda()
    idx, d2, fl = A.knn(Xt, k, prec=prec, k_cand=kc, query_ids=q)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), d2.cpu().numpy(), fl.cpu().numpy()
