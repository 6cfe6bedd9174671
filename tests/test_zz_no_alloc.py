"""The allocation-free symmetrisation (atsne_symmetrize_noalloc) against the
allocating entry point (atsne_symmetrize), through the C ABI: identical CSR
output bit for bit on two calls in a row (the second with a smaller input,
over the scratch the first left behind), and inputs beyond its fixed scratch
refused before any work."""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_common import lib, say

pytestmark = pytest.mark.gpu


def _rows(N, k, seed):
    rng = np.random.default_rng(seed)
    idx = np.empty((N, k), np.int32)
    for i in range(N):
        c = rng.choice(N - 1, size=k, replace=False)
        idx[i] = np.where(c >= i, c + 1, c)  # no self
    P = rng.dirichlet(np.ones(k), size=N).astype(np.float32)
    return torch.from_numpy(idx).cuda(), torch.from_numpy(P).cuda()


def _call(L, fn, idx, P, ws=None):
    N, k = idx.shape
    rp = torch.full((N + 1,), -7, dtype=torch.int64, device="cuda")
    col = torch.full((2 * N * k,), -7, dtype=torch.int32, device="cuda")
    val = torch.full((2 * N * k,), -7.0, dtype=torch.float32, device="cuda")
    nnz = ctypes.c_int64(-1)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    if fn == "noalloc":
        s = L.atsne_symmetrize_noalloc(ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(P.data_ptr()), N, k,
                                       ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                                       ctypes.c_void_p(val.data_ptr()), ctypes.byref(nnz), st)
    else:
        s = L.atsne_symmetrize(ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(P.data_ptr()), N, k,
                               ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                               ctypes.c_void_p(val.data_ptr()), ctypes.byref(nnz), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), st)
    torch.cuda.synchronize()
    return s, nnz.value, rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()


def test_noalloc_equals_allocating_entry_point():
    A = lib()
    L = A.load()
    for N, k, seed in [(6000, 90, 1), (1500, 30, 2)]:  # second call smaller, over the first's scratch
        say("  symmetrize N=%d k=%d: noalloc vs allocating" % (N, k))
        idx, P = _rows(N, k, seed)
        b = ctypes.c_size_t()
        assert L.atsne_symmetrize_workspace_size(N, N * k, ctypes.byref(b)) == A.OK
        ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
        s0, n0, rp0, c0, v0 = _call(L, "alloc", idx, P, ws)
        s1, n1, rp1, c1, v1 = _call(L, "noalloc", idx, P)
        assert s0 == A.OK and s1 == A.OK, L.atsne_last_error()
        assert n0 == n1 and N * k <= n1 <= 2 * N * k
        assert np.array_equal(rp0, rp1)
        assert np.array_equal(c0[:n0], c1[:n1]) and np.array_equal(v0[:n0], v1[:n1])
        say("    nnz %d, identical" % n1)


SCRATCH_BYTES = 64 << 20  # the allocation-free symmetrisation's device array


def test_noalloc_refuses_inputs_beyond_its_scratch():
    A = lib()
    L = A.load()
    N, k = 100000, 90
    # the refusal happens on the host before any work: the input must need
    # more scratch than the array holds, or the call would run its kernels on
    # the placeholder buffers below
    b = ctypes.c_size_t()
    assert L.atsne_symmetrize_workspace_size(N, N * k, ctypes.byref(b)) == A.OK
    assert b.value > 2 * SCRATCH_BYTES
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    nnz = ctypes.c_int64(-1)
    p = ctypes.c_void_p(dummy.data_ptr())
    s = L.atsne_symmetrize_noalloc(p, p, N, k, p, p, p, ctypes.byref(nnz), None)
    assert s == A.E_NOMEM and b"allocation-free" in L.atsne_last_error()
    assert nnz.value == -1
