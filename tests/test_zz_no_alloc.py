"""The allocation-free entry point (lbg_assign_distortion_noalloc, scratch in
the library's fixed per-GPU array) against lbg_assign_distortion with a
caller workspace, through the C ABI: identical allocations, distances and
distortion, on two calls in a row, the second with a smaller input (the
array keeps the first call's contents, which the second must not read)."""
import ctypes as ct

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_0910_4711_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def _call_ws(P, X, C, prec):
    lib = P.load()
    M, L = X.shape
    N = C.shape[0]
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    mind = torch.empty(M, dtype=torch.float32, device=X.device)
    D = torch.empty((), dtype=torch.float64, device=X.device)
    nb = lib.lbg_workspace_size(P.OP_ASSIGN, M, L, N, prec)
    ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    s = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.lbg_assign_distortion(ct.c_void_p(X.data_ptr()), M, L, ct.c_void_p(C.data_ptr()),
                                   N, ct.c_void_p(idx.data_ptr()), ct.c_void_p(mind.data_ptr()),
                                   prec, ct.c_void_p(D.data_ptr()), ct.c_void_p(ws.data_ptr()),
                                   nb, s)
    assert rc == P.OK, lib.lbg_last_error()
    return idx, mind, D


def _call_noalloc(P, X, C, prec):
    lib = P.load()
    M, L = X.shape
    N = C.shape[0]
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    mind = torch.empty(M, dtype=torch.float32, device=X.device)
    D = torch.empty((), dtype=torch.float64, device=X.device)
    s = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.lbg_assign_distortion_noalloc(ct.c_void_p(X.data_ptr()), M, L,
                                           ct.c_void_p(C.data_ptr()), N,
                                           ct.c_void_p(idx.data_ptr()),
                                           ct.c_void_p(mind.data_ptr()), prec,
                                           ct.c_void_p(D.data_ptr()), s)
    assert rc == P.OK, lib.lbg_last_error()
    return idx, mind, D


# (M, L, N, precision): resident codebooks, a chunked one staged from the
# prepared copy in the scratch array, the exhaustive FP64 kernel (L > 128)
@pytest.mark.parametrize("first,second", [
    ((200_000, 16, 256, 0), (3_001, 16, 40, 0)),
    ((100_000, 64, 2048, 0), (5_000, 64, 300, 0)),
    ((150_000, 64, 1024, 1), (777, 64, 33, 1)),
    ((20_000, 200, 9, 0), (1_000, 200, 7, 0)),
])
def test_noalloc_matches_workspace_entry(P, first, second):
    for k, (M, L, N, prec) in enumerate((first, second)):
        X = torch.from_numpy(synth.gmm(300 + k + L, M, L, 16)).cuda()
        C = X[torch.randperm(M, generator=torch.Generator().manual_seed(k))[:N].cuda()].contiguous()
        a = _call_ws(P, X, C, prec)
        b = _call_noalloc(P, X, C, prec)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]), f"call {k}: allocation differs"
        assert torch.equal(a[1], b[1]), f"call {k}: distances differ"
        assert float(a[2].item()) == float(b[2].item()), f"call {k}: distortion differs"


def test_noalloc_rejects_oversized_problems(P):
    lib = P.load()
    cap = lib.lbg_noalloc_scratch_bytes()
    assert cap == 8 << 20
    M = 40_000_000  # FP64 partials alone: 10 MB
    assert lib.lbg_workspace_size(P.OP_ASSIGN, M, 16, 16, 0) > cap
    fake = ct.c_void_p(1 << 20)  # never dereferenced: the size check fails first
    rc = lib.lbg_assign_distortion_noalloc(fake, M, 16, fake, 16, fake, None, 0, fake, None)
    assert rc == P.EINVAL and b"scratch" in lib.lbg_last_error()
