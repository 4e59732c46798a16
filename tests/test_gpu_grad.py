"""Differentiation form: D(X, C) = mean_m min_k ||x_m - c_k||^2 as an
autograd function with the library's forward and hand-written backward
kernels, checked against FP64 central finite differences of D itself.

D is piecewise quadratic.  Away from ties (the two best codevectors of a row
far apart) the central difference of a quadratic is exact up to rounding, so
the bar is rounding-level agreement:
  * X: D is row-separable; for selected rows every coordinate is perturbed
    by +-h and the row's minimum over ALL codevectors is recomputed in FP64
    (best candidates by the expanded form, value in direct form);
  * C: perturbing c_k changes min(d(x, c_k'), best other) for every row; the
    best other is the oracle's FP64 second-best for rows of cell k and the
    best for the others, so D(C') is exact in O(M L) per probe; probes whose
    perturbation would move a row to another cell are skipped (then rows of
    other cells contribute the same term on both sides and cancel).
The backward is FP32 (2/M)(x - c) and (2/M) sum (c - x) per cell.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_0910_4711_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def _row_min(xs, C, c2):
    """FP64 min over codevectors of ||x - c||^2 for each row of xs."""
    e = (xs * xs).sum(1)[:, None] - 2.0 * xs @ C.T + c2[None, :]
    best = np.argsort(e, axis=1)[:, :3]
    d = ((xs[:, None, :] - C[best]) ** 2).sum(2)
    return d.min(1)


@pytest.fixture(scope="module")
def case(P):
    M, L, K, N = 65536, 64, 512, 1024
    X = synth.gmm_diag(20000, M, L, K)
    C = X[synth.distinct_rows(X, N, 20001)].astype(np.float32)
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    Ct = torch.from_numpy(C).cuda().requires_grad_(True)
    D = P.Distortion.apply(Xt, Ct)
    D.backward()
    idx, d1, d2 = oracle.assign(X, C.astype(np.float64))
    return dict(X=X.astype(np.float64), C=C.astype(np.float64), D=float(D.item()),
                gX=Xt.grad.cpu().numpy(), gC=Ct.grad.cpu().numpy(), idx=idx, d1=d1, d2=d2)


def test_forward_is_the_fp64_distortion(case):
    assert abs(case["D"] - case["d1"].mean()) <= 1e-12 * case["d1"].mean()


def test_grad_x_finite_differences(case):
    X, C, d1, d2 = case["X"], case["C"], case["d1"], case["d2"]
    M, L = X.shape
    h = 1e-3
    ok = np.flatnonzero((d2 - d1) > 1e-3 * (d1 + 1.0))
    rows = np.random.default_rng(20002).choice(ok, 256, replace=False)
    c2 = (C * C).sum(1)
    fd = np.empty((rows.size, L))
    for l in range(L):
        xp = X[rows].copy()
        xm = X[rows].copy()
        xp[:, l] += h
        xm[:, l] -= h
        fd[:, l] = (_row_min(xp, C, c2) - _row_min(xm, C, c2)) / (2 * h) / M
    g = case["gX"][rows].astype(np.float64)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_grad_c_finite_differences(case):
    X, C, idx, d1, d2 = case["X"], case["C"], case["idx"], case["d1"], case["d2"]
    M, L = X.shape
    h = 1e-4
    rng = np.random.default_rng(20003)
    counts = np.bincount(idx, minlength=C.shape[0])
    ks = rng.choice(np.flatnonzero(counts > 0), 24, replace=False)
    checked = 0
    for k in ks:
        l = int(rng.integers(L))
        own = idx == k
        Xo, oth_o = X[own], d2[own]          # best other codevector: second best
        Xn, oth_n = X[~own], d1[~own]        # rows of other cells: their best
        mins, moved = [], False
        for sgn in (1.0, -1.0):
            ck = C[k].copy()
            ck[l] += sgn * h
            dk_o = ((Xo - ck) ** 2).sum(1)
            dk_n = ((Xn - ck) ** 2).sum(1)
            if np.any(dk_o >= oth_o) or np.any(dk_n <= oth_n):
                moved = True  # some row would change cell: not a smooth probe
            mins.append(np.minimum(dk_o, oth_o))
        if moved:
            continue
        # rows of other cells keep min = their best on both sides and cancel
        fd = (mins[0] - mins[1]).sum() / (2 * h) / M
        g = float(case["gC"][k, l])
        assert abs(g - fd) <= 1e-5 * abs(fd) + 1e-12, (k, l, g, fd)
        checked += 1
    assert checked >= 16


def test_grad_c_is_cell_sum_closed_form(case):
    X, C, idx = case["X"], case["C"], case["idx"]
    M = X.shape[0]
    ref = np.zeros_like(C)
    np.add.at(ref, idx, C[idx] - X)
    ref *= 2.0 / M
    np.testing.assert_allclose(case["gC"], ref, rtol=2 ** -20, atol=1e-12)


@pytest.mark.parametrize("M,L,n", [(1, 1, 1), (999, 3, 5), (4097, 16, 64), (3001, 17, 9),
                                   (2049, 64, 300), (513, 200, 7), (70001, 16, 256)])
def test_grad_x_exact_layouts(P, M, L, n):
    # dD/dX = (2g/M)(x - c_idx) in FP64, rounded once: bit-identical to the
    # oracle's closed form rounded to FP32, on the 16-byte path (L % 4 == 0)
    # and the scalar path (other L, misaligned X); rows whose index is out of
    # range get zeros and leave the other rows unchanged
    X = (synth.gmm(M + 5, M, L, 7)).astype(np.float32)
    rng = np.random.default_rng(M * 3 + L)
    C = rng.normal(100.0, 30.0, size=(n, L)).astype(np.float32)
    idx = rng.integers(0, n, size=M).astype(np.int32)
    g = 0.75
    want, _ = oracle.grad(X, C.astype(np.float64), idx, g=g)
    want = want.astype(np.float32)
    Cd = torch.from_numpy(C).cuda()
    bad = np.zeros(M, bool)
    if M > 1:
        bad[rng.choice(M, size=M // 50 + 1, replace=False)] = True
    idx_bad = np.where(bad, n, idx).astype(np.int32)
    for misaligned in (False, True):
        if misaligned:
            buf = torch.zeros(M * L + 1, dtype=torch.float32, device="cuda")
            buf[1:] = torch.from_numpy(X).cuda().reshape(-1)
            Xd = buf[1:].view(M, L)
        else:
            Xd = torch.from_numpy(X).cuda()
        gX, _ = P.distortion_backward(Xd, Cd, torch.from_numpy(idx).cuda(), g, need_c=False)
        np.testing.assert_array_equal(gX.cpu().numpy(), want)
        gB, _ = P.distortion_backward(Xd, Cd, torch.from_numpy(idx_bad).cuda(), g,
                                      need_c=False)
        got = gB.cpu().numpy()
        assert np.all(got[bad] == 0.0)
        np.testing.assert_array_equal(got[~bad], want[~bad])


@pytest.mark.parametrize("M,L,N", [(20000, 64, 4096), (7777, 48, 6000), (300, 64, 4096)])
def test_grad_c_sorted_cells(P, M, L, N):
    # codebooks beyond the fixed-point path's LDS budget sum the cells through
    # the sorted allocation: sum_cell (c - x) in FP64, times 2g/M, rounded
    # once; the oracle accumulates -(2g/M)(x - c) row by row in FP64, so the
    # two agree to FP32 rounding (empty cells: exactly 0)
    X = synth.gmm(M + 9, M, L, 31).astype(np.float32)
    rng = np.random.default_rng(N + L)
    C = (X[rng.choice(M, size=min(M, N), replace=False)] + 0.5).astype(np.float32)
    if C.shape[0] < N:
        C = np.concatenate([C, rng.normal(size=(N - C.shape[0], L)).astype(np.float32)])
    idx = rng.integers(0, min(M, N), size=M).astype(np.int32)
    g = 1.25
    _, want = oracle.grad(X, C.astype(np.float64), idx, g=g)
    _, gC = P.distortion_backward(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(),
                                  torch.from_numpy(idx).cuda(), g, need_x=False)
    got = gC.cpu().numpy().astype(np.float64)
    used = np.zeros(N, bool)
    used[idx] = True
    assert np.all(got[~used] == 0.0)
    scale = np.abs(want[used]).max()
    np.testing.assert_allclose(got[used], want[used], rtol=2.0 ** -22, atol=1e-12 * scale)
