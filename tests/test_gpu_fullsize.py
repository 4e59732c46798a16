"""Full-size parity: the benchmark's own workloads, in the launch shapes it
times, against the FP64 oracle.

* LBG run on the 16-picture workload (M = 262,144, L = 16, N = 256): pixel
  data are integers, so every sum is exact and the run equals the oracle's
  with FP32 codebook storage -- allocations, codebooks, per-level iteration
  counts -- and D agrees to rounding of the final sum.
* Differentiation form (X [1,048,576 x 64], C [4096 x 64]): the forward D
  against the oracle's FP64 distortion of the returned allocation; dD/dX on
  1,024 sampled rows away from ties against FP64 central finite differences
  of D; dD/dC for every cell against the closed form (2/M) sum (c - x),
  summed in FP64.  For the finite differences a row's minimum is taken over
  its 8 best codevectors by the expanded form: the rows kept have a gap of
  at least 1e-3 (d1 + 1) between their two best distances, far above what a
  perturbation of 1e-3 changes, so the minimum stays among them.
* Precision form (256 pictures of 1024 x 1024 in 8 x 8 blocks: M =
  4,194,304, L = 64, N = 1024): from the codebook of 10 exact iterations,
  the exact step equals the oracle (allocation on a 65,536-row subsample,
  update on every row); the BF16 step is within relative 1e-3 per
  codevector and in D, with few and cheap misallocations on the subsample.
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


def test_train_benchmark_workload_matches_oracle(P):
    cfg = synth.CONFIG1
    X = synth.image_training_set(cfg["seeds"], cfg["W"], cfg["H"], cfg["b"])
    assert X.shape == (262_144, 16)
    C, idx, D, st = P.train(torch.from_numpy(X).cuda(), cfg["N"])
    ref = oracle.train(X, cfg["N"], store_fp32=True)
    np.testing.assert_array_equal(st["level_iters"], ref["level_iters"])
    np.testing.assert_array_equal(idx.cpu().numpy(), ref["idx"])
    np.testing.assert_array_equal(C.cpu().numpy(), ref["C"].astype(np.float32))
    assert abs(D - ref["D"]) <= 1e-12 * ref["D"]


def _top(xs, C64, c2, k):
    e = (xs * xs).sum(1)[:, None] - 2.0 * xs @ C64.T + c2[None, :]
    return np.argpartition(e, k, axis=1)[:, :k]


def _dist(xs, C64, cand):
    return ((xs[:, None, :] - C64[cand]) ** 2).sum(2)


def test_differentiation_full_size(P):
    M, L, K, N = 1_048_576, 64, 512, 4096
    X = synth.gmm_diag(20000, M, L, K)
    C = np.ascontiguousarray(X[synth.distinct_rows(X, N, 20001)])
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    Ct = torch.from_numpy(C).cuda().requires_grad_(True)
    D = P.Distortion.apply(Xt, Ct)
    D.backward()
    Dv = float(D.item())
    gX = Xt.grad.cpu().numpy()
    gC = Ct.grad.cpu().numpy().astype(np.float64)
    idx, _ = P.assign(Xt.detach(), Ct.detach(), with_mind=False)
    idx = idx.cpu().numpy()

    # forward: the oracle's FP64 distortion of this allocation
    want_D = oracle.distortion(X, C.astype(np.float64), idx)
    assert abs(Dv - want_D) <= 1e-12 * want_D

    # the allocation of 8,192 sampled rows against the oracle's exhaustive
    # FP64 search (every row: the allocation is exact, ties included); the
    # finite differences on 1,024 of them whose oracle top-2 gap keeps the
    # argmin fixed under the step
    C64 = C.astype(np.float64)
    c2 = (C64 * C64).sum(1)
    rng = np.random.default_rng(20003)
    pool = np.sort(rng.choice(M, 8192, replace=False))
    xs = X[pool].astype(np.float64)
    io, d1, d2 = oracle.assign(X[pool], C64)
    np.testing.assert_array_equal(idx[pool], io)
    ok = np.flatnonzero((d2 - d1) > 1e-3 * (d1 + 1.0))
    assert ok.size >= 1024
    sel = ok[:1024]
    rows = pool[sel]

    h = 1e-3
    xr = xs[sel]
    # the perturbed rows' distances to their eight nearest codevectors (the
    # minimum cannot leave them for a step of 1e-3)
    cr = _top(xr, C64, c2, 8)
    fd = np.empty((rows.size, L))
    for l in range(L):
        xp = xr.copy()
        xm = xr.copy()
        xp[:, l] += h
        xm[:, l] -= h
        fd[:, l] = (_dist(xp, C64, cr).min(1) - _dist(xm, C64, cr).min(1)) / (2 * h) / M
    np.testing.assert_allclose(gX[rows].astype(np.float64), fd, rtol=1e-6,
                               atol=1e-9 * np.abs(fd).max())

    # dD/dC: (2/M) sum over the cell of (c - x), every cell, FP64 sums
    o = np.argsort(idx, kind="stable")
    starts = np.searchsorted(idx[o], np.arange(N))
    counts = np.bincount(idx, minlength=N)
    sums = np.zeros((N, L))
    nz = counts > 0
    sums[nz] = np.add.reduceat(X[o].astype(np.float64), starts[nz], axis=0)
    want_C = (2.0 / M) * (counts[:, None] * C64 - sums)
    assert np.all(gC[~nz] == 0.0)
    scale = np.abs(want_C).max()
    np.testing.assert_allclose(gC, want_C, rtol=2.0 ** -21, atol=1e-9 * scale)


def _pictures_b8(seeds):
    import concurrent.futures as cf
    # threads (NumPy releases the GIL in the blob sums): no fork of a process
    # that holds the GPU
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        parts = list(ex.map(lambda s: synth.blocks(synth.image(s, 1024, 1024), 8), seeds))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def test_precision_form_full_size(P):
    # 256 pictures of 1024 x 1024 in 8 x 8 blocks (M = 4,194,304, L = 64),
    # N = 1024 distinct training vectors, 10 exact iterations give the
    # reference codebook; then one exact step and one BF16 step from it
    cfg = synth.CONFIG2
    X = _pictures_b8(cfg["seeds"])
    M, L, N = X.shape[0], X.shape[1], cfg["N"]
    assert (M, L) == (4_194_304, 64)
    C0 = np.ascontiguousarray(X[synth.distinct_rows(X, N, 1000)])
    Xd = torch.from_numpy(X).cuda()
    Cref, _, _, st = P.train(Xd, N, C_init=torch.from_numpy(C0).cuda(), fixed_iters=10)
    assert st["level_iters"] == [10]
    idx_f, _ = P.assign(Xd, Cref, P.FP32, with_mind=False)
    idx_b, _ = P.assign(Xd, Cref, P.BF16_RESCORE, with_mind=False)
    Cf1, _ = P.update(Xd, idx_f, Cref)
    Cb1, _ = P.update(Xd, idx_b, Cref)
    D_f = float(P.distortion(Xd, Cref, idx_f))
    D_b = float(P.distortion(Xd, Cref, idx_b))
    Ch = Cref.cpu().numpy().astype(np.float64)
    f_idx = idx_f.cpu().numpy()
    # exact step: allocation on a 65,536-row subsample, update on all rows
    rows = np.sort(np.random.default_rng(1001).choice(M, 65_536, replace=False))
    idx_o, d1, d2 = oracle.assign(X[rows], Ch)
    np.testing.assert_array_equal(f_idx[rows], idx_o)
    want_C, _ = oracle.update(X, f_idx, Ch, store_fp32=True)
    np.testing.assert_array_equal(Cf1.cpu().numpy(), want_C.astype(np.float32))
    # BF16 step: per-codevector relative 1e-3 against the exact step, D 1e-3;
    # a row it allocates differently costs at most a small excess distance
    cb, cf = Cb1.cpu().numpy().astype(np.float64), Cf1.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(cb - cf, axis=1) / np.maximum(np.linalg.norm(cf, axis=1), 1e-30)
    assert rel.max() <= 1e-3
    assert abs(D_b - D_f) <= 1e-3 * D_f
    ib = idx_b.cpu().numpy()[rows]
    dsel = ((X[rows].astype(np.float64) - Ch[ib]) ** 2).sum(1)
    assert np.all(dsel >= d1 * (1.0 - 1e-12))  # (numpy sums in another order)
    assert ((dsel - d1) / np.maximum(d1, 1e-30)).max() <= 1e-2
    assert (ib != idx_o).mean() <= 1e-3
