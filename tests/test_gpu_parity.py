"""GPU library vs the FP64 CPU oracle, element by element, on seeded inputs.

Bars (from the arithmetic of each step):
  * allocation (FP32 mode): identical indices -- the library proves its
    screen or searches again in FP64, so it returns the FP64 direct-form
    argmin; the winning distance equals the oracle's FP64 distance rounded
    to FP32;
  * split: identical to the oracle's split with FP32 storage (both form the
    product in FP64 and round once);
  * centroid / update: identical for integer-valued data (FP64 sums of
    integers are exact in any order); otherwise within 1 FP32 ulp of the
    oracle's FP64 mean rounded to FP32;
  * distortion: relative 1e-12 (same per-row FP64 values, different order of
    the final sum);
  * whole LBG on integer-valued images: identical codebooks, allocations and
    per-level iteration counts as the oracle with FP32 codebook storage;
    against the FP64-storage oracle: codebooks within relative 1e-5 per
    codevector and final distortion within relative 1e-6.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _gmm(seed, M, L, K, scale=1.0):
    return (synth.gmm(seed, M, L, K) * scale).astype(np.float32)


def _img_rows(M, L=16, seed=0):
    b = int(round(L ** 0.5))
    X = synth.image_training_set((seed,), 512, 512, b)
    return np.ascontiguousarray(X[:M])


ASSIGN_CASES = [
    # (M, L, n, kind)
    (1, 16, 1, "img"),
    (37, 16, 5, "img"),
    (1000, 16, 64, "img"),
    (4097, 16, 256, "img"),
    (3000, 16, 257, "img"),
    (2000, 64, 100, "img"),
    (2500, 1, 7, "gmm"),
    (1500, 3, 33, "gmm"),
    (1300, 8, 128, "gmm"),
    (999, 17, 40, "gmm"),
    (777, 32, 300, "gmm"),
    (800, 100, 20, "gmm"),
    (600, 128, 129, "gmm"),
    (300, 200, 9, "gmm"),
    # small codebooks take the direct FP64 search (several 64-vector groups
    # per wave, ragged ends), and just above it the screen again
    (70001, 16, 2, "gmm"),
    (16383, 16, 2, "img"),
    (4097, 16, 8, "img"),
    (3001, 8, 4, "gmm"),
    (2049, 32, 8, "gmm"),
    (999, 17, 3, "gmm"),
    (1000, 16, 9, "img"),
    # codebooks resident only in one eight-wave workgroup's LDS, and larger
    # ones staged chunk by chunk
    (5000, 16, 700, "img"),
    (3000, 64, 400, "gmm"),
    (2000, 64, 700, "gmm"),
]


def _case(M, L, n, kind, seed):
    if kind == "img":
        X = _img_rows(M, L, seed)
    else:
        X = _gmm(seed, M, L, max(2, n // 2))
    rng = np.random.default_rng(seed + 100)
    C = X[rng.integers(0, M, size=n)].astype(np.float64)
    C = (C + rng.normal(0, 3.0, size=C.shape)).astype(np.float32)
    return X, C


@pytest.mark.parametrize("M,L,n,kind", ASSIGN_CASES)
def test_assign_fp32_exact(P, M, L, n, kind):
    X, C = _case(M, L, n, kind, seed=M + L + n)
    idx_o, d1, _ = oracle.assign(X, C.astype(np.float64))
    idx, mind = P.assign(dev(X), dev(C), P.FP32)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(idx), idx_o)
    np.testing.assert_array_equal(host(mind), d1.astype(np.float32))


def test_assign_ties_lowest_index(P):
    # duplicated codevectors and vectors exactly midway between two of them
    rng = np.random.default_rng(5)
    C = rng.integers(-20, 20, size=(40, 16)).astype(np.float32) * 2
    C[7] = C[3]
    C[30] = C[3]
    C[12] = C[29]
    X = np.concatenate([
        C[[3, 7, 30, 12, 29]],
        ((C[5] + C[6]) / 2)[None],
        ((C[1] + C[9]) / 2)[None],
        rng.integers(-40, 40, size=(500, 16)).astype(np.float32),
    ]).astype(np.float32)
    idx_o, _, _ = oracle.assign(X, C.astype(np.float64))
    idx, _ = P.assign(dev(X), dev(C), P.FP32)
    np.testing.assert_array_equal(host(idx), idx_o)
    assert host(idx)[0] == 3 and host(idx)[1] == 3 and host(idx)[3] == 12


@pytest.mark.parametrize("L,eps", [(16, 1e-3), (16, 1e-5), (16, 1e-7), (32, 1e-6), (64, 1e-6)])
def test_assign_split_siblings_exact(P, L, eps):
    # codebooks of split pairs c(1 + eps), c(1 - eps) (children 2i, 2i + 1),
    # the near ties the second acceptance test and the exhaustive search
    # settle; vectors drawn around the parents and exactly at some of them
    rng = np.random.default_rng(int(1e6 * eps) + L)
    par = rng.uniform(0, 255, size=(40, L))
    C = np.empty((80, L), np.float32)
    C[0::2] = (par * (1 + eps)).astype(np.float32)
    C[1::2] = (par * (1 - eps)).astype(np.float32)
    X = (par[rng.integers(0, 40, size=6000)] + rng.normal(0, 4.0, size=(6000, L))).astype(np.float32)
    X[:40] = par.astype(np.float32)
    idx_o, d1, _ = oracle.assign(X, C.astype(np.float64))
    idx, mind = P.assign(dev(X), dev(C), P.FP32)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(idx), idx_o)
    np.testing.assert_array_equal(host(mind), d1.astype(np.float32))


@pytest.mark.parametrize("L,n", [(8, 100), (16, 300), (32, 96), (64, 64)])
def test_assign_large_offset_exact(P, L, n):
    # a common offset of 1e4 with a spread of a few units: |x|^2 dwarfs the
    # distances, so the screen's error bound is large relative to the gaps
    # and many rows need the second test or the search
    rng = np.random.default_rng(L + n)
    base = 1e4 + rng.normal(0, 1.0, size=L)
    C = (base + rng.normal(0, 3.0, size=(n, L))).astype(np.float32)
    X = (base + rng.normal(0, 3.0, size=(5000, L))).astype(np.float32)
    idx_o, d1, _ = oracle.assign(X, C.astype(np.float64))
    idx, mind = P.assign(dev(X), dev(C), P.FP32)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(idx), idx_o)
    np.testing.assert_array_equal(host(mind), d1.astype(np.float32))


def test_assign_all_equal_and_zero(P):
    X = np.full((513, 16), 255.0, np.float32)
    X[100:200] = 0.0
    C = np.stack([np.full(16, 255.0), np.zeros(16), np.full(16, 255.0), np.zeros(16)]).astype(np.float32)
    idx, mind = P.assign(dev(X), dev(C), P.FP32)
    h = host(idx)
    assert np.all(h[:100] == 0) and np.all(h[100:200] == 1) and np.all(h[200:] == 0)
    assert np.all(host(mind) == 0)


def test_split_matches_oracle(P):
    rng = np.random.default_rng(3)
    C = (rng.normal(size=(33, 17)) * 50).astype(np.float32)
    C[4] = 0.0
    for eps in (0.01, 0.25):
        got = host(P.split(dev(C), eps=eps))
        want = oracle.split(C.astype(np.float64), eps=eps, store_fp32=True)
        np.testing.assert_array_equal(got, want.astype(np.float32))
    got = host(P.split(dev(C), mode=P.SPLIT_ADD, delta=0.37))
    want = oracle.split(C.astype(np.float64), mode=oracle.SPLIT_ADD, delta=0.37, store_fp32=True)
    np.testing.assert_array_equal(got, want.astype(np.float32))


@pytest.mark.parametrize("M,L", [(1, 1), (255, 16), (4096, 16), (10007, 64), (3000, 200)])
def test_centroid(P, M, L):
    Xi = _gmm(M, M, L, 3)
    Xint = np.rint(Xi)
    for X, exact in ((Xint, True), (Xi, False)):
        got = host(P.centroid(dev(X)))[0]
        want = oracle.centroid(X)[0]
        if exact:
            np.testing.assert_array_equal(got, want.astype(np.float32))
        else:
            np.testing.assert_allclose(got, want, rtol=2 ** -23, atol=1e-30)


UPDATE_CASES = [(1, 1, 1), (100, 16, 7), (4096, 16, 64), (20000, 16, 256), (9000, 64, 1024),
                (5000, 3, 9), (3000, 100, 50), (1000, 200, 5), (70000, 8, 4096),
                # codebooks beyond the fixed-point path's LDS budget: cells summed
                # through the sorted allocation (LDS histogram; N > 8192: global one)
                (30000, 64, 4096), (4000, 128, 2000), (3000, 256, 1000), (50000, 16, 20000)]


@pytest.mark.parametrize("M,L,n", UPDATE_CASES)
def test_update(P, M, L, n):
    rng = np.random.default_rng(M + L + n)
    Xf = _gmm(n, M, L, 4)
    Xint = np.rint(Xf).astype(np.float32)
    C_old = rng.normal(size=(n, L)).astype(np.float32)
    # skewed cell sizes with some empty cells and one very large cell
    idx = rng.integers(0, max(1, n - 2), size=M).astype(np.int32)
    idx[: M // 3] = 0
    for X, exact in ((Xint, True), (Xf, False)):
        C_new, counts = P.update(dev(X), dev(idx), dev(C_old))
        want, cnt = oracle.update(X, idx, C_old.astype(np.float64), store_fp32=True)
        np.testing.assert_array_equal(host(counts), cnt)
        got = host(C_new)
        if exact:
            np.testing.assert_array_equal(got, want.astype(np.float32))
        else:
            np.testing.assert_allclose(got, want, rtol=2 ** -23, atol=0)
        empty = cnt == 0
        np.testing.assert_array_equal(got[empty], C_old[empty])


def test_update_in_place_and_invalid_indices(P):
    rng = np.random.default_rng(11)
    M, L, n = 5000, 16, 32
    X = np.rint(_gmm(1, M, L, 4))
    idx = rng.integers(0, n, size=M).astype(np.int32)
    idx[::7] = -1
    idx[::11] = n + 3
    C = rng.normal(size=(n, L)).astype(np.float32)
    Cd = dev(C)
    _, counts = P.update(dev(X), dev(idx), Cd, out=Cd)
    keep = (idx >= 0) & (idx < n)
    want, cnt = oracle.update(X[keep], idx[keep], C.astype(np.float64), store_fp32=True)
    np.testing.assert_array_equal(host(counts), cnt)
    np.testing.assert_array_equal(host(Cd), want.astype(np.float32))


@pytest.mark.parametrize("M,L,n", [(1, 4, 1), (1000, 16, 64), (33333, 64, 256), (500, 200, 7)])
def test_distortion(P, M, L, n):
    X = _gmm(M, M, L, 5)
    rng = np.random.default_rng(2)
    C = rng.normal(size=(n, L)).astype(np.float32) * 10
    idx = rng.integers(0, n, size=M).astype(np.int32)
    got = float(P.distortion(dev(X), dev(C), dev(idx)))
    want = oracle.distortion(X, C.astype(np.float64), idx)
    assert abs(got - want) <= 1e-12 * abs(want)


@pytest.mark.parametrize("M,L,n", [(1, 16, 1), (1000, 20, 37), (4097, 64, 300),
                                   (70001, 16, 256), (999, 3, 5), (3001, 200, 20),
                                   (2049, 32, 8), (5000, 17, 40)])
def test_distortion_rows_in_lds(P, M, L, n):
    # the distortion pass stages rows through LDS 16 dimensions at a time:
    # ragged chunks (L = 17, 20, 200), one row, misaligned X (scalar path)
    X = _gmm(M + 3, M, L, 5)
    rng = np.random.default_rng(L)
    C = rng.normal(size=(n, L)).astype(np.float32) * 10
    idx = rng.integers(0, n, size=M).astype(np.int32)
    if M > 1:
        idx[rng.choice(M, size=M // 100 + 1, replace=False)] = n  # rows that add 0
    good = idx < n
    want_sum = oracle.distortion(X[good], C.astype(np.float64), idx[good]) * int(good.sum())
    got = float(P.distortion(dev(X), dev(C), dev(idx)))
    assert abs(got * M - want_sum) <= 1e-12 * abs(want_sum)
    buf = torch.zeros(M * L + 1, dtype=torch.float32, device="cuda")
    buf[1:] = dev(X).reshape(-1)
    got_mis = float(P.distortion(buf[1:].view(M, L), dev(C), dev(idx)))
    assert got_mis == got  # same per-row values, same order


@pytest.mark.parametrize("M,L,n,prec", [(70001, 16, 256, "fp32"), (4097, 64, 300, "fp32"),
                                        (999, 3, 5, "fp32"), (3001, 200, 20, "fp32"),
                                        (2049, 32, 8, "fp32"), (1, 16, 4, "fp32"),
                                        (5000, 64, 129, "bf16"), (5000, 16, 64, "bf16")])
def test_assign_distortion_one_pass(P, M, L, n, prec):
    # allocation + distortion in one pass: the allocation of lbg_assign, and
    # the oracle's FP64 distortion of it (same per-row values, another order)
    X = _img_rows(M) if (L == 16 and M <= 16384) else _gmm(M + 11, M, L, 9)
    rng = np.random.default_rng(M + L)
    C = np.ascontiguousarray(X[rng.choice(M, size=min(n, M), replace=False)])
    while C.shape[0] < n:
        C = np.concatenate([C, C[-1:] + 1.0])
    Xd, Cd = dev(X), dev(C)
    idx, mind, D = P.assign_distortion(Xd, Cd, prec, with_mind=True)
    idx2, mind2 = P.assign(Xd, Cd, prec)
    assert torch.equal(idx, idx2) and torch.equal(mind, mind2)
    want = oracle.distortion(X, C.astype(np.float64), host(idx))
    # FP64 per-row distances (exact form); the BF16 form rescores its rows in
    # FP32, within (L + 4) 2^-24 of each row's FP64 distance
    tol = 1e-12 if prec == "fp32" else (L + 4) * 2.0 ** -24
    assert abs(float(D) - want) <= tol * abs(want)
    assert abs(float(D) - float(P.distortion(Xd, Cd, idx))) <= tol * abs(want)


def _config0():
    return synth.image_training_set((0,), 256, 256, 4)


def test_train_config0_matches_oracle(P):
    X = _config0()
    C, idx, D, st = P.train(dev(X), 64)
    ref = oracle.train(X, 64, store_fp32=True)
    np.testing.assert_array_equal(st["level_iters"], ref["level_iters"])
    np.testing.assert_array_equal(host(idx), ref["idx"])
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))
    assert abs(D - ref["D"]) <= 1e-12 * ref["D"]
    np.testing.assert_allclose(st["D_trace"], ref["D_trace"], rtol=1e-12)
    # the FP64-storage oracle (spec tolerances)
    r64 = oracle.train(X, 64, store_fp32=False)
    Cg = host(C).astype(np.float64)
    num = np.linalg.norm(Cg - r64["C"], axis=1)
    den = np.linalg.norm(r64["C"], axis=1)
    assert np.all(np.where(den > 0, num / np.maximum(den, 1e-300), num) <= 1e-5)
    assert abs(D - r64["D"]) <= 1e-6 * r64["D"]


def test_train_small_cases(P):
    # N = 1, C_init, fixed iterations, additive split, point masses (D = 0)
    X = _img_rows(2000, 16, 3)
    C, idx, D, st = P.train(dev(X), 1)
    ref = oracle.train(X, 1, store_fp32=True)
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))
    assert abs(D - ref["D"]) <= 1e-12 * ref["D"]

    rng = np.random.default_rng(4)
    C0 = X[rng.permutation(2000)[:16]]
    C, idx, D, st = P.train(dev(X), 16, C_init=dev(C0), fixed_iters=5)
    ref = oracle.train(X, 16, C_init=C0.astype(np.float64), fixed_iters=5, store_fp32=True)
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))
    np.testing.assert_array_equal(host(idx), ref["idx"])
    assert st["level_iters"] == [5]

    C, idx, D, st = P.train(dev(X), 8, split_mode=P.SPLIT_ADD, delta=0.5)
    ref = oracle.train(X, 8, split_mode=oracle.SPLIT_ADD, delta=0.5, store_fp32=True)
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))

    Xp = np.array([[1.0]] * 5 + [[3.0]] * 3, np.float32)
    C, idx, D, st = P.train(dev(Xp), 2, max_iter=50)
    assert st["status"] == P.OK and D == 0.0 and list(host(C)[:, 0]) == [3.0, 1.0]


def test_train_wide_codebook_matches_oracle(P):
    # L = 64, N = 512: the device-side loop runs the allocation in eight-wave
    # workgroups with the whole codebook resident
    X = _img_rows(4096, 64, 11)
    C, idx, D, st = P.train(dev(X), 512)
    ref = oracle.train(X, 512, store_fp32=True)
    np.testing.assert_array_equal(st["level_iters"], ref["level_iters"])
    np.testing.assert_array_equal(host(idx), ref["idx"])
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))
    assert abs(D - ref["D"]) <= 1e-12 * ref["D"]


@pytest.mark.parametrize("M,L,N", [(2000, 200, 16), (2048, 256, 1024), (3000, 160, 64)])
def test_train_host_loop_matches_oracle(P, M, L, N):
    # L > 128 runs the host-controlled loop (FP64 allocation); at L = 256,
    # N = 1024 its updates sum the cells through the sorted allocation; at
    # L = 160, N = 64 through five 32-dimension slices of 32-bit sums.
    # Integer-valued data: every sum is exact, so the run equals the oracle's
    # with FP32 codebook storage
    X = np.rint(_gmm(L + N, M, L, 12)).astype(np.float32)
    C, idx, D, st = P.train(dev(X), N)
    ref = oracle.train(X, N, store_fp32=True)
    np.testing.assert_array_equal(st["level_iters"], ref["level_iters"])
    np.testing.assert_array_equal(host(idx), ref["idx"])
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))
    assert abs(D - ref["D"]) <= 1e-12 * ref["D"]


def test_train_deterministic(P):
    X = _img_rows(30000, 16, 1)
    a = P.train(dev(X), 32)
    b = P.train(dev(X), 32)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]


# codebook resident in four-wave workgroups, resident in one eight-wave
# workgroup, staged in chunks; ragged row counts
@pytest.mark.parametrize("images,M,N", [(2, 2048, 128), (4, 4000, 1024), (4, 3001, 1200)])
def test_bf16_rescore_close_to_oracle(P, images, M, N):
    X = synth.image_training_set(tuple(range(images)), 256, 256, 8)[:M]  # L = 64
    C = X[synth.distinct_rows(X, N, 1000)]
    idx, mind = P.assign(dev(X), dev(C), P.BF16_RESCORE)
    idx_o, d1, d2 = oracle.assign(X, C.astype(np.float64))
    h = host(idx)
    miss = h != idx_o
    # a miss is allowed only where the BF16 screen could not separate the
    # two best codevectors: the true gap is below the BF16 rounding scale
    gap = (d2 - d1)[miss]
    assert miss.mean() < 0.01
    xx = (X.astype(np.float64) ** 2).sum(1)[miss]
    assert np.all(gap <= 2 ** -6 * (xx + d1[miss] + 1))
    # the FP32 rescore is exact for the chosen codevector on pixel data
    # (integer differences, squares and sums below 2^24)
    Xd = X.astype(np.float64)
    dd = ((Xd - C.astype(np.float64)[h]) ** 2).sum(1)
    np.testing.assert_array_equal(host(mind), dd.astype(np.float32))


# other dimensions: rows of exactly 16 floats, padded rows (33 -> 64, 100 ->
# 128, 8 -> 16), Gaussian-mixture data
@pytest.mark.parametrize("M,L,N", [(3000, 16, 200), (2500, 33, 64), (1500, 100, 40),
                                   (2000, 8, 32), (777, 32, 300)])
def test_bf16_rescore_dimensions(P, M, L, N):
    X = _gmm(M + L, M, L, max(2, N // 4))
    C = X[synth.distinct_rows(X, N, 1001)]
    idx, mind = P.assign(dev(X), dev(C), P.BF16_RESCORE)
    idx_o, d1, d2 = oracle.assign(X, C.astype(np.float64))
    h = host(idx)
    miss = h != idx_o
    assert miss.mean() < 0.01
    xx = (X.astype(np.float64) ** 2).sum(1)[miss]
    assert np.all((d2 - d1)[miss] <= 2 ** -6 * (xx + d1[miss] + 1))
    # the chosen codevector's distance rescored in FP32 (direct form, fused
    # multiply-adds): within (L + 4) units of 2^-24 of the FP64 value
    dd = ((X.astype(np.float64) - C.astype(np.float64)[h]) ** 2).sum(1)
    np.testing.assert_allclose(host(mind), dd, rtol=(L + 4) * 2.0 ** -24, atol=1e-30)


def test_train_bf16_one_update_within_tolerance(P):
    # one Lloyd iteration from the same codebook: the BF16 form's codebook
    # against the exact one (spec bar: relative 1e-3 per codevector)
    X = synth.image_training_set((0, 1, 2, 3), 256, 256, 8)  # M = 4096, L = 64
    C0 = X[synth.distinct_rows(X, 256, 1002)]
    Cb, _, Db, _ = P.train(dev(X), 256, C_init=dev(C0), fixed_iters=1, precision=P.BF16_RESCORE)
    Cf, _, Df, _ = P.train(dev(X), 256, C_init=dev(C0), fixed_iters=1)
    ref = oracle.train(X, 256, C_init=C0.astype(np.float64), fixed_iters=1, store_fp32=True)
    np.testing.assert_array_equal(host(Cf), ref["C"].astype(np.float32))
    cb, cf = host(Cb).astype(np.float64), host(Cf).astype(np.float64)
    rel = np.linalg.norm(cb - cf, axis=1) / np.maximum(np.linalg.norm(cf, axis=1), 1e-30)
    assert rel.max() <= 1e-3
    assert abs(Db - Df) <= 1e-3 * Df


def test_backward_matches_oracle(P):
    X = _gmm(7, 6000, 16, 20)
    rng = np.random.default_rng(7)
    C = X[rng.permutation(6000)[:50]] + 0.5
    idx_o, _, _ = oracle.assign(X, C.astype(np.float64))
    gX, gC = P.distortion_backward(dev(X), dev(C), dev(idx_o.astype(np.int32)), g=1.5)
    rX, rC = oracle.grad(X, C.astype(np.float64), idx_o, g=1.5)
    np.testing.assert_allclose(host(gX), rX, rtol=2 ** -22, atol=1e-30)
    np.testing.assert_allclose(host(gC), rC, rtol=2 ** -22, atol=1e-12)


def test_train_graph_replays_match_eager(P):
    # On a non-default stream the iterations run as a captured hipGraph,
    # replayed many times per run and reused across runs; every run must
    # equal the eager (graph-free) run and the oracle, with other GPU work
    # and synchronisations between the runs.
    X = synth.image_training_set((2,), 256, 256, 4)
    Xd = dev(X)
    ref = oracle.train(X, 32, store_fp32=True)
    eager = P.train(Xd, 32)
    np.testing.assert_array_equal(host(eager[0]), ref["C"].astype(np.float32))
    side = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(side):
            C, idx, D, st = P.train(Xd, 32, graph=True)
        side.synchronize()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(C), host(eager[0]))
        np.testing.assert_array_equal(host(idx), host(eager[1]))
        assert D == eager[2]
        assert st["level_iters"] == eager[3]["level_iters"]
        _ = (Xd * 2).sum().item()  # unrelated eager work between runs
    # timing through graph-captured events
    with torch.cuda.stream(side):
        C, idx, D, st = P.train(Xd, 32, timing=True, graph=True)
    side.synchronize()
    np.testing.assert_array_equal(host(C), host(eager[0]))
    assert st["ms_assign"] > 0 and st["ms_update"] > 0


@pytest.mark.parametrize("M,L,N,kind", [(4096, 16, 64, "img"), (2000, 200, 16, "gmm")])
def test_train_resume_mid_level(P, M, L, N, kind):
    # A run stopped after two updates of its last level and resumed from that
    # codebook with the distortion before the last update (D_prev_init) and
    # the update count (it_init) gives the uninterrupted run bit for bit (the
    # device-controlled loop for L = 16, the host loop for L = 200).
    X = _config0() if kind == "img" else np.rint(_gmm(5, M, L, 12)).astype(np.float32)
    C, idx, D, st = P.train(dev(X), N)
    li = st["level_iters"]
    assert li[-1] >= 3, li
    C2, _, _, st1 = P.train(dev(X), N, forced_iters=li[:-1] + [2])
    D_prev = st1["D_trace"][-2]
    Cr, idxr, Dr, str_ = P.train(dev(X), N, C_init=C2, D_prev_init=D_prev, it_init=2)
    assert str_["level_iters"] == [li[-1]]
    assert torch.equal(Cr, C) and torch.equal(idxr, idx) and Dr == D
    ref = oracle.train(X, N, store_fp32=True)
    np.testing.assert_array_equal(host(Cr), ref["C"].astype(np.float32))


def test_train_statistics(P):
    # empty cells and near-tie rows of the final allocation, against the
    # oracle's allocation and FP64 top-two distances for the same codebook
    for X, N in [(_config0(), 64), (_img_rows(40, 16, 2), 64), (_gmm(8, 3000, 8, 6), 32)]:
        C, idx, D, st = P.train(dev(X), N, stats_ties=True)
        Ch = host(C).astype(np.float64)
        io, d1, d2 = oracle.assign(X, Ch)
        np.testing.assert_array_equal(host(idx), io)
        counts = np.bincount(io, minlength=N)
        assert st["empty_cells"] == int((counts == 0).sum())
        xx = (X.astype(np.float64) ** 2).sum(1)
        assert st["near_tie_rows"] == int(((d2 - d1) < 1e-6 * xx).sum())
        _, _, _, st0 = P.train(dev(X), N)
        assert st0["near_tie_rows"] == -1 and st0["empty_cells"] == st["empty_cells"]


def test_update_dimension_slices_misaligned(P):
    # N = 1024, L = 64: the cells' sums are formed in 16-dimension slices;
    # X 16-byte aligned (vector loads) and offset by one float (scalar loads)
    rng = np.random.default_rng(77)
    M, L, n = 20000, 64, 1024
    X = np.rint(_gmm(3, M, L, 8)).astype(np.float32)
    idx = rng.integers(0, n - 5, size=M).astype(np.int32)
    C_old = rng.normal(size=(n, L)).astype(np.float32)
    want, cnt = oracle.update(X, idx, C_old.astype(np.float64), store_fp32=True)
    flat = torch.empty(M * L + 1, dtype=torch.float32, device="cuda")
    Xm = flat[1:].view(M, L)
    Xm.copy_(dev(X))
    assert Xm.data_ptr() % 16 != 0
    for Xd in (dev(X), Xm):
        C_new, counts = P.update(Xd, dev(idx), dev(C_old))
        np.testing.assert_array_equal(host(counts), cnt)
        np.testing.assert_array_equal(host(C_new), want.astype(np.float32))


def _grid_bits(X, M):
    """(e, g, b) of the update's 32-bit condition, from the data alone:
    max|x| < 2^e, every coordinate a multiple of 2^-g (g as small as
    possible), M < 2^b.  The cell sums fit 32 bits when e + g + b <= 31."""
    a = np.abs(X[X != 0].astype(np.float64))
    e = int(np.frexp(a.max())[1])
    m, E = np.frexp(a)
    sig = (m * 2.0 ** 53).astype(np.uint64)
    tz = np.zeros(sig.shape, np.int64)
    s = sig.copy()
    while np.any(s & np.uint64(1) == 0):
        z = (s & np.uint64(1)) == 0
        tz += z
        s = np.where(z, s >> np.uint64(1), s)
    g = int((-(E - 53 + tz)).max())
    return e, g, int(M).bit_length()


# Whole Lloyd iterations from a given codebook on data whose cell sums do or
# do not fit 32 bits: the update then sums 32-dimension slices in 32-bit
# words, or 16-dimension slices in 64-bit words; either way the sums are
# exact and the runs equal the oracle's (FP32 codebook storage) bit for bit.
# Signed integers at the limit e + g + b = 31 and one bit past it, eighths
# (g = 3) at L = 96 (three 32-bit slices), multiples of 4 (g = -2) at L = 32
# (one slice), and X offset by one float (scalar loads).
@pytest.mark.parametrize("case", ["limit", "past_limit", "eighths", "fours", "misaligned"])
def test_train_32bit_slices_match_oracle(P, case):
    rng = np.random.default_rng({"limit": 31, "past_limit": 32, "eighths": 33, "fours": 34,
                                 "misaligned": 35}[case])
    if case in ("limit", "past_limit", "misaligned"):
        M, L, N = 4096, 64, 256
        top = 2 ** 18 - 1 if case != "past_limit" else 2 ** 19 - 1
        X = np.rint(_gmm(21, M, L, 12) * (top / 4.0))
        X = np.clip(X, -top, top)
        X[0, 0], X[1, 1] = top, -top
        X = X.astype(np.float32)
        want = case != "past_limit"
    elif case == "eighths":
        M, L, N = 3001, 96, 256
        X = (np.rint(_gmm(22, M, L, 10) * 800.0) / 8.0).astype(np.float32)
        want = True
    else:
        M, L, N = 5000, 32, 512
        X = (np.rint(_gmm(23, M, L, 16) * 50.0) * 4.0).astype(np.float32)
        want = True
    e, g, b = _grid_bits(X, M)
    assert (e + g + b <= 31) == want, (e, g, b)
    C0 = X[rng.permutation(M)[:N]] + rng.normal(size=(N, L)).astype(np.float32)
    ref = oracle.train(X, N, C_init=C0.astype(np.float64), fixed_iters=4, store_fp32=True)
    Xd = dev(X)
    if case == "misaligned":
        flat = torch.empty(M * L + 1, dtype=torch.float32, device="cuda")
        Xd = flat[1:].view(M, L)
        Xd.copy_(dev(X))
        assert Xd.data_ptr() % 16 != 0
    C, idx, D, st = P.train(Xd, N, C_init=dev(C0), fixed_iters=4)
    assert st["level_iters"] == [4]
    np.testing.assert_array_equal(host(idx), ref["idx"])
    np.testing.assert_array_equal(host(C), ref["C"].astype(np.float32))
    assert abs(D - ref["D"]) <= 1e-12 * ref["D"]
