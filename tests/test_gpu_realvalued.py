"""Whole LBG runs on real-valued data against the FP64 oracle, and the
contracts for non-finite input and far-away codevectors.

Real-valued data are where the update's fixed-point sums are not trivially
exact: the library sums every coordinate as round(x 2^s) plus, for data off
that grid, a second word round(residual 2^t), and divides once.  The oracle
sums in FP64 in index order.  Bars (the benchmark spec's tolerances, C19/C20 of the
readings):
  * the final allocation equals the oracle's FP64 argmin for the library's
    own final codebook, row for row (the allocation is exact);
  * iteration counts equal the oracle's (FP32 codebook storage); where they
    differ, the oracle's relative change at that level's stop lies within
    1e-6 of the threshold, and the oracle is run in lockstep with the
    library's counts;
  * codebooks: per codevector ||c - c_ref|| / ||c_ref|| <= 1e-5 (absolute
    1e-5 for a zero codevector), end to end against the oracle with FP32
    codebook storage (the library's storage), and per step against the
    oracle with FP64 storage: one FP64 update of the library's final
    codebook against the library's update of it;
  * distortion: relative 1e-6.
End to end, the FP64-storage oracle follows another trajectory wherever a
row sits in the tie band (gap below 1e-6 ||x||^2): a one-row cell split
into two children equidistant from it in exact arithmetic goes to whichever
child the storage rounding favours, and the other child keeps its value, a
2 eps difference that later iterations can amplify.  Such runs are compared
per step (C20, mode i), as above.
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


def _rel_rows(C, R):
    C = np.asarray(C, np.float64)
    R = np.asarray(R, np.float64)
    num = np.linalg.norm(C - R, axis=1)
    den = np.linalg.norm(R, axis=1)
    return np.where(den > 0, num / np.maximum(den, 1e-300), num)


def _check_run(P, X, N, C, idx, D, level_iters, where, tol_c=1e-5):
    """The library's run (C, idx, D, per-level update counts) against the
    oracle.  Returns the lockstep FP32-storage oracle result."""
    Cg = host(C).astype(np.float64)
    ig = host(idx)
    # the final allocation is the exact FP64 argmin for the final codebook
    io, d1, d2 = oracle.assign(X, Cg)
    assert np.array_equal(ig, io), f"{where}: allocation differs from the FP64 argmin"
    # natural stops: equal counts, or the oracle's stop ratio at the first
    # differing level within 1e-6 of the threshold (then lockstep)
    nat = oracle.train(X, N, store_fp32=True)
    if list(nat["level_iters"]) != list(level_iters):
        lv = next(i for i, (a, b) in enumerate(zip(nat["level_iters"], level_iters)) if a != b)
        r = nat["level_stop_ratio"][lv]
        assert abs(r - 1e-3) <= 1e-6, (
            f"{where}: level {lv} stops after {level_iters[lv]} updates, the oracle after "
            f"{nat['level_iters'][lv]} (stop ratio {r!r})")
    ref = oracle.train(X, N, store_fp32=True, forced_iters=list(level_iters))
    r32 = _rel_rows(Cg, ref["C"])
    assert r32.max() <= tol_c, f"{where}: codebook vs FP32-storage oracle {r32.max():.3g}"
    assert abs(D - ref["D"]) <= 1e-6 * abs(ref["D"]), f"{where}: D {D!r} vs {ref['D']!r}"
    # one more step from the library's final codebook: the FP64 oracle's
    # update (FP64 storage) against the library's, and both distortions
    Xd = dev(X)
    Cn, _ = P.update(Xd, idx, C)
    Dg = float(P.distortion(Xd, C, idx).item())
    c64, _ = oracle.update(X, io, Cg)
    rr = _rel_rows(host(Cn), c64)
    assert rr.max() <= tol_c, f"{where}: one update vs the FP64 oracle {rr.max():.3g}"
    d64 = oracle.distortion(X, Cg, io)
    assert abs(Dg - d64) <= 1e-6 * abs(d64) and abs(D - d64) <= 1e-6 * abs(d64), where
    return ref


# (M, L, N, seed): Gaussian mixtures as in the batched workload (means
# U[0,255]^L, sigma U[4, 20]), unrounded FP32
GMM_CASES = [
    (4096, 16, 64, 101),
    (6000, 64, 256, 102),
    (20000, 16, 256, 103),
    (3001, 33, 32, 104),
]


@pytest.mark.parametrize("M,L,N,seed", GMM_CASES)
def test_train_gmm_matches_oracle(P, M, L, N, seed):
    X = synth.gmm(seed, M, L, N)
    C, idx, D, st = P.train(dev(X), N)
    _check_run(P, X, N, C, idx, D, st["level_iters"], f"gmm {M}x{L} N={N}")


def test_train_batched_gmm_matches_oracle(P):
    # twelve instances of the batched workload's generator at full size
    # (M_i from 11,571 to 61,054, L_i in {16, 64}, N_i from 16 to 256; seed
    # 20,000 is M = 50,389, L = 64, N = 256) and four small ones
    inst = synth.batched_instances(8, base_seed=10_000)
    inst += synth.batched_instances(4, base_seed=20_000)
    inst += synth.batched_instances(4, base_seed=30_000, scale=0.05)
    res, stats = P.train_batched([dev(X) for X, _ in inst], [N for _, N in inst])
    for i, ((X, N), (C, idx, D, info)) in enumerate(zip(inst, res)):
        # the per-level counts of the instance come from a single run on it,
        # which the batched form reproduces bit for bit
        C1, idx1, D1, st1 = P.train(dev(X), N)
        assert torch.equal(C, C1) and torch.equal(idx, idx1) and D == D1, f"instance {i}"
        _check_run(P, X, N, C, idx, D, st1["level_iters"], f"instance {i} ({X.shape}, N={N})")


def _wide_range(M=8192, L=16, seed=7):
    # four clusters within 1e-6 of zero (sigma 1e-8) and four near 1e6
    # (sigma 10): one fixed-point word at the shift set by 1e6 would leave
    # the small cells' means off by up to 1e-4 of their size
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 8, M)
    small = np.arange(8) < 4
    means = np.where(small[:, None], rng.uniform(-1e-6, 1e-6, (8, L)),
                     1e6 + rng.uniform(0, 1e3, (8, L)))
    sig = np.where(small, 1e-8, 10.0)
    X = means[lab] + sig[lab, None] * rng.standard_normal((M, L))
    return np.ascontiguousarray(X.astype(np.float32)), lab


def test_update_wide_range_matches_oracle(P):
    X, lab = _wide_range()
    C_old = np.zeros((8, X.shape[1]), np.float32)
    Cn, counts = P.update(dev(X), dev(lab.astype(np.int32)), dev(C_old))
    ref, rc = oracle.update(X, lab.astype(np.int32), C_old.astype(np.float64))
    np.testing.assert_array_equal(host(counts), rc)
    r = _rel_rows(host(Cn), ref)
    # the exact mean rounded to FP32 (plus the FP64 roundings of the sum)
    assert r.max() <= 2.0 ** -22, r


def test_train_wide_range_matches_oracle(P):
    X, _ = _wide_range()
    C, idx, D, st = P.train(dev(X), 8)
    _check_run(P, X, 8, C, idx, D, st["level_iters"], "wide range")


def test_nonfinite_rows_contract(P):
    # a row with a NaN or an infinite coordinate has no finite distance: it is
    # allocated to codevector 0 with distance +inf (the oracle's strict-<
    # search from +inf gives the same), in every form of the allocation
    rng = np.random.default_rng(5)
    for L, n in [(16, 4), (16, 40), (64, 300), (200, 9)]:
        X = rng.uniform(0, 255, (300, L)).astype(np.float32)
        X[3, 1] = np.nan
        X[77, 0] = np.inf
        X[150, L - 1] = -np.inf
        C = X[rng.permutation(300)[:n]].copy()
        C[np.isnan(C).any(1) | np.isinf(C).any(1)] = 1.0
        io, d1, _ = oracle.assign(X, C.astype(np.float64))
        for prec in ([P.FP32, P.BF16_RESCORE] if L <= 128 else [P.FP32]):
            idx, mind = P.assign(dev(X), dev(C), prec)
            ig, mg = host(idx), host(mind)
            for r in (3, 77, 150):
                assert ig[r] == 0 and io[r] == 0 and mg[r] == np.inf and d1[r] == np.inf, (L, n, r)
            if prec == P.FP32:
                np.testing.assert_array_equal(ig, io)
        idx, _, Dd = P.assign_distortion(dev(X), dev(C))
        assert float(Dd.item()) == np.inf
    # training stops at the first allocation and reports LBG_EINVAL
    X = synth.gmm(9, 2000, 16, 8)
    X[10, 3] = np.nan
    with pytest.raises(P.LBGError, match="not finite"):
        P.train(dev(X), 8)
    Xs = [synth.gmm(11, 1500, 16, 4), X, synth.gmm(12, 900, 64, 8)]
    res, stats = P.train_batched([dev(a) for a in Xs], [4, 8, 8])
    assert stats["status"] == P.EINVAL
    assert res[1][3]["status"] == P.EINVAL
    for i in (0, 2):
        C1, idx1, D1, _ = P.train(dev(Xs[i]), [4, 8, 8][i])
        assert res[i][3]["status"] == P.OK
        assert torch.equal(res[i][0], C1) and torch.equal(res[i][1], idx1) and res[i][2] == D1


@pytest.mark.parametrize("c", [3.0, -250.0, 1e7, -3e9])
def test_backward_far_codevector(P, c):
    # dD/dC for a codevector far outside the data (uniform in [0, 1), M = 2e6):
    # count * c is far beyond the fixed-point sums' range; the closed form
    # 2/M sum (c - x) in FP64
    rng = np.random.default_rng(21)
    M, L = 2_000_000, 4
    X = rng.random((M, L), dtype=np.float32)
    C = np.array([[c] * L, [0.5] * L], np.float32)
    idx = np.zeros(M, np.int32)
    idx[M // 2:] = 1
    gX, gC = P.distortion_backward(dev(X), dev(C), dev(idx), 1.0)
    _, gref = oracle.grad(X, C.astype(np.float64), idx, 1.0)
    got = host(gC).astype(np.float64)
    np.testing.assert_allclose(got[0], gref[0], rtol=1e-6)
    # the other cell: codevector at the data's mean, where cancellation
    # leaves a small gradient -- compared on the scale of the cell's terms
    assert np.abs(got[1] - gref[1]).max() <= 1e-6 * (2.0 / M) * (M // 2) * 0.5
