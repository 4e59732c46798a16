"""Batched form (many independent LBG runs per launch) on the GPU.

Bar: every instance's codebook, allocation, distortion and iteration counts
are bit-identical to lbg_train on that instance alone (the batched kernels
reproduce the single run's tiles, partial sums and integer cell sums), for
any launch configuration; on integer-valued data the runs also equal the
FP64 oracle with FP32 codebook storage.
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


# (M, L, N, seed): mixed dimensions (vector and scalar loads), codebook
# sizes from 1 to 256, more codevectors than vectors, one row, ragged tiles.
CASES = [
    (3000, 16, 64, 1),
    (500, 64, 16, 2),
    (40000, 16, 256, 3),
    (7000, 64, 256, 4),
    (100, 5, 8, 5),
    (2048, 33, 32, 6),
    (50, 16, 128, 7),
    (4096, 64, 1, 8),
    (1, 16, 1, 9),
    (9000, 8, 2, 10),
    (130, 12, 4, 11),
]


def _data(cases):
    out = []
    for M, L, N, seed in cases:
        X = synth.gmm(seed, M, L, max(1, min(N, 32)))
        out.append((X, N))
    return out


def _single(P, X, N):
    C, idx, D, st = P.train(dev(X), N)
    return C, idx, D, st


def _same(P, got, X, N, where):
    C, idx, D, info = got
    C1, idx1, D1, st1 = _single(P, X, N)
    assert torch.equal(C, C1), f"{where}: codebook differs"
    assert torch.equal(idx, idx1), f"{where}: allocation differs"
    assert D == D1, f"{where}: D {D!r} vs {D1!r}"
    assert info["n_assign"] == st1["total_assigns"], where
    assert info["n_update"] == st1["total_updates"], where
    assert info["n_levels"] == len(st1["level_n"]), where
    assert info["status"] == st1["status"], where


def test_batched_equals_single_runs(P):
    data = _data(CASES)
    res, stats = P.train_batched([dev(X) for X, _ in data], [N for _, N in data])
    assert stats["grab"] >= 1 and stats["grid"] >= 1
    for (X, N), got, case in zip(data, res, CASES):
        _same(P, got, X, N, f"case {case}")


# screen 1: FP32 screen; 2: split BF16 screen where its codebook layout fits
# (both exact, so the allocations, and everything after them, are the same)
@pytest.mark.parametrize("grab,grid,graph,screen", [(1, 256, False, 1), (16, 512, True, 2),
                                                    (3, 97, True, 2), (4, 256, False, 2)])
def test_batched_configuration_does_not_change_results(P, grab, grid, graph, screen):
    data = _data(CASES)
    ref, _ = P.train_batched([dev(X) for X, _ in data], [N for _, N in data], grab=1, grid=512,
                             graph=False, screen=1)
    # graphs are captured on non-default streams only
    side = torch.cuda.Stream()
    Xs = [dev(X) for X, _ in data]
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        got, st = P.train_batched(Xs, [N for _, N in data], grab=grab, grid=grid, graph=graph,
                                  screen=screen)
        got2, _ = P.train_batched(Xs, [N for _, N in data], grab=grab, grid=grid, graph=graph,
                                  screen=screen)
    side.synchronize()
    assert st["grab"] == grab and st["grid"] == grid and st["graph"] == (1 if graph else 0)
    assert st["screen"] == screen
    for a, b in zip(got, got2):  # a second call replays the cached graph
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]
    for a, b in zip(ref, got):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]


def test_batched_timing_keeps_results(P):
    data = _data(CASES[:4])
    ref, _ = P.train_batched([dev(X) for X, _ in data], [N for _, N in data])
    got, st = P.train_batched([dev(X) for X, _ in data], [N for _, N in data], timing=True)
    assert st["graph"] == 0 and st["ms_assign"] > 0 and st["ms_update"] > 0
    for a, b in zip(ref, got):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]
        assert b[3]["distances"] > 0


def test_batched_matches_oracle_on_images(P):
    img = synth.blocks(synth.image(0, 512, 512), 4).astype(np.float32)
    sets = [(img[:4096], 64), (img[4096:6144], 16), (img[8192:20480], 128)]
    res, _ = P.train_batched([dev(X) for X, _ in sets], [N for _, N in sets])
    for (X, N), (C, idx, D, info) in zip(sets, res):
        r = oracle.train(X, N, store_fp32=True)
        np.testing.assert_array_equal(C.cpu().numpy(), r["C"].astype(np.float32))
        np.testing.assert_array_equal(idx.cpu().numpy(), r["idx"])
        assert abs(D - r["D"]) <= 1e-12 * max(1.0, abs(r["D"]))


def test_batched_many_instances(P):
    inst = synth.batched_instances(48, scale=0.05)
    res, st = P.train_batched([dev(X) for X, _ in inst], [N for _, N in inst])
    assert st["total_distances"] > 0
    for k in (0, 7, 19, 33, 47):
        X, N = inst[k]
        _same(P, res[k], X, N, f"instance {k}")


def test_batched_more_instances_than_one_list_workgroup(P):
    # 1100 small instances: the round's finish list is built 1024 instances at
    # a time, and the instances stop at different rounds, so the running set
    # shrinks unevenly across both passes
    rng = np.random.default_rng(77)
    inst = []
    for k in range(1100):
        M = int(rng.integers(1, 400))
        L = int(rng.choice([3, 16, 64]))
        N = int(rng.choice([1, 2, 4, 8, 16, 32]))
        inst.append((synth.gmm(1000 + k, M, L, max(1, min(N, 8))), N))
    Xs = [dev(X) for X, _ in inst]
    res, st = P.train_batched(Xs, [N for _, N in inst], grab=2, grid=256)
    assert st["rounds"] > 1
    for k in list(range(0, 1100, 37)) + [1023, 1024, 1099]:
        X, N = inst[k]
        _same(P, res[k], X, N, f"instance {k}")
    got, _ = P.train_batched(Xs, [N for _, N in inst], grab=1, grid=512)
    for a, b in zip(res, got):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]


def test_batched_rejects_bad_instances(P):
    X = dev(np.zeros((100, 16), np.float32))
    with pytest.raises(Exception):
        P.train_batched([X], [6])          # not a power of two
    with pytest.raises(Exception):
        P.train_batched([dev(np.zeros((10, 65), np.float32))], [4])  # L > 64
    with pytest.raises(Exception):
        P.train_batched([dev(np.zeros((10, 64), np.float32))], [512])  # codebook too large


# items of the batched single steps: ragged M (1, 31, 33, several tiles), L
# from 1 to 64 (vector and scalar rows), codebooks of 1 to 256 codevectors
# (the direct search up to 8), Gaussian mixtures; one item with a non-finite
# row, one with a misaligned X
STEP_ITEMS = [(1, 16, 1, 21), (31, 16, 8, 22), (33, 64, 9, 23), (5000, 16, 256, 24),
              (4097, 64, 100, 25), (700, 5, 3, 26), (2048, 33, 40, 27), (9000, 1, 7, 28),
              (3001, 64, 256, 29), (1500, 12, 17, 30)]


def _step_data():
    rng = np.random.default_rng(99)
    Xs, Cs = [], []
    for M, L, N, seed in STEP_ITEMS:
        X = synth.gmm(seed, max(M, N), L, max(1, N // 2))[:M]
        C = X[rng.integers(0, M, N)] + rng.normal(0, 1, (N, L)).astype(np.float32)
        Xs.append(np.ascontiguousarray(X))
        Cs.append(np.ascontiguousarray(C.astype(np.float32)))
    Xs[3][17, 2] = np.nan
    return Xs, Cs


def test_assign_batched_equals_single_calls(P):
    Xs, Cs = _step_data()
    Xd = [dev(X) for X in Xs]
    # a misaligned training set: the rows of a larger buffer from offset 1
    big = dev(np.concatenate([np.zeros(1, np.float32), Xs[1].ravel()]))
    Xd[1] = big[1:].view(Xs[1].shape)
    Cd = [dev(C) for C in Cs]
    idxs, Ds = P.assign_batched(Xd, Cd)
    for i, (X, C) in enumerate(zip(Xd, Cd)):
        idx1, _, D1 = P.assign_distortion(X, C, P.FP32)
        assert torch.equal(idxs[i], idx1), f"item {i}"
        assert float(Ds[i].item()) == float(D1.item()) or (
            np.isinf(float(D1.item())) and np.isinf(float(Ds[i].item()))), f"item {i}"
    io, _, _ = oracle.assign(Xs[4], Cs[4].astype(np.float64))
    assert np.array_equal(idxs[4].cpu().numpy(), io)
    idxs2, Ds2 = P.assign_batched(Xd, Cd, with_D=False)
    assert all(d is None for d in Ds2)
    assert all(torch.equal(a, b) for a, b in zip(idxs, idxs2))


def test_update_batched_equals_single_calls(P):
    Xs, Cs = _step_data()
    Xs[3][17, 2] = 0.5  # finite data for the update
    Xd = [dev(X) for X in Xs]
    Cd = [dev(C) for C in Cs]
    idxs, _ = P.assign_batched(Xd, Cd, with_D=False)
    idxs[5][3] = -1          # joins no cell
    idxs[6][0] = Cs[6].shape[0]  # outside [0, N): joins no cell
    news, counts = P.update_batched(Xd, idxs, Cd)
    for i, (X, idx, C) in enumerate(zip(Xd, idxs, Cd)):
        C1, n1 = P.update(X, idx, C)
        assert torch.equal(news[i], C1), f"item {i}"
        assert torch.equal(counts[i], n1), f"item {i}"
    ref, rc = oracle.update(Xs[4], idxs[4].cpu().numpy(), Cs[4].astype(np.float64))
    np.testing.assert_array_equal(counts[4].cpu().numpy(), rc)
