"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each ``pin_*`` function takes a loaded oracle library and raises
AssertionError when the oracle disagrees with the paper or the mathematics:
exact rational brute force on tiny inputs, closed forms, a hand-worked
example, invariants and special cases that reduce to NumPy routines.  They
are collected by ``test_oracle_pins.py`` and re-run against deliberately
broken copies of the oracle by ``test_oracle_mutants.py``.
"""

from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ----------------------------------------------------------------------------
# exact rational brute force (shares nothing with the oracle)
# ----------------------------------------------------------------------------

def _frac_rows(A):
    return [[Fraction(float(v)) for v in row] for row in np.asarray(A)]


def _brute_assign(Xf, Cf):
    idx, d1, d2 = [], [], []
    for x in Xf:
        ds = [sum((a - b) * (a - b) for a, b in zip(x, c)) for c in Cf]
        best = min(ds)
        k = ds.index(best)            # first index attaining the minimum
        rest = ds[:k] + ds[k + 1:]
        idx.append(k)
        d1.append(best)
        d2.append(min(rest) if rest else None)
    return idx, d1, d2


def _tiny_case(rng, with_ties):
    M = int(rng.integers(1, 41))
    L = int(rng.integers(1, 5))
    n = int(rng.integers(1, 9))
    X = rng.integers(-6, 7, size=(M, L)).astype(np.float32)
    C = rng.integers(-12, 13, size=(n, L)).astype(np.float64) / 2.0
    if with_ties and n >= 2:
        # duplicated codevectors and training vectors midway between two
        # codevectors give exact distance ties
        C[-1] = C[0]
        a = rng.integers(-3, 4, size=L) * 2.0
        b = rng.integers(-3, 4, size=L) * 2.0
        C[0], C[1 % n] = a, b
        X[0] = ((a + b) / 2).astype(np.float32)
    return X, C


def pin_brute_assign(lib):
    """Cell Allocation vs exact rationals: index (lowest index on ties),
    winning distance and second distance, on random tiny integer inputs
    including exact ties."""
    rng = np.random.default_rng(1)
    for t in range(60):
        X, C = _tiny_case(rng, with_ties=(t % 2 == 1))
        idx, d1, d2 = oracle.assign(X, C, lib=lib)
        bi, bd1, bd2 = _brute_assign(_frac_rows(X), _frac_rows(C))
        assert list(idx) == bi, (t, list(idx), bi)
        assert all(Fraction(float(a)) == b for a, b in zip(d1, bd1)), t
        for a, b in zip(d2, bd2):
            if b is None:
                assert math.isinf(a)
            else:
                assert Fraction(float(a)) == b, t


def pin_brute_update_distortion(lib):
    """Codebook Updation and average distortion vs exact rationals: each
    codevector is the mean of its cell (correctly rounded), an empty cell keeps
    its codevector, D is the exact mean squared distance (correctly rounded)."""
    rng = np.random.default_rng(2)
    for t in range(40):
        X, C = _tiny_case(rng, with_ties=False)
        M, L = X.shape
        n = C.shape[0]
        idx = rng.integers(0, n, size=M).astype(np.int32)
        Cn, cnt = oracle.update(X, idx, C, lib=lib)
        Xf = _frac_rows(X)
        for k in range(n):
            members = [Xf[m] for m in range(M) if idx[m] == k]
            assert cnt[k] == len(members)
            for l in range(L):
                if members:
                    exact = sum(r[l] for r in members) / len(members)
                    assert Cn[k, l] == float(exact), (t, k, l)
                else:
                    assert Cn[k, l] == C[k, l]
        assert int(cnt.sum()) == M
        Cf = _frac_rows(C)
        exactD = sum(sum((a - b) ** 2 for a, b in zip(Xf[m], Cf[idx[m]]))
                     for m in range(M)) / M
        assert oracle.distortion(X, C, idx, lib=lib) == float(exactD), t


def _lbg_rational(Xf, N, thr, eps, max_iter=200):
    """Exact-rational LBG on tiny inputs (Algorithm 1 with the readings of
    the oracle).  Returns (C, idx, D, per-level updates) or None when an
    exact distance tie makes the FP64 run ill-defined."""
    M, L = len(Xf), len(Xf[0])
    C = [[sum(x[l] for x in Xf) / M for l in range(L)]]
    levels = []
    e = Fraction(eps)
    D = None
    idx = None
    while len(C) < N:
        C2 = []
        for c in C:
            C2.append([v * (1 + e) for v in c])
            C2.append([v * (1 - e) for v in c])
        C = C2
        D_prev, first, it = None, True, 0
        while True:
            idx, D = [], Fraction(0)
            for x in Xf:
                ds = [sum((a - b) ** 2 for a, b in zip(x, c)) for c in C]
                best = min(ds)
                if ds.count(best) > 1:
                    return None
                idx.append(ds.index(best))
                D += best
            D /= M
            if not first and (D_prev - D) <= thr * D_prev:
                break
            if it >= max_iter:
                break
            newC = []
            for k, c in enumerate(C):
                mem = [Xf[m] for m in range(M) if idx[m] == k]
                newC.append([sum(r[l] for r in mem) / len(mem) for l in range(L)]
                            if mem else c)
            C, D_prev, first, it = newC, D, False, it + 1
        levels.append(it)
    return C, idx, D, levels


def pin_brute_train(lib):
    """Whole LBG run with splitting vs an exact-rational run on tiny random
    inputs (runs whose rational trajectory meets an exact tie are skipped)."""
    rng = np.random.default_rng(3)
    done = 0
    for t in range(40):
        M = int(rng.integers(4, 13))
        L = int(rng.integers(1, 3))
        N = int(rng.choice([2, 4]))
        X = rng.integers(0, 20, size=(M, L)).astype(np.float32)
        ref = _lbg_rational(_frac_rows(X), N, Fraction(1, 1000), 0.01)
        if ref is None:
            continue
        Cr, ir, Dr, lv = ref
        out = oracle.train(X, N, thr=1e-3, eps_split=0.01, lib=lib)
        assert list(out["idx"]) == ir, t
        assert list(out["level_iters"]) == lv, (t, list(out["level_iters"]), lv)
        for k in range(N):
            for l in range(L):
                assert abs(out["C"][k, l] - float(Cr[k][l])) <= 1e-12 * (1 + abs(float(Cr[k][l]))), t
        assert abs(out["D"] - float(Dr)) <= 1e-12 * (1 + float(Dr)), t
        done += 1
    assert done >= 15, done


# ----------------------------------------------------------------------------
# hand-worked example (tests/golden)
# ----------------------------------------------------------------------------

def _read_golden(name):
    X, levels = None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rest = line.split(":", 1)
            if key == "X":
                X = [Fraction(v) for v in rest.split()]
            elif key == "level":
                head, cb, al, d = [s.strip() for s in rest.split("|")]
                n, upd = [int(v) for v in head.split()]
                levels.append(dict(n=n, updates=upd,
                                   C=[Fraction(v) for v in cb.split()],
                                   idx=[int(v) for v in al.split()],
                                   D=Fraction(d)))
    return X, levels


def pin_golden_tiny_1d(lib):
    """The hand-worked two-level run of tests/golden/tiny_1d_two_levels.txt."""
    Xg, levels = _read_golden("tiny_1d_two_levels.txt")
    X = np.array([[float(v)] for v in Xg], np.float32)
    for lv in levels:
        out = oracle.train(X, lv["n"], thr=1e-3, eps_split=0.01, lib=lib)
        assert out["status"] == oracle.OK
        assert list(out["idx"]) == lv["idx"]
        assert int(out["level_iters"][-1]) == lv["updates"]
        for k, c in enumerate(lv["C"]):
            assert abs(out["C"][k, 0] - float(c)) <= 1e-14 * (1 + abs(float(c)))
        assert abs(out["D"] - float(lv["D"])) <= 1e-14


# ----------------------------------------------------------------------------
# closed forms and special cases
# ----------------------------------------------------------------------------

def pin_centroid_and_single_level(lib):
    """Initialization is the column mean (Table 1); at N = 1 the distortion is
    the summed per-dimension variance (ddof = 0)."""
    rng = np.random.default_rng(4)
    X = (rng.normal(size=(3000, 7)) * 3 + 5).astype(np.float32)
    c0 = oracle.centroid(X, lib=lib)
    ref = X.astype(np.float64).mean(axis=0)
    assert np.allclose(c0[0], ref, rtol=1e-13, atol=1e-13)
    out = oracle.train(X, 1, lib=lib)
    var = X.astype(np.float64).var(axis=0).sum()
    assert abs(out["D"] - var) <= 1e-11 * var
    assert np.all(out["idx"] == 0)


def pin_split(lib):
    """Codebook Splitting doubles the codebook: rows 2i and 2i+1 are the "+" and
    "-" children of row i, symmetric about it, apart by 2*eps*|c| (multiplicative)
    or 2*delta (additive)."""
    rng = np.random.default_rng(5)
    C = rng.normal(size=(9, 5)) * 4
    for mode, eps, delta in [(oracle.SPLIT_MULT, 0.01, 0.0), (oracle.SPLIT_MULT, 0.2, 0.0),
                             (oracle.SPLIT_ADD, 0.0, 0.37)]:
        C2 = oracle.split(C, eps=eps, mode=mode, delta=delta, lib=lib)
        assert C2.shape == (18, 5)
        up, dn = C2[0::2], C2[1::2]
        assert np.allclose((up + dn) / 2, C, rtol=1e-15, atol=1e-15)
        want = 2 * eps * C if mode == oracle.SPLIT_MULT else np.full_like(C, 2 * delta)
        assert np.allclose(up - dn, want, rtol=1e-13, atol=1e-14)
    f = oracle.split(C, eps=0.01, store_fp32=True, lib=lib)
    assert np.all(f == f.astype(np.float32).astype(np.float64))


def pin_uniform_grid_two_levels(lib):
    """Closed form: uniform grid x_j = (j + 1/2)/M on [0, 1], N = 2.  The split
    of the mean 1/2 separates the halves, the update gives [3/4, 1/4] ("+" child
    first) and the run stops on the next unchanged allocation: 3 allocations,
    2 updates, D = 1/48 - 1/(12 M^2)."""
    M = 1024
    X = ((np.arange(M) + 0.5) / M).astype(np.float32)[:, None]
    out = oracle.train(X, 2, thr=1e-3, eps_split=0.01, lib=lib)
    assert out["C"][0, 0] == 0.75 and out["C"][1, 0] == 0.25
    assert list(out["level_iters"]) == [2]
    assert len(out["D_trace"]) == 3
    exact = Fraction(1, 48) - Fraction(1, 12 * M * M)
    assert out["D"] == float(exact)
    assert out["D_trace"][1] == out["D_trace"][2] == float(exact)


def pin_point_masses_zero_distortion(lib):
    """Two point masses p < q with positive mean, N = 2: the run must end with
    C = [q, p] and D = 0.  This pins the '<=' form of the stop test: with D_prev
    = D = 0 only (D_prev - D) <= thr * D_prev terminates."""
    X = np.array([[1.0]] * 5 + [[3.0]] * 3, np.float32)
    out = oracle.train(X, 2, thr=1e-3, max_iter=50, lib=lib)
    assert out["status"] == oracle.OK
    assert list(out["C"][:, 0]) == [3.0, 1.0]
    assert out["D"] == 0.0
    assert list(out["level_iters"]) == [2]


def pin_gaussian_lloyd_max(lib):
    """Level 2 of LBG on a 1-D Gaussian N(m0, s^2) converges to the two-level
    Lloyd-Max quantizer m0 +/- s*sqrt(2/pi) with distortion s^2 (1 - 2/pi);
    tolerance is sampling error only."""
    M, m0, s = 400_000, 3.0, 2.0
    rng = np.random.default_rng(6)
    X = (m0 + s * rng.standard_normal(M)).astype(np.float32)[:, None]
    out = oracle.train(X, 2, thr=1e-9, lib=lib)
    tol = 5 * s / math.sqrt(M)
    assert abs(out["C"][0, 0] - (m0 + s * math.sqrt(2 / math.pi))) < tol
    assert abs(out["C"][1, 0] - (m0 - s * math.sqrt(2 / math.pi))) < tol
    assert abs(out["D"] - s * s * (1 - 2 / math.pi)) < 5 * s * s / math.sqrt(M)


def pin_uniform_quantizer_fixed_point(lib):
    """The uniform N-level quantizer {(2i+1)/(2N)} is a fixed point of one
    allocation + update on the uniform grid when N divides M."""
    M, N = 1024, 8
    X = ((np.arange(M) + 0.5) / M).astype(np.float32)[:, None]
    C = ((2 * np.arange(N) + 1) / (2 * N))[:, None]
    idx, _, _ = oracle.assign(X, C, lib=lib)
    Cn, cnt = oracle.update(X, idx, C, lib=lib)
    assert np.array_equal(Cn, C)
    assert np.all(cnt == M // N)


def pin_update_matches_numpy(lib):
    """Updation on real-valued data: codevectors equal NumPy masked means,
    empty cells keep their old value, counts equal the bincount and sum to M."""
    rng = np.random.default_rng(7)
    X = (rng.normal(size=(5000, 6)) * 10).astype(np.float32)
    n = 37
    idx = rng.integers(0, n - 3, size=5000).astype(np.int32)   # last 3 cells empty
    C = rng.normal(size=(n, 6))
    Cn, cnt = oracle.update(X, idx, C, lib=lib)
    assert np.array_equal(cnt, np.bincount(idx, minlength=n))
    assert cnt.sum() == 5000
    for k in range(n):
        if cnt[k]:
            assert np.allclose(Cn[k], X[idx == k].astype(np.float64).mean(0), rtol=1e-12, atol=1e-12)
        else:
            assert np.array_equal(Cn[k], C[k])


def pin_assign_matches_numpy(lib):
    """Allocation on real-valued data equals NumPy's argmin of the squared
    distance matrix (first index on ties) and min / second-min values."""
    rng = np.random.default_rng(8)
    X = (rng.normal(size=(700, 5)) * 3).astype(np.float32)
    C = rng.normal(size=(23, 5)) * 3
    idx, d1, d2 = oracle.assign(X, C, lib=lib)
    Dm = ((X.astype(np.float64)[:, None, :] - C[None]) ** 2).sum(-1)
    assert np.array_equal(idx, Dm.argmin(1))
    s = np.sort(Dm, axis=1)
    assert np.allclose(d1, s[:, 0], rtol=1e-13)
    assert np.allclose(d2, s[:, 1], rtol=1e-13)


# ----------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------

def _small_image_set():
    """4x4 blocks of the 128 x 128 top-left corner of a 512 x 512 synthetic
    picture (M = 1024, L = 16, integer values 0..255)."""
    import synth
    return synth.blocks(synth.image(0, 512, 512)[:128, :128], 4).astype(np.float32)


def pin_monotone_and_split_bound(lib):
    """Within a level the distortion never increases (Lloyd descent); across a
    split the first distortion is at most the last one plus
    eps^2 * M^-1 sum ||c_a||^2 (each vector may keep the '+' or '-' copy of its
    codevector)."""
    X = _small_image_set()
    eps = 0.01
    full = oracle.train(X, 16, thr=1e-3, eps_split=eps, lib=lib)
    D = full["D_trace"]
    pos = 0
    prev_last = None
    prev_level_C = None
    for n, its in zip(full["level_n"], full["level_iters"]):
        seg = D[pos:pos + its + 1]
        pos += its + 1
        assert np.all(seg[1:] <= seg[:-1] * (1 + 1e-12)), n
        if prev_last is not None:
            idx, _, _ = oracle.assign(X, prev_level_C, lib=lib)
            cn = (prev_level_C[idx] ** 2).sum(1).mean()
            assert seg[0] <= prev_last + eps * eps * cn * (1 + 1e-12), n
        prev_last = seg[-1]
        prev_level_C = oracle.train(X, int(n), thr=1e-3, eps_split=eps, lib=lib)["C"]
    assert pos == len(D)


def pin_thread_count_invariance(lib):
    """The parallel allocation does not change the result (the paper's claim
    that distributing the work does not raise the distortion): every output is
    bit-identical for 1, 2, 3 and 8 threads."""
    X = _small_image_set()
    ref = oracle.train(X, 16, nthreads=1, lib=lib)
    for nt in (2, 3, 8):
        out = oracle.train(X, 16, nthreads=nt, lib=lib)
        assert np.array_equal(out["C"], ref["C"])
        assert np.array_equal(out["idx"], ref["idx"])
        assert out["D"] == ref["D"]
        assert np.array_equal(out["D_trace"], ref["D_trace"])


def pin_zero_threshold_fixed_point(lib):
    """With threshold 0 a level ends only at a fixed point: re-allocating with
    the returned codebook gives the returned allocation, and updating it gives
    the codebook back on every non-empty cell."""
    rng = np.random.default_rng(9)
    X = np.concatenate([rng.normal(loc=c, size=(200, 2)) for c in
                        ([0, 0], [6, 1], [2, 7], [9, 9])]).astype(np.float32)
    out = oracle.train(X, 4, thr=0.0, lib=lib)
    idx, _, _ = oracle.assign(X, out["C"], lib=lib)
    assert np.array_equal(idx, out["idx"])
    Cn, cnt = oracle.update(X, idx, out["C"], lib=lib)
    assert np.array_equal(Cn[cnt > 0], out["C"][cnt > 0])


def pin_store_fp32(lib):
    """With FP32 codebook storage every returned codevector is an FP32 value and
    the run stays within FP32 rounding of the FP64 run."""
    X = _small_image_set()
    a = oracle.train(X, 8, store_fp32=True, lib=lib)
    b = oracle.train(X, 8, store_fp32=False, lib=lib)
    assert np.all(a["C"] == a["C"].astype(np.float32).astype(np.float64))
    assert np.allclose(a["C"], b["C"], rtol=1e-5, atol=1e-5)
    assert abs(a["D"] - b["D"]) <= 1e-6 * b["D"]


def pin_gradient_finite_differences(lib):
    """The gradient of D(C, X) = mean_m min_k ||x_m - c_k||^2 equals central
    finite differences of D computed by NumPy (D is piecewise quadratic, so the
    difference is exact up to rounding while no allocation changes)."""
    rng = np.random.default_rng(10)
    X = (rng.normal(size=(60, 3)) * 4).astype(np.float32)
    C = rng.normal(size=(5, 3)) * 4
    idx, d1, d2 = oracle.assign(X, C, lib=lib)
    gX, gC = oracle.grad(X, C, idx, g=1.7, lib=lib)

    def D(Xd, Cd):
        return 1.7 * ((Xd[:, None, :] - Cd[None]) ** 2).sum(-1).min(1).mean()

    Xd = X.astype(np.float64)
    h = 1e-5
    for k in range(C.shape[0]):
        for l in range(3):
            Cp, Cm = C.copy(), C.copy()
            Cp[k, l] += h
            Cm[k, l] -= h
            fd = (D(Xd, Cp) - D(Xd, Cm)) / (2 * h)
            assert abs(fd - gC[k, l]) <= 1e-6 * (1 + abs(fd)), (k, l, fd, gC[k, l])
    for m in range(0, 60, 7):
        for l in range(3):
            Xp, Xm = Xd.copy(), Xd.copy()
            Xp[m, l] += h
            Xm[m, l] -= h
            fd = (D(Xp, C) - D(Xm, C)) / (2 * h)
            assert abs(fd - gX[m, l]) <= 1e-6 * (1 + abs(fd)), (m, l)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
