"""FP64 CPU oracle of LBG codebook design -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps ``lbg_oracle.c`` (plain C, FP64)
through ctypes and shares no code with the GPU library.

Every function states the passage of the paper (Annaji & Rao, "Parallelization
of the LBG Vector Quantization Algorithm for Shared Memory Systems") it
follows; the C source lists the readings taken where the paper is silent.
"""

from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbg_oracle.c")
_LIB = os.path.join(_HERE, "liblbg_oracle.so")
_lock = threading.Lock()
_lib = None

SPLIT_MULT = 0
SPLIT_ADD = 1
OK = 0
EINVAL = -1
WMAXITER = 1


def build(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math,
    no FMA contraction so sums round exactly as written)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-std=c11", *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Params(ct.Structure):
    _fields_ = [
        ("thr", ct.c_double),
        ("eps_split", ct.c_double),
        ("delta", ct.c_double),
        ("split_mode", ct.c_int32),
        ("max_iter", ct.c_int32),
        ("store_fp32", ct.c_int32),
        ("fixed_iters", ct.c_int32),
        ("forced_iters", ct.POINTER(ct.c_int32)),
        ("n_forced", ct.c_int32),
        ("C_init", ct.POINTER(ct.c_double)),
        ("N_init", ct.c_int64),
        ("nthreads", ct.c_int32),
    ]


class _Trace(ct.Structure):
    _fields_ = [
        ("cap_D", ct.c_int64),
        ("n_D", ct.c_int64),
        ("D", ct.POINTER(ct.c_double)),
        ("cap_levels", ct.c_int64),
        ("n_levels", ct.c_int64),
        ("level_n", ct.POINTER(ct.c_int64)),
        ("level_iters", ct.POINTER(ct.c_int32)),
        ("level_stop_ratio", ct.POINTER(ct.c_double)),
    ]


def _p(a, t):
    return a.ctypes.data_as(ct.POINTER(t))


def load(path: str = _LIB):
    """Load the oracle library, building it when missing or older than its
    source."""
    global _lib
    with _lock:
        if _lib is not None and path == _LIB:
            return _lib
        if (not os.path.exists(path)
                or (path == _LIB and os.path.getmtime(path) < os.path.getmtime(_SRC))):
            build(out=path)
        lib = ct.CDLL(path)
        P64, PI32, PF32, PF64 = (ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32),
                                 ct.POINTER(ct.c_float), ct.POINTER(ct.c_double))
        i64 = ct.c_int64
        lib.lbg_oracle_centroid.argtypes = [PF32, i64, i64, PF64]
        lib.lbg_oracle_centroid.restype = None
        lib.lbg_oracle_split.argtypes = [PF64, i64, i64, ct.c_int32, ct.c_double,
                                         ct.c_double, ct.c_int32, PF64]
        lib.lbg_oracle_split.restype = None
        lib.lbg_oracle_assign.argtypes = [PF32, i64, i64, PF64, i64, PI32, PF64,
                                          PF64, ct.c_int32]
        lib.lbg_oracle_assign.restype = None
        lib.lbg_oracle_distortion.argtypes = [PF32, i64, i64, PF64, PI32]
        lib.lbg_oracle_distortion.restype = ct.c_double
        lib.lbg_oracle_update.argtypes = [PF32, i64, i64, PI32, PF64, i64,
                                          ct.c_int32, PF64, P64]
        lib.lbg_oracle_update.restype = None
        lib.lbg_oracle_grad.argtypes = [PF32, i64, i64, PF64, i64, PI32,
                                        ct.c_double, PF64, PF64]
        lib.lbg_oracle_grad.restype = None
        lib.lbg_oracle_train.argtypes = [PF32, i64, i64, i64, ct.POINTER(_Params),
                                         PF64, PI32, PF64, ct.POINTER(_Trace)]
        lib.lbg_oracle_train.restype = ct.c_int
        lib.lbg_oracle_max_threads.argtypes = []
        lib.lbg_oracle_max_threads.restype = ct.c_int32
        if path == _LIB:
            _lib = lib
        return lib


def _X(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be M x L")
    return X


def _C(C):
    C = np.ascontiguousarray(C, dtype=np.float64)
    if C.ndim != 2:
        raise ValueError("C must be n x L")
    return C


def max_threads(lib=None) -> int:
    return int((lib or load()).lbg_oracle_max_threads())


def centroid(X, lib=None):
    """Initial codebook: the mean of all training vectors (Algorithm 1,
    Initialization; Table 1)."""
    lib = lib or load()
    X = _X(X)
    c0 = np.empty((1, X.shape[1]), np.float64)
    lib.lbg_oracle_centroid(_p(X, ct.c_float), X.shape[0], X.shape[1],
                            _p(c0, ct.c_double))
    return c0


def split(C, eps=0.01, mode=SPLIT_MULT, delta=0.0, store_fp32=False, lib=None):
    """Codebook Splitting (Algorithm 1; Sec. 3.2): row 2i = "+" child, row
    2i+1 = "-" child of codevector i."""
    lib = lib or load()
    C = _C(C)
    n, L = C.shape
    C2 = np.empty((2 * n, L), np.float64)
    lib.lbg_oracle_split(_p(C, ct.c_double), n, L, mode, eps, delta,
                         int(store_fp32), _p(C2, ct.c_double))
    return C2


def assign(X, C, nthreads=0, lib=None):
    """Cell Allocation (Algorithm 1; Sec. 3.2): nearest codevector by squared
    Euclidean distance, lowest index on ties.  Returns (idx int32, d1, d2)
    with d1 the winning distance and d2 the smallest distance to any other
    codevector (inf when n == 1)."""
    lib = lib or load()
    X, C = _X(X), _C(C)
    M, L = X.shape
    if C.shape[1] != L:
        raise ValueError("dimension mismatch")
    idx = np.empty(M, np.int32)
    d1 = np.empty(M, np.float64)
    d2 = np.empty(M, np.float64)
    lib.lbg_oracle_assign(_p(X, ct.c_float), M, L, _p(C, ct.c_double),
                          C.shape[0], _p(idx, ct.c_int32), _p(d1, ct.c_double),
                          _p(d2, ct.c_double), int(nthreads))
    return idx, d1, d2


def distortion(X, C, idx, lib=None):
    """Average distortion D = M^-1 sum ||x_m - c_idx_m||^2 (LBG restatement,
    Sec. 2.2), index-order sum."""
    lib = lib or load()
    X, C = _X(X), _C(C)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    return float(lib.lbg_oracle_distortion(_p(X, ct.c_float), X.shape[0], X.shape[1],
                                           _p(C, ct.c_double), _p(idx, ct.c_int32)))


def update(X, idx, C_old, store_fp32=False, lib=None):
    """Codebook Updation (Algorithm 1; Sec. 3.2): per-cell means, empty cell
    keeps its codevector.  Returns (C_new, counts)."""
    lib = lib or load()
    X, C_old = _X(X), _C(C_old)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n, L = C_old.shape
    C_new = np.empty_like(C_old)
    counts = np.empty(n, np.int64)
    lib.lbg_oracle_update(_p(X, ct.c_float), X.shape[0], L, _p(idx, ct.c_int32),
                          _p(C_old, ct.c_double), n, int(store_fp32),
                          _p(C_new, ct.c_double), _p(counts, ct.c_int64))
    return C_new, counts


def grad(X, C, idx, g=1.0, lib=None):
    """Closed-form gradient of D(C, X) at allocation idx (derivative of the
    LBG average distortion of Sec. 2.2).  Returns (gX, gC)."""
    lib = lib or load()
    X, C = _X(X), _C(C)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    gX = np.empty(X.shape, np.float64)
    gC = np.empty(C.shape, np.float64)
    lib.lbg_oracle_grad(_p(X, ct.c_float), X.shape[0], X.shape[1], _p(C, ct.c_double),
                        C.shape[0], _p(idx, ct.c_int32), float(g),
                        _p(gX, ct.c_double), _p(gC, ct.c_double))
    return gX, gC


def train(X, N, thr=1e-3, eps_split=0.01, split_mode=SPLIT_MULT, delta=0.0,
          max_iter=1000, store_fp32=False, fixed_iters=0, forced_iters=None,
          C_init=None, nthreads=0, lib=None, cap_D=1 << 16):
    """LBG with splitting (Algorithm 1).  Returns a dict with C, idx, D,
    status and the trace (D per allocation, per-level size / updates /
    stopping ratio)."""
    lib = lib or load()
    X = _X(X)
    M, L = X.shape
    p = _Params()
    p.thr, p.eps_split, p.delta = float(thr), float(eps_split), float(delta)
    p.split_mode, p.max_iter = int(split_mode), int(max_iter)
    p.store_fp32, p.fixed_iters = int(store_fp32), int(fixed_iters)
    p.nthreads = int(nthreads)
    keep = []
    if forced_iters is not None:
        f = np.ascontiguousarray(forced_iters, dtype=np.int32)
        keep.append(f)
        p.forced_iters, p.n_forced = _p(f, ct.c_int32), len(f)
    if C_init is not None:
        ci = _C(C_init)
        keep.append(ci)
        p.C_init, p.N_init = _p(ci, ct.c_double), ci.shape[0]
    cap_lv = 64
    Dbuf = np.zeros(cap_D, np.float64)
    lvn = np.zeros(cap_lv, np.int64)
    lvi = np.zeros(cap_lv, np.int32)
    lvr = np.zeros(cap_lv, np.float64)
    tr = _Trace(cap_D, 0, _p(Dbuf, ct.c_double), cap_lv, 0, _p(lvn, ct.c_int64),
                _p(lvi, ct.c_int32), _p(lvr, ct.c_double))
    C = np.zeros((N, L), np.float64)
    idx = np.zeros(M, np.int32)
    D = ct.c_double(0.0)
    st = lib.lbg_oracle_train(_p(X, ct.c_float), M, L, int(N), ct.byref(p),
                              _p(C, ct.c_double), _p(idx, ct.c_int32), ct.byref(D),
                              ct.byref(tr))
    if st == EINVAL:
        raise ValueError("oracle rejected the arguments")
    nD, nl = min(tr.n_D, cap_D), min(tr.n_levels, cap_lv)
    return dict(C=C, idx=idx, D=D.value, status=int(st), D_trace=Dbuf[:nD].copy(),
                level_n=lvn[:nl].copy(), level_iters=lvi[:nl].copy(),
                level_stop_ratio=lvr[:nl].copy())
