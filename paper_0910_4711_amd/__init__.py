"""MI355X (gfx950) LBG codebook design -- thin Python binding of liblbg.so.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The
library must have been built (``python -m paper_0910_4711_amd.build``); there
is no fallback of any kind.

Functions follow Algorithm 1 of Annaji & Rao, "Parallelization of the LBG
Vector Quantization Algorithm for Shared Memory Systems":
``centroid`` (Initialization), ``split`` (Codebook Splitting), ``assign``
(Cell Allocation), ``distortion`` (IntegrateDistortions), ``update``
(Codebook Updation), ``train`` (the whole algorithm), plus the distortion's
gradient and ``Distortion`` (a torch.autograd.Function).
"""

from __future__ import annotations

import ctypes as ct
import os
import threading

import torch

__all__ = [
    "FP32", "BF16_RESCORE", "SPLIT_MULT", "SPLIT_ADD", "LBGError",
    "library_path", "load", "centroid", "split", "assign", "update",
    "distortion", "distortion_backward", "train", "Distortion",
    "encode", "decode", "image_blocks", "decode_image", "rate", "psnr", "assign_distortion",
]

FP32 = 0
BF16_RESCORE = 1
SPLIT_MULT = 0
SPLIT_ADD = 1
OK, EINVAL, ENOWS, EHIP, WMAXITER = 0, -1, -2, -3, 1
OP_ASSIGN, OP_UPDATE, OP_DISTORTION, OP_TRAIN, OP_BACKWARD, OP_CENTROID = 1, 2, 3, 4, 5, 6

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbg.so")
_lock = threading.Lock()
_lib = None


class LBGError(RuntimeError):
    """A library call returned an error code."""


class Params(ct.Structure):
    _fields_ = [
        ("thr", ct.c_double),
        ("eps_split", ct.c_double),
        ("delta", ct.c_double),
        ("split_mode", ct.c_int32),
        ("max_iter", ct.c_int32),
        ("precision", ct.c_int32),
        ("fixed_iters", ct.c_int32),
        ("forced_iters", ct.POINTER(ct.c_int32)),
        ("n_forced", ct.c_int32),
        ("C_init", ct.c_void_p),
        ("N_init", ct.c_int64),
        ("timing", ct.c_int32),
        ("graph", ct.c_int32),
        ("D_prev_init", ct.c_double),
        ("it_init", ct.c_int32),
        ("stats_ties", ct.c_int32),
    ]


class Stats(ct.Structure):
    _fields_ = [
        ("n_levels", ct.c_int32),
        ("level_n", ct.c_int32 * 32),
        ("level_iters", ct.c_int32 * 32),
        ("total_updates", ct.c_int32),
        ("total_assigns", ct.c_int32),
        ("total_distances", ct.c_int64),
        ("fallback_rows", ct.c_int64),
        ("D_trace", ct.POINTER(ct.c_double)),
        ("D_cap", ct.c_int32),
        ("n_D", ct.c_int32),
        ("ms_assign", ct.c_double),
        ("ms_update", ct.c_double),
        ("ms_split", ct.c_double),
        ("empty_cells", ct.c_int32),
        ("near_tie_rows", ct.c_int64),
    ]


class Instance(ct.Structure):
    _fields_ = [
        ("X", ct.c_void_p),
        ("M", ct.c_int64),
        ("L", ct.c_int64),
        ("N", ct.c_int64),
        ("C_out", ct.c_void_p),
        ("idx_out", ct.c_void_p),
    ]


class AssignItem(ct.Structure):
    _fields_ = [
        ("X", ct.c_void_p),
        ("M", ct.c_int64),
        ("L", ct.c_int64),
        ("C", ct.c_void_p),
        ("N", ct.c_int64),
        ("idx", ct.c_void_p),
        ("D", ct.c_void_p),
    ]


class UpdateItem(ct.Structure):
    _fields_ = [
        ("X", ct.c_void_p),
        ("M", ct.c_int64),
        ("L", ct.c_int64),
        ("idx", ct.c_void_p),
        ("C_old", ct.c_void_p),
        ("N", ct.c_int64),
        ("C_new", ct.c_void_p),
        ("counts", ct.c_void_p),
    ]


class BatchConfig(ct.Structure):
    _fields_ = [
        ("grab", ct.c_int32),
        ("grid", ct.c_int32),
        ("graph", ct.c_int32),
        ("rounds_per_poll", ct.c_int32),
        ("timing", ct.c_int32),
        ("screen", ct.c_int32),
    ]


class BatchResult(ct.Structure):
    _fields_ = [
        ("D", ct.c_double),
        ("status", ct.c_int32),
        ("n_levels", ct.c_int32),
        ("n_assign", ct.c_int32),
        ("n_update", ct.c_int32),
        ("fallback_rows", ct.c_int64),
        ("distances", ct.c_int64),
    ]


class BatchStats(ct.Structure):
    _fields_ = [
        ("rounds", ct.c_int32),
        ("grab", ct.c_int32),
        ("grid", ct.c_int32),
        ("graph", ct.c_int32),
        ("tuned", ct.c_int32),
        ("total_distances", ct.c_int64),
        ("ms_tune", ct.c_double),
        ("ms_assign", ct.c_double),
        ("ms_update", ct.c_double),
        ("screen", ct.c_int32),
    ]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load liblbg.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise LBGError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_0910_4711_amd.build`")
        lib = ct.CDLL(_LIB_PATH)
        i64, i32, vp, dbl, sz = ct.c_int64, ct.c_int, ct.c_void_p, ct.c_double, ct.c_size_t
        sig = {
            "lbg_split": [vp, i64, i64, dbl, vp, vp],
            "lbg_split_add": [vp, i64, i64, dbl, vp, vp],
            "lbg_centroid": [vp, i64, i64, vp, vp, sz, vp],
            "lbg_assign": [vp, i64, i64, vp, i64, vp, vp, i32, vp, sz, vp],
            "lbg_update": [vp, i64, i64, vp, vp, i64, vp, vp, vp, sz, vp],
            "lbg_distortion": [vp, i64, i64, vp, i64, vp, vp, vp, sz, vp],
            "lbg_distortion_backward": [vp, i64, i64, vp, i64, vp, dbl, vp, vp, vp, sz, vp],
            "lbg_encode": [vp, i64, i64, vp, i64, vp, vp, sz, vp],
            "lbg_assign_distortion": [vp, i64, i64, vp, i64, vp, vp, i32, vp, vp, sz, vp],
            "lbg_assign_distortion_noalloc": [vp, i64, i64, vp, i64, vp, vp, i32, vp, vp],
            "lbg_decode": [vp, i64, vp, i64, i64, vp, vp],
            "lbg_image_blocks": [vp, i64, i64, i64, i64, vp, vp],
            "lbg_decode_image": [vp, vp, i64, i64, i64, i64, i64, vp, vp],
            "lbg_rate": [i64, i64, ct.POINTER(ct.c_double)],
            "lbg_psnr": [dbl, i64, dbl, ct.POINTER(ct.c_double)],
            "lbg_train": [vp, i64, i64, i64, ct.POINTER(Params), vp, vp,
                          ct.POINTER(ct.c_double), ct.POINTER(Stats), vp, sz, vp],
            "lbg_train_batched": [ct.POINTER(Instance), i32, ct.POINTER(Params),
                                  ct.POINTER(BatchConfig), ct.POINTER(BatchResult),
                                  ct.POINTER(BatchStats), vp, sz, vp],
            "lbg_assign_batched": [ct.POINTER(AssignItem), i32, vp, sz, vp],
            "lbg_update_batched": [ct.POINTER(UpdateItem), i32, vp, sz, vp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ct.c_int
        lib.lbg_noalloc_scratch_bytes.argtypes = []
        lib.lbg_noalloc_scratch_bytes.restype = ct.c_size_t
        lib.lbg_workspace_size.argtypes = [ct.c_int, i64, i64, i64, ct.c_int]
        lib.lbg_workspace_size.restype = ct.c_size_t
        lib.lbg_last_error.argtypes = []
        lib.lbg_last_error.restype = ct.c_char_p
        lib.lbg_version.argtypes = []
        lib.lbg_version.restype = ct.c_char_p
        lib.lbg_params_default.argtypes = [ct.POINTER(Params)]
        lib.lbg_params_default.restype = None
        lib.lbg_batch_config_default.argtypes = [ct.POINTER(BatchConfig)]
        lib.lbg_batch_config_default.restype = None
        lib.lbg_train_batched_workspace.argtypes = [ct.POINTER(Instance), i32]
        lib.lbg_train_batched_workspace.restype = ct.c_size_t
        lib.lbg_assign_batched_workspace.argtypes = [ct.POINTER(AssignItem), i32]
        lib.lbg_assign_batched_workspace.restype = ct.c_size_t
        lib.lbg_update_batched_workspace.argtypes = [ct.POINTER(UpdateItem), i32]
        lib.lbg_update_batched_workspace.restype = ct.c_size_t
        _lib = lib
        return lib


def _check(rc: int, what: str) -> int:
    if rc < 0:
        msg = load().lbg_last_error().decode(errors="replace")
        raise LBGError(f"{what} failed ({rc}): {msg}")
    return rc


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f32_2d(name, t):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float32 tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _i32_1d(name, t, n):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or t.dim() != 1 or t.numel() != n:
        raise TypeError(f"{name} must be a 1-D int32 tensor of {n} entries")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous GPU tensor")
    return t


def _ws(op, M, L, N, precision, device):
    nb = load().lbg_workspace_size(op, M, L, N, precision)
    if nb == 0:
        return None, 0
    return torch.empty(nb, dtype=torch.uint8, device=device), nb


def _prec(p):
    if p in (FP32, "fp32", "f32"):
        return FP32
    if p in (BF16_RESCORE, "bf16", "bf16_rescore"):
        return BF16_RESCORE
    raise ValueError(f"unknown precision {p!r}")


def centroid(X):
    """Initial codebook: mean of the rows of X (1 x L, FP32)."""
    X = _f32_2d("X", X)
    M, L = X.shape
    c0 = torch.empty((1, L), dtype=torch.float32, device=X.device)
    ws, nb = _ws(OP_CENTROID, M, L, 1, FP32, X.device)
    _check(load().lbg_centroid(_ptr(X), M, L, _ptr(c0), _ptr(ws), nb, _stream(X.device)),
           "lbg_centroid")
    return c0


def split(C, eps=0.01, mode=SPLIT_MULT, delta=0.0):
    """Codebook Splitting: (2n x L) children, row 2i = '+', 2i+1 = '-'."""
    C = _f32_2d("C", C)
    n, L = C.shape
    C2 = torch.empty((2 * n, L), dtype=torch.float32, device=C.device)
    lib = load()
    if mode == SPLIT_ADD:
        rc = lib.lbg_split_add(_ptr(C), n, L, float(delta), _ptr(C2), _stream(C.device))
    else:
        rc = lib.lbg_split(_ptr(C), n, L, float(eps), _ptr(C2), _stream(C.device))
    _check(rc, "lbg_split")
    return C2


def assign(X, C, precision=FP32, with_mind=True):
    """Cell Allocation: (idx int32 [M], mind float32 [M] or None)."""
    X, C = _f32_2d("X", X), _f32_2d("C", C)
    M, L = X.shape
    N = C.shape[0]
    if C.shape[1] != L:
        raise ValueError("X and C differ in dimension")
    if C.device != X.device:
        raise ValueError("X and C are on different devices")
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    mind = torch.empty(M, dtype=torch.float32, device=X.device) if with_mind else None
    ws, nb = _ws(OP_ASSIGN, M, L, N, _prec(precision), X.device)
    _check(load().lbg_assign(_ptr(X), M, L, _ptr(C), N, _ptr(idx), _ptr(mind),
                             _prec(precision), _ptr(ws), nb, _stream(X.device)),
           "lbg_assign")
    return idx, mind


def assign_distortion(X, C, precision=FP32, with_mind=False):
    """Cell Allocation and its average distortion in one pass:
    (idx int32 [M], mind float32 [M] or None, D 0-d float64 GPU tensor)."""
    X, C = _f32_2d("X", X), _f32_2d("C", C)
    M, L = X.shape
    N = C.shape[0]
    if C.shape[1] != L:
        raise ValueError("X and C differ in dimension")
    if C.device != X.device:
        raise ValueError("X and C are on different devices")
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    mind = torch.empty(M, dtype=torch.float32, device=X.device) if with_mind else None
    D = torch.empty((), dtype=torch.float64, device=X.device)
    ws, nb = _ws(OP_ASSIGN, M, L, N, _prec(precision), X.device)
    _check(load().lbg_assign_distortion(_ptr(X), M, L, _ptr(C), N, _ptr(idx), _ptr(mind),
                                        _prec(precision), _ptr(D), _ptr(ws), nb,
                                        _stream(X.device)), "lbg_assign_distortion")
    return idx, mind, D


def assign_distortion_noalloc(X, C, precision=FP32, with_mind=False):
    """assign_distortion through the entry point that takes no workspace (its
    scratch is the library's fixed per-GPU array): (idx, mind or None, D)."""
    X, C = _f32_2d("X", X), _f32_2d("C", C)
    M, L = X.shape
    N = C.shape[0]
    if C.shape[1] != L or C.device != X.device:
        raise ValueError("X and C differ in dimension or device")
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    mind = torch.empty(M, dtype=torch.float32, device=X.device) if with_mind else None
    D = torch.empty((), dtype=torch.float64, device=X.device)
    _check(load().lbg_assign_distortion_noalloc(_ptr(X), M, L, _ptr(C), N, _ptr(idx),
                                                _ptr(mind), _prec(precision), _ptr(D),
                                                _stream(X.device)),
           "lbg_assign_distortion_noalloc")
    return idx, mind, D


def update(X, idx, C_old, out=None):
    """Codebook Updation: (C_new [N x L] float32, counts [N] int32)."""
    X, C_old = _f32_2d("X", X), _f32_2d("C_old", C_old)
    M, L = X.shape
    N = C_old.shape[0]
    if C_old.shape[1] != L:
        raise ValueError("X and C differ in dimension")
    idx = _i32_1d("idx", idx, M)
    C_new = out if out is not None else torch.empty_like(C_old)
    _f32_2d("out", C_new)
    counts = torch.empty(N, dtype=torch.int32, device=X.device)
    ws, nb = _ws(OP_UPDATE, M, L, N, FP32, X.device)
    _check(load().lbg_update(_ptr(X), M, L, _ptr(idx), _ptr(C_old), N, _ptr(C_new),
                             _ptr(counts), _ptr(ws), nb, _stream(X.device)), "lbg_update")
    return C_new, counts


def distortion(X, C, idx):
    """Average distortion of allocation idx: 0-d float64 GPU tensor."""
    X, C = _f32_2d("X", X), _f32_2d("C", C)
    M, L = X.shape
    N = C.shape[0]
    idx = _i32_1d("idx", idx, M)
    D = torch.empty((), dtype=torch.float64, device=X.device)
    ws, nb = _ws(OP_DISTORTION, M, L, N, FP32, X.device)
    _check(load().lbg_distortion(_ptr(X), M, L, _ptr(C), N, _ptr(idx), _ptr(D), _ptr(ws),
                                 nb, _stream(X.device)), "lbg_distortion")
    return D


def encode(X, C):
    """Encoder: index of the nearest codevector of every row of X (int32 [M])."""
    X, C = _f32_2d("X", X), _f32_2d("C", C)
    M, L = X.shape
    N = C.shape[0]
    if C.shape[1] != L:
        raise ValueError("X and C differ in dimension")
    if C.device != X.device:
        raise ValueError("X and C are on different devices")
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    ws, nb = _ws(OP_ASSIGN, M, L, N, FP32, X.device)
    _check(load().lbg_encode(_ptr(X), M, L, _ptr(C), N, _ptr(idx), _ptr(ws), nb,
                             _stream(X.device)), "lbg_encode")
    return idx


def decode(idx, C):
    """Decoder: Y [M x L] with Y[m] = C[idx[m]] (NaN rows for indices outside
    [0, N))."""
    C = _f32_2d("C", C)
    N, L = C.shape
    if not isinstance(idx, torch.Tensor) or idx.dim() != 1:
        raise TypeError("idx must be a 1-D int32 tensor")
    M = idx.numel()
    idx = _i32_1d("idx", idx, M)
    Y = torch.empty((M, L), dtype=torch.float32, device=C.device)
    _check(load().lbg_decode(_ptr(idx), M, _ptr(C), N, L, _ptr(Y), _stream(C.device)),
           "lbg_decode")
    return Y


def _pictures(name, t):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 3:
        raise TypeError(f"{name} must be a 3-D float32 tensor (pictures x rows x columns)")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous GPU tensor")
    return t


def image_blocks(img, b):
    """Training vectors of pictures img (nimg x H x W): b x b blocks in raster
    order, pixels row-major inside a block ([nimg (H/b)(W/b)] x b*b)."""
    img = _pictures("img", img)
    nimg, H, W = img.shape
    if b < 1 or H % b or W % b:
        raise ValueError("picture size must be a multiple of b")
    X = torch.empty((nimg * (H // b) * (W // b), b * b), dtype=torch.float32, device=img.device)
    _check(load().lbg_image_blocks(_ptr(img), nimg, H, W, b, _ptr(X), _stream(img.device)),
           "lbg_image_blocks")
    return X


def decode_image(idx, C, nimg, H, W, b):
    """Decoder into pictures: block v of the output (the layout of
    image_blocks) is codevector idx[v] as b x b pixels."""
    C = _f32_2d("C", C)
    N, L = C.shape
    if L != b * b:
        raise ValueError("codevectors must have b * b dimensions")
    if b < 1 or H % b or W % b:
        raise ValueError("picture size must be a multiple of b")
    idx = _i32_1d("idx", idx, nimg * (H // b) * (W // b))
    img = torch.empty((nimg, H, W), dtype=torch.float32, device=C.device)
    _check(load().lbg_decode_image(_ptr(idx), _ptr(C), N, nimg, H, W, b, _ptr(img),
                                   _stream(C.device)), "lbg_decode_image")
    return img


def rate(N, L):
    """Bits per sample, log2(N) / L."""
    out = ct.c_double()
    _check(load().lbg_rate(int(N), int(L), ct.byref(out)), "lbg_rate")
    return out.value


def psnr(D, L, peak=255.0):
    """PSNR in dB of a reconstruction with average distortion D (a float or
    a 0-d tensor, as from distortion()) over L-dimensional vectors."""
    if isinstance(D, torch.Tensor):
        D = float(D.item())
    out = ct.c_double()
    _check(load().lbg_psnr(float(D), int(L), float(peak), ct.byref(out)), "lbg_psnr")
    return out.value


def distortion_backward(X, C, idx, g=1.0, need_x=True, need_c=True):
    """Gradient of D at allocation idx scaled by g: (gX or None, gC or None)."""
    X, C = _f32_2d("X", X), _f32_2d("C", C)
    M, L = X.shape
    N = C.shape[0]
    idx = _i32_1d("idx", idx, M)
    gX = torch.empty_like(X) if need_x else None
    gC = torch.empty_like(C) if need_c else None
    ws, nb = _ws(OP_BACKWARD, M, L, N, FP32, X.device)
    _check(load().lbg_distortion_backward(_ptr(X), M, L, _ptr(C), N, _ptr(idx), float(g),
                                          _ptr(gX), _ptr(gC), _ptr(ws), nb,
                                          _stream(X.device)), "lbg_distortion_backward")
    return gX, gC


def train(X, N, thr=1e-3, eps_split=0.01, split_mode=SPLIT_MULT, delta=0.0,
          max_iter=1000, precision=FP32, fixed_iters=0, forced_iters=None,
          C_init=None, D_cap=4096, workspace=None, timing=False, graph=False,
          D_prev_init=None, it_init=0, stats_ties=False):
    """LBG with splitting (Algorithm 1).  Returns (C, idx, D, stats) with C
    [N x L] float32, idx [M] int32, D a Python float and stats a dict.
    D_prev_init / it_init resume a level in its middle (with C_init)."""
    X = _f32_2d("X", X)
    M, L = X.shape
    lib = load()
    p = Params()
    lib.lbg_params_default(ct.byref(p))
    p.thr, p.eps_split, p.delta = float(thr), float(eps_split), float(delta)
    p.split_mode, p.max_iter = int(split_mode), int(max_iter)
    p.precision, p.fixed_iters = _prec(precision), int(fixed_iters)
    p.timing = 1 if timing else 0
    p.graph = 1 if graph else 0
    if D_prev_init is not None:
        p.D_prev_init = float(D_prev_init)
    p.it_init = int(it_init)
    p.stats_ties = 1 if stats_ties else 0
    keep = []
    if forced_iters is not None:
        f = (ct.c_int32 * len(forced_iters))(*[int(v) for v in forced_iters])
        keep.append(f)
        p.forced_iters = ct.cast(f, ct.POINTER(ct.c_int32))
        p.n_forced = len(forced_iters)
    if C_init is not None:
        C_init = _f32_2d("C_init", C_init)
        if C_init.shape[1] != L:
            raise ValueError("C_init has the wrong dimension")
        p.C_init, p.N_init = C_init.data_ptr(), C_init.shape[0]
    C = torch.empty((N, L), dtype=torch.float32, device=X.device)
    idx = torch.empty(M, dtype=torch.int32, device=X.device)
    Dbuf = (ct.c_double * max(1, D_cap))()
    st = Stats()
    st.D_trace = ct.cast(Dbuf, ct.POINTER(ct.c_double))
    st.D_cap = D_cap
    nb = lib.lbg_workspace_size(OP_TRAIN, M, L, N, p.precision)
    ws = workspace
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    D = ct.c_double(0.0)
    rc = lib.lbg_train(_ptr(X), M, L, int(N), ct.byref(p), _ptr(C), _ptr(idx), ct.byref(D),
                       ct.byref(st), _ptr(ws), nb, _stream(X.device))
    _check(rc, "lbg_train")
    nl = st.n_levels
    stats = dict(
        status=rc,
        level_n=list(st.level_n[:nl]),
        level_iters=list(st.level_iters[:nl]),
        total_updates=st.total_updates,
        total_assigns=st.total_assigns,
        total_distances=st.total_distances,
        fallback_rows=st.fallback_rows,
        D_trace=[Dbuf[i] for i in range(min(st.n_D, D_cap))],
        ms_assign=st.ms_assign,
        ms_update=st.ms_update,
        ms_split=st.ms_split,
        empty_cells=st.empty_cells,
        near_tie_rows=st.near_tie_rows,
    )
    return C, idx, D.value, stats


def train_batched(Xs, Ns, thr=1e-3, eps_split=0.01, split_mode=SPLIT_MULT, delta=0.0,
                  max_iter=1000, fixed_iters=0, grab=0, grid=0, graph=True,
                  rounds_per_poll=8, workspace=None, timing=False, screen=0):
    """Independent LBG runs (Algorithm 1 on every instance) advanced together
    by the batched kernels.  Xs: list of [M_i x L_i] float32 device tensors,
    Ns: list of powers of two.  Returns (results, stats): results[i] =
    (C_i, idx_i, D_i, info_i), each bit-identical to train(Xs[i], Ns[i]).
    timing: direct launches with events around every round's allocation and
    update (stats ms_assign, ms_update).  screen: 0 autotuned, 1 FP32, 2
    split BF16 where it fits (the same results either way)."""
    if len(Xs) != len(Ns) or len(Xs) == 0:
        raise ValueError("need as many codebook sizes as training sets (at least one)")
    Xs = [_f32_2d(f"Xs[{i}]", X) for i, X in enumerate(Xs)]
    dev = Xs[0].device
    if any(X.device != dev for X in Xs):
        raise ValueError("all training sets must be on one device")
    lib = load()
    n = len(Xs)
    inst = (Instance * n)()
    outs = []
    for i, (X, N) in enumerate(zip(Xs, Ns)):
        M, L = X.shape
        C = torch.empty((int(N), L), dtype=torch.float32, device=dev)
        idx = torch.empty(M, dtype=torch.int32, device=dev)
        inst[i].X, inst[i].M, inst[i].L, inst[i].N = X.data_ptr(), M, L, int(N)
        inst[i].C_out, inst[i].idx_out = C.data_ptr(), idx.data_ptr()
        outs.append((C, idx))
    p = Params()
    lib.lbg_params_default(ct.byref(p))
    p.thr, p.eps_split, p.delta = float(thr), float(eps_split), float(delta)
    p.split_mode, p.max_iter, p.fixed_iters = int(split_mode), int(max_iter), int(fixed_iters)
    cfg = BatchConfig()
    lib.lbg_batch_config_default(ct.byref(cfg))
    cfg.grab, cfg.grid, cfg.graph = int(grab), int(grid), 1 if graph else 0
    cfg.rounds_per_poll = int(rounds_per_poll)
    cfg.timing = 1 if timing else 0
    cfg.screen = int(screen)
    nb = lib.lbg_train_batched_workspace(inst, n)
    if nb == 0:
        raise LBGError("lbg_train_batched_workspace: bad instances")
    ws = workspace
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    res = (BatchResult * n)()
    st = BatchStats()
    rc = lib.lbg_train_batched(inst, n, ct.byref(p), ct.byref(cfg), res, ct.byref(st), _ptr(ws),
                               nb, _stream(dev))
    # an instance stopped on non-finite data reports it in its own status;
    # the other instances' results are valid
    if not (rc == EINVAL and any(res[i].status == EINVAL for i in range(n))):
        _check(rc, "lbg_train_batched")
    results = []
    for i, (C, idx) in enumerate(outs):
        r = res[i]
        results.append((C, idx, r.D, dict(status=r.status, n_levels=r.n_levels,
                                          n_assign=r.n_assign, n_update=r.n_update,
                                          fallback_rows=r.fallback_rows,
                                          distances=r.distances)))
    stats = dict(status=rc, rounds=st.rounds, grab=st.grab, grid=st.grid, graph=st.graph,
                 tuned=st.tuned, total_distances=st.total_distances, ms_tune=st.ms_tune,
                 ms_assign=st.ms_assign, ms_update=st.ms_update, screen=st.screen)
    return results, stats


class Distortion(torch.autograd.Function):
    """D(X, C) = mean_m min_k ||x_m - c_k||^2 with the library's forward
    (exact FP32-mode allocation + FP64 distortion) and hand-written backward
    kernels (dD/dX, dD/dC)."""

    @staticmethod
    def forward(ctx, X, C):
        idx, _, D = assign_distortion(X, C, FP32)
        ctx.save_for_backward(X, C, idx)
        return D

    @staticmethod
    def backward(ctx, g):
        X, C, idx = ctx.saved_tensors
        gv = float(g.item())
        gX, gC = distortion_backward(X, C, idx, gv, need_x=ctx.needs_input_grad[0],
                                     need_c=ctx.needs_input_grad[1])
        return gX, gC


def assign_batched(Xs, Cs, with_D=True, workspace=None):
    """Cell Allocation of many independent (X_i, C_i) pairs in one persistent
    launch (exact, as assign(X_i, C_i, FP32)).  Returns (idxs, Ds): idxs[i]
    int32 [M_i]; Ds[i] a 0-d float64 GPU tensor (assign_distortion's D) or
    None when with_D is false."""
    if len(Xs) != len(Cs) or len(Xs) == 0:
        raise ValueError("need as many codebooks as training sets (at least one)")
    Xs = [_f32_2d(f"Xs[{i}]", X) for i, X in enumerate(Xs)]
    Cs = [_f32_2d(f"Cs[{i}]", C) for i, C in enumerate(Cs)]
    dev = Xs[0].device
    if any(t.device != dev for t in Xs + Cs):
        raise ValueError("all tensors must be on one device")
    n = len(Xs)
    items = (AssignItem * n)()
    idxs, Ds = [], []
    for i, (X, C) in enumerate(zip(Xs, Cs)):
        M, L = X.shape
        if C.shape[1] != L:
            raise ValueError(f"Cs[{i}] has {C.shape[1]} columns, Xs[{i}] {L}")
        idx = torch.empty(M, dtype=torch.int32, device=dev)
        D = torch.empty((), dtype=torch.float64, device=dev) if with_D else None
        items[i].X, items[i].M, items[i].L = X.data_ptr(), M, L
        items[i].C, items[i].N = C.data_ptr(), C.shape[0]
        items[i].idx = idx.data_ptr()
        items[i].D = D.data_ptr() if with_D else None
        idxs.append(idx)
        Ds.append(D)
    lib = load()
    nb = lib.lbg_assign_batched_workspace(items, n)
    if nb == 0:
        raise LBGError("lbg_assign_batched_workspace: bad items")
    ws = workspace
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib.lbg_assign_batched(items, n, _ptr(ws), nb, _stream(dev)), "lbg_assign_batched")
    return idxs, Ds


def update_batched(Xs, idxs, Cs_old, workspace=None):
    """Codebook Updation of many independent items in a few launches (exact,
    as update(X_i, idx_i, C_i)).  Returns (C_news, counts)."""
    if not (len(Xs) == len(idxs) == len(Cs_old)) or len(Xs) == 0:
        raise ValueError("need as many allocations and codebooks as training sets")
    Xs = [_f32_2d(f"Xs[{i}]", X) for i, X in enumerate(Xs)]
    Cs_old = [_f32_2d(f"Cs_old[{i}]", C) for i, C in enumerate(Cs_old)]
    dev = Xs[0].device
    n = len(Xs)
    items = (UpdateItem * n)()
    outs, cnts, keep = [], [], []
    for i, (X, idx, C) in enumerate(zip(Xs, idxs, Cs_old)):
        M, L = X.shape
        if idx.dtype != torch.int32 or idx.numel() != M or not idx.is_contiguous():
            raise ValueError(f"idxs[{i}] must be a contiguous int32 tensor of {M} entries")
        if C.shape[1] != L or any(t.device != dev for t in (idx, C)):
            raise ValueError(f"item {i}: codebook columns or device differ from Xs[{i}]")
        Cn = torch.empty_like(C)
        cnt = torch.empty(C.shape[0], dtype=torch.int32, device=dev)
        items[i].X, items[i].M, items[i].L = X.data_ptr(), M, L
        items[i].idx, items[i].C_old, items[i].N = idx.data_ptr(), C.data_ptr(), C.shape[0]
        items[i].C_new, items[i].counts = Cn.data_ptr(), cnt.data_ptr()
        outs.append(Cn)
        cnts.append(cnt)
        keep.append(idx)
    lib = load()
    nb = lib.lbg_update_batched_workspace(items, n)
    if nb == 0:
        raise LBGError("lbg_update_batched_workspace: bad items")
    ws = workspace
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib.lbg_update_batched(items, n, _ptr(ws), nb, _stream(dev)), "lbg_update_batched")
    return outs, cnts
