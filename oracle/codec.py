"""Encoder/decoder half of vector quantization, plain NumPy -- TEST
INFRASTRUCTURE ONLY (like the rest of ``oracle``: only the tests, the smoke
check and the CPU-baseline leg of the benchmark use it).

The paper (Introduction) splits VQ compression into codebook design and the
replacement of data by the codebook: the encoder sends, for each input
vector, the index of its nearest codevector (log2 N bits), the decoder puts
that codevector in its place, so the rate is log2(N)/L bits per sample.  The
nearest-codevector search is ``oracle.assign``; this module holds the rest,
written as the definitions, with loops over blocks where a picture is
involved:

* ``decode``        -- row m of the reconstruction is codevector idx[m];
                       an index outside [0, N) is a row of NaNs (the GPU
                       library's convention for a corrupt code);
* ``image_blocks``  -- a picture cut into b x b blocks in raster order,
                       pixels row-major inside a block (the training vectors
                       of an image coder);
* ``decode_image``  -- every block of every picture replaced by its
                       codevector, laid back out as b x b pixels;
* ``rate``          -- log2(N) / L bits per sample (Introduction);
* ``psnr``          -- peak signal-to-noise ratio.  The paper names no
                       quality figure; this is the usual image-coding one,
                       10 log10(peak^2 / MSE) dB with the MSE taken per
                       sample in FP64 (reading stated with the design notes).
"""

from __future__ import annotations

import math

import numpy as np


def decode(C, idx):
    """Reconstruction Y (M x L, FP64): Y[m] = C[idx[m]]; NaN rows for
    indices outside [0, N)."""
    C = np.asarray(C, dtype=np.float64)
    idx = np.asarray(idx).astype(np.int64)
    N, L = C.shape
    Y = np.full((idx.shape[0], L), np.nan)
    for m, k in enumerate(idx):
        if 0 <= k < N:
            Y[m] = C[k]
    return Y


def image_blocks(imgs, b):
    """Block vectors of pictures ``imgs`` (nimg x H x W): vector
    (p (H/b) + by) (W/b) + bx is block (by, bx) of picture p, row-major."""
    imgs = np.asarray(imgs)
    nimg, H, W = imgs.shape
    if H % b or W % b:
        raise ValueError("picture size must be a multiple of b")
    nby, nbx = H // b, W // b
    X = np.empty((nimg * nby * nbx, b * b), dtype=imgs.dtype)
    v = 0
    for p in range(nimg):
        for by in range(nby):
            for bx in range(nbx):
                blk = imgs[p, by * b:(by + 1) * b, bx * b:(bx + 1) * b]
                for dy in range(b):
                    X[v, dy * b:(dy + 1) * b] = blk[dy]
                v += 1
    return X


def decode_image(C, idx, nimg, H, W, b):
    """Pictures (nimg x H x W, FP64) whose block v is codevector idx[v]
    reshaped to b x b (row-major); NaN blocks for indices outside [0, N)."""
    C = np.asarray(C, dtype=np.float64)
    idx = np.asarray(idx).astype(np.int64)
    N, L = C.shape
    if L != b * b:
        raise ValueError("codevectors must have b * b dimensions")
    nby, nbx = H // b, W // b
    if idx.shape[0] != nimg * nby * nbx:
        raise ValueError("one index per block expected")
    out = np.empty((nimg, H, W))
    v = 0
    for p in range(nimg):
        for by in range(nby):
            for bx in range(nbx):
                k = idx[v]
                blk = C[k].reshape(b, b) if 0 <= k < N else np.full((b, b), np.nan)
                out[p, by * b:(by + 1) * b, bx * b:(bx + 1) * b] = blk
                v += 1
    return out


def rate(N, L):
    """Bits per sample of an L-dimensional quantizer with N codevectors:
    log2(N) per vector, shared by its L samples (Introduction)."""
    if N < 1 or L < 1:
        raise ValueError("N and L must be positive")
    return math.log2(N) / L


def psnr(ref, rec, peak=255.0):
    """10 log10(peak^2 / MSE) in dB, MSE the FP64 mean over all samples of
    (ref - rec)^2; +inf for a perfect reconstruction."""
    ref = np.asarray(ref, dtype=np.float64)
    rec = np.asarray(rec, dtype=np.float64)
    if ref.shape != rec.shape:
        raise ValueError("shapes differ")
    mse = float(np.mean((ref - rec) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(peak * peak / mse)
