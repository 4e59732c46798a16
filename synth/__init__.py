"""Seeded synthetic inputs for LBG codebook design.

This module only draws numbers and lays them out; it holds none of the
method's arithmetic (no distances, no means, no splitting).  The same arrays
feed the FP64 CPU oracle and the GPU library, so the two sides see identical
inputs.

The paper trains on "any numerical data ... obtained by processing an image or
a speech signal" (Sec. 3.1) and reports an experiment on 2000 training vectors
of dimension 2..10 (Sec. 5) whose data is not published.  The generators below
stand in for that data:

* ``image``       -- a grey-scale picture made of Gaussian blobs plus noise,
                     uint8, the kind of source an image VQ codes;
* ``blocks``      -- non-overlapping b x b blocks of an image, one training
                     vector per block (the M x k training matrix of Sec. 3.1);
* ``gmm``         -- an isotropic Gaussian mixture (independent LBG instances);
* ``gmm_diag``    -- a mixture with per-component diagonal sigma;
* ``distinct_rows`` -- a seeded choice of distinct rows (codebook seeds).

Recipes (all FP64 on the host, NumPy ``default_rng``):

image(seed, W, H):
    for each of 32 blobs, in this order: cx ~ U[0, W), cy ~ U[0, H),
    a ~ U[40, 200], sigma ~ U[8, 48] pixels; the blob adds
    a * exp(-(col-cx)^2 / (2 sigma^2)) * exp(-(row-cy)^2 / (2 sigma^2))
    at integer pixel coordinates; then N(0, 6^2) noise is added per pixel,
    the picture is clipped to [0, 255], rounded half-to-even and cast to uint8.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "image",
    "blocks",
    "image_training_set",
    "gmm",
    "gmm_diag",
    "distinct_rows",
    "batched_instances",
    "CONFIG0",
    "CONFIG1",
    "CONFIG2",
]

N_BLOBS = 32

# Named workloads.  Sizes are those of the image/block recipes above.
CONFIG0 = dict(name="img256x256_b4_M4096_L16_N64", seeds=(0,), W=256, H=256,
               b=4, N=64)
CONFIG1 = dict(name="img16x512x512_b4_M262144_L16_N256", seeds=tuple(range(16)),
               W=512, H=512, b=4, N=256)
CONFIG2 = dict(name="img256x1024x1024_b8_M4194304_L64_N1024",
               seeds=tuple(range(256)), W=1024, H=1024, b=8, N=1024)


def image(seed: int, W: int, H: int) -> np.ndarray:
    """Synthetic uint8 picture (H rows x W columns) from ``seed``."""
    rng = np.random.default_rng(seed)
    img = np.zeros((H, W), dtype=np.float64)
    cols = np.arange(W, dtype=np.float64)
    rows = np.arange(H, dtype=np.float64)
    for _ in range(N_BLOBS):
        cx = rng.uniform(0.0, W)
        cy = rng.uniform(0.0, H)
        a = rng.uniform(40.0, 200.0)
        s = rng.uniform(8.0, 48.0)
        gx = np.exp(-((cols - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((rows - cy) ** 2) / (2.0 * s * s))
        img += a * np.outer(gy, gx)
    img += rng.normal(0.0, 6.0, size=(H, W))
    np.clip(img, 0.0, 255.0, out=img)
    return np.rint(img).astype(np.uint8)


def blocks(img: np.ndarray, b: int) -> np.ndarray:
    """Cut ``img`` into non-overlapping b x b blocks.

    Blocks are taken in raster order; inside a block pixels are row-major.
    Returns an (H/b * W/b) x (b*b) array of the image's dtype.
    """
    H, W = img.shape
    if H % b or W % b:
        raise ValueError("image size must be a multiple of the block size")
    t = img.reshape(H // b, b, W // b, b).transpose(0, 2, 1, 3)
    return np.ascontiguousarray(t.reshape(-1, b * b))


def image_training_set(seeds, W: int, H: int, b: int) -> np.ndarray:
    """FP32 training matrix: blocks of images ``image(s, W, H)`` for s in
    ``seeds``, concatenated in seed order.  Values are integers 0..255."""
    parts = [blocks(image(s, W, H), b) for s in seeds]
    return np.ascontiguousarray(np.concatenate(parts, axis=0).astype(np.float32))


def gmm(seed: int, M: int, L: int, K: int, mean_lo=0.0, mean_hi=255.0,
        sigma_lo=4.0, sigma_hi=20.0) -> np.ndarray:
    """M x L FP32 sample of an equal-weight mixture of K isotropic Gaussians.

    Draw order: means (K x L, U[mean_lo, mean_hi]), sigmas (K, U[sigma_lo,
    sigma_hi]), component labels (M, uniform), unit normals (M x L)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(mean_lo, mean_hi, size=(K, L))
    sig = rng.uniform(sigma_lo, sigma_hi, size=K)
    lab = rng.integers(0, K, size=M)
    z = rng.standard_normal(size=(M, L))
    X = means[lab] + sig[lab, None] * z
    return np.ascontiguousarray(X.astype(np.float32))


def gmm_diag(seed: int, M: int, L: int, K: int, mean_sd=10.0, sigma_lo=0.5,
             sigma_hi=3.0) -> np.ndarray:
    """M x L FP32 sample of an equal-weight mixture of K Gaussians with
    means N(0, mean_sd^2) per dimension and a diagonal sigma U[sigma_lo,
    sigma_hi] per component and dimension.  Draw order: means, sigmas,
    labels, unit normals.  Generated in row slabs to bound host memory."""
    rng = np.random.default_rng(seed)
    means = rng.normal(0.0, mean_sd, size=(K, L))
    sig = rng.uniform(sigma_lo, sigma_hi, size=(K, L))
    lab = rng.integers(0, K, size=M)
    X = np.empty((M, L), dtype=np.float32)
    slab = 1 << 16
    for s in range(0, M, slab):
        e = min(M, s + slab)
        z = rng.standard_normal(size=(e - s, L))
        X[s:e] = (means[lab[s:e]] + sig[lab[s:e]] * z).astype(np.float32)
    return X


def distinct_rows(X: np.ndarray, n: int, seed: int) -> np.ndarray:
    """``n`` rows of X that are pairwise distinct, taken in the order of a
    seeded permutation of the row indices; returns their indices."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(X.shape[0])
    seen = set()
    out = []
    for r in perm:
        key = X[r].tobytes()
        if key in seen:
            continue
        seen.add(key)
        out.append(int(r))
        if len(out) == n:
            break
    if len(out) < n:
        raise ValueError("not enough distinct rows")
    return np.asarray(out, dtype=np.int64)


def batched_instances(n_inst: int, base_seed: int = 10_000, M_lo=2048,
                      M_hi=65536, Ls=(16, 64), Ns=(16, 32, 64, 128, 256),
                      scale: float = 1.0):
    """Shapes and data of independent LBG instances.

    Instance i draws from ``default_rng(base_seed + i)``: M_i ~ U{M_lo..M_hi}
    (scaled by ``scale``, at least 1), L_i from ``Ls``, N_i from ``Ns``; its
    rows come from ``gmm`` with N_i components seeded from the same stream.
    Returns a list of (X_i, N_i)."""
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(base_seed + i)
        M = int(rng.integers(M_lo, M_hi + 1))
        L = int(rng.choice(Ls))
        N = int(rng.choice(Ns))
        dseed = int(rng.integers(0, 2**31 - 1))
        M = max(1, int(round(M * scale)))
        out.append((gmm(dseed, M, L, N), N))
    return out
