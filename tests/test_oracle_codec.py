"""The encoder/decoder oracle against what fixes it (no GPU).

Pins:
  * rate: the paper's count (Introduction) -- a codebook of N = 2^k needs k
    bits per vector, shared by L samples -- checked with integer bit counts;
  * psnr: closed forms (a constant error e gives 20 log10(peak / e); 48.13 dB
    for e = 1 on 8-bit data; doubling the error costs 20 log10 2 dB);
  * decode: an identity codebook turns indices into one-hot rows;
  * image_blocks: a 4 x 4 picture cut by hand, and a second implementation
    (reshape / transpose of the synthetic-input module);
  * decode_image: the inverse of image_blocks (codebook = the blocks
    themselves) and the same values as decode in block layout;
  * the PSNR of a decoded training set equals the one computed from the LBG
    distortion as 10 log10(peak^2 L / D), which ties lbg_psnr's formula to
    the per-sample mean squared error.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import codec


def test_rate_counts_bits():
    for k in range(0, 17):
        N = 1 << k
        for L in (1, 2, 3, 16, 64):
            assert codec.rate(N, L) == (N.bit_length() - 1) / L
    # non-powers of two: 2^(rate * L) recovers N
    for N in (3, 5, 100, 1000):
        assert abs(2.0 ** (codec.rate(N, 7) * 7) - N) < 1e-9 * N
    with pytest.raises(ValueError):
        codec.rate(0, 4)


def test_psnr_closed_forms():
    rng = np.random.default_rng(0)
    ref = rng.integers(0, 256, size=(37, 16)).astype(np.float64)
    assert abs(codec.psnr(ref, ref + 1.0) - 48.1308036086791) < 1e-9
    for e in (0.5, 2.0, 3.0, 10.0):
        assert abs(codec.psnr(ref, ref - e) - 20.0 * math.log10(255.0 / e)) < 1e-9
    a = codec.psnr(ref, ref + 3.0)
    b = codec.psnr(ref, ref + 6.0)
    assert abs((a - b) - 20.0 * math.log10(2.0)) < 1e-9
    assert codec.psnr(ref, ref) == math.inf
    # peak scales as 20 log10
    assert abs(codec.psnr(ref, ref + 1.0, peak=1.0)) < 1e-12


def test_decode_identity_codebook():
    L = 6
    C = np.eye(L)
    idx = np.array([0, 5, 2, 2, 4, 1, 3, 0])
    Y = codec.decode(C, idx)
    for m, k in enumerate(idx):
        want = np.zeros(L)
        want[k] = 1.0
        assert np.array_equal(Y[m], want)
    bad = codec.decode(C, np.array([-1, 6, 1 << 30, 2]))
    assert np.isnan(bad[:3]).all() and np.array_equal(bad[3], np.eye(L)[2])


def test_image_blocks_by_hand():
    img = np.arange(16, dtype=np.float64).reshape(1, 4, 4)
    X = codec.image_blocks(img, 2)
    want = np.array([[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]], float)
    assert np.array_equal(X, want)
    # two pictures: the second picture's blocks follow the first's
    two = np.stack([img[0], img[0] + 100.0])
    X2 = codec.image_blocks(two, 2)
    assert np.array_equal(X2[:4], want) and np.array_equal(X2[4:], want + 100.0)
    # b = 1: every pixel is a vector, in raster order
    assert np.array_equal(codec.image_blocks(img, 1)[:, 0], np.arange(16.0))


@pytest.mark.parametrize("b", [1, 2, 3, 4, 8])
def test_image_blocks_matches_reshape(b):
    H, W = 6 * b, 5 * b
    pics = [synth.image(s, W, H) for s in (3, 4)]
    X = codec.image_blocks(np.stack(pics), b)
    want = np.concatenate([synth.blocks(p, b) for p in pics])
    assert np.array_equal(X, want)


@pytest.mark.parametrize("b", [1, 2, 4, 5])
def test_decode_image_inverts_blocks(b):
    rng = np.random.default_rng(b)
    imgs = rng.integers(0, 256, size=(3, 4 * b, 7 * b)).astype(np.float64)
    X = codec.image_blocks(imgs, b)
    back = codec.decode_image(X, np.arange(X.shape[0]), 3, 4 * b, 7 * b, b)
    assert np.array_equal(back, imgs)
    # arbitrary codes: block layout of decode_image = decode
    C = rng.normal(size=(9, b * b))
    idx = rng.integers(-1, 10, size=X.shape[0])
    pic = codec.decode_image(C, idx, 3, 4 * b, 7 * b, b)
    assert np.array_equal(codec.image_blocks(pic, b), codec.decode(C, idx), equal_nan=True)


def test_psnr_from_distortion(olib):
    b, N = 4, 16
    X = synth.image_training_set((5,), 256, 256, b).astype(np.float64)
    r = oracle.train(X.astype(np.float32), N, lib=olib)
    C, idx = r["C"], r["idx"]
    D = oracle.distortion(X.astype(np.float32), C, idx, lib=olib)
    Y = codec.decode(C, idx)
    direct = codec.psnr(X, Y)
    from_d = 10.0 * math.log10(255.0 ** 2 * (b * b) / D)
    assert abs(direct - from_d) < 1e-9 * abs(direct)
    assert 20.0 < direct < 60.0
