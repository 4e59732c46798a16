"""Encoder/decoder on the GPU vs the oracle (``oracle.codec``, ``oracle.assign``).

The decoder and the picture kernels only move FP32 values, so the bar is
bit-identity (NaN rows for indices outside [0, N) included, compared as bit
patterns); the encoder is the allocation, so its indices equal the oracle's
FP64 nearest-codevector search.  Cases span several workgroups and ragged
tails: row counts that are not multiples of a pass, L and b off the 16-byte
path, misaligned codebooks (scalar kernels), single rows and pictures of one
block.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import codec

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


def same_bits(a, b):
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    assert a.shape == b.shape
    na, nb = np.isnan(a), np.isnan(b)
    assert np.array_equal(na, nb)
    assert np.array_equal(a[~na].view(np.uint32), b[~nb].view(np.uint32))


DECODE_CASES = [
    # (M, L, N, bad indices)
    (1, 16, 1, False),
    (1000, 16, 256, False),
    (262_147, 16, 256, True),
    (4097, 64, 1024, True),
    (999, 1, 7, True),
    (777, 3, 5, True),
    (513, 17, 33, False),
    (300, 4, 2, False),
    (129, 256, 65, True),
    (2049, 200, 9, False),
]


@pytest.mark.parametrize("M,L,N,bad", DECODE_CASES)
def test_decode_exact(P, M, L, N, bad):
    rng = np.random.default_rng(M + 7 * L + N)
    C = rng.normal(0.0, 50.0, size=(N, L)).astype(np.float32)
    idx = rng.integers(0, N, size=M).astype(np.int32)
    if bad:
        pick = rng.choice(M, size=max(1, M // 50), replace=False)
        idx[pick] = rng.choice(np.array([-1, N, N + 5, -(1 << 30), (1 << 31) - 1], np.int32),
                               size=pick.size)
    Y = P.decode(dev(idx), dev(C))
    torch.cuda.synchronize()
    same_bits(host(Y), codec.decode(C, idx))


def test_decode_misaligned_codebook(P):
    # C one float into its buffer: 4-byte aligned only, so the scalar path
    rng = np.random.default_rng(3)
    M, L, N = 5000, 16, 40
    buf = dev(rng.normal(size=N * L + 1).astype(np.float32))
    C = buf[1:].view(N, L)
    idx = rng.integers(0, N, size=M).astype(np.int32)
    Y = P.decode(dev(idx), C)
    torch.cuda.synchronize()
    same_bits(host(Y), codec.decode(host(C), idx))


PICTURE_CASES = [
    # (nimg, H, W, b)
    (1, 4, 4, 4),
    (1, 8, 8, 2),
    (2, 512, 512, 4),
    (3, 64, 1000, 4),
    (1, 1024, 1024, 8),
    (2, 48, 80, 16),
    (2, 30, 45, 3),
    (1, 7, 13, 1),
    (5, 40, 40, 5),
    (1, 16, 2048, 8),
    (2, 16, 256, 4),    # 64 blocks per block row: stores staged through LDS
    (1, 8, 1280, 4),    # 320 blocks per row: staged, whole waves idle on the second pass
]


@pytest.mark.parametrize("nimg,H,W,b", PICTURE_CASES)
def test_image_blocks_exact(P, nimg, H, W, b):
    rng = np.random.default_rng(nimg * 1000 + H + W + b)
    imgs = rng.integers(0, 256, size=(nimg, H, W)).astype(np.float32)
    X = P.image_blocks(dev(imgs), b)
    torch.cuda.synchronize()
    same_bits(host(X), codec.image_blocks(imgs, b))


@pytest.mark.parametrize("nimg,H,W,b", PICTURE_CASES)
def test_decode_image_exact(P, nimg, H, W, b):
    rng = np.random.default_rng(nimg * 1000 + H + W + b + 1)
    N = 37
    C = rng.normal(100.0, 40.0, size=(N, b * b)).astype(np.float32)
    nv = nimg * (H // b) * (W // b)
    idx = rng.integers(0, N, size=nv).astype(np.int32)
    idx[rng.choice(nv, size=max(1, nv // 97), replace=False)] = N  # corrupt codes
    img = P.decode_image(dev(idx), dev(C), nimg, H, W, b)
    torch.cuda.synchronize()
    same_bits(host(img), codec.decode_image(C, idx, nimg, H, W, b))


def test_picture_round_trip_large(P):
    # 256 pictures of 1024 x 1024, b = 8: blocks, then the blocks as the
    # codebook's stand-in rows, decoded back -- the identity, at full size
    # (4,194,304 vectors of 64 dimensions)
    nimg, H, W, b = 256, 1024, 1024, 8
    g = torch.Generator(device="cuda").manual_seed(11)
    imgs = torch.randint(0, 256, (nimg, H, W), generator=g, device="cuda").to(torch.float32)
    X = P.image_blocks(imgs, b)
    assert X.shape == (nimg * (H // b) * (W // b), b * b)
    # sampled blocks against the oracle's cut of their picture
    for p in (0, 131, 255):
        want = codec.image_blocks(host(imgs[p:p + 1]), b)
        v0 = p * (H // b) * (W // b)
        same_bits(host(X[v0:v0 + want.shape[0]]), want)
    # decode through a codebook made of the first 65,536 blocks: every block
    # whose index lies in range comes back as itself
    N = 65_536
    idx = torch.arange(X.shape[0], device="cuda", dtype=torch.int32)
    back = P.decode_image(idx, X[:N].contiguous(), nimg, H, W, b)
    p_full = N // ((H // b) * (W // b))  # pictures whose blocks all lie below N
    assert torch.equal(back[:p_full], imgs[:p_full])
    assert torch.isnan(back[p_full:]).all()


def test_encode_is_the_allocation(P):
    X = synth.image_training_set((2,), 256, 256, 4)
    rng = np.random.default_rng(5)
    C = np.ascontiguousarray(X[rng.choice(X.shape[0], 64, replace=False)])
    idx = P.encode(dev(X), dev(C))
    torch.cuda.synchronize()
    want, _, _ = oracle.assign(X, C)
    assert np.array_equal(host(idx), want)


def test_codec_end_to_end(P):
    # train on one picture set, code another: PSNR of the decoded pictures
    # (oracle, per sample, FP64) equals the library's PSNR from the GPU
    # distortion, and the rate is log2(N) / L
    b, N = 4, 64
    train_imgs = np.stack([synth.image(s, 256, 256) for s in (20, 21)]).astype(np.float32)
    test_imgs = np.stack([synth.image(s, 256, 256) for s in (30, 31, 32)]).astype(np.float32)
    Xt = P.image_blocks(dev(train_imgs), b)
    C, _, _, _ = P.train(Xt, N)
    Xq = P.image_blocks(dev(test_imgs), b)
    idx = P.encode(Xq, C)
    rec = P.decode_image(idx, C, 3, 256, 256, b)
    D = P.distortion(Xq, C, idx)
    torch.cuda.synchronize()
    ps_lib = P.psnr(D, b * b)
    ps_oracle = codec.psnr(test_imgs, host(rec))
    assert abs(ps_lib - ps_oracle) < 1e-9 * ps_oracle
    assert P.rate(N, b * b) == codec.rate(N, b * b) == 6 / 16
    # the indices are the oracle's nearest codevectors for the GPU codebook
    want, _, _ = oracle.assign(host(Xq), host(C))
    assert np.array_equal(host(idx), want)
    assert math.isfinite(ps_lib) and ps_lib > 20.0


def test_codec_argument_checks(P):
    C = dev(np.zeros((4, 16), np.float32))
    with pytest.raises(ValueError):
        P.decode_image(dev(np.zeros(4, np.int32)), C, 1, 6, 8, 4)  # H not a multiple of b
    with pytest.raises(ValueError):
        P.decode_image(dev(np.zeros(4, np.int32)), C, 1, 8, 8, 3)  # L != b * b
    with pytest.raises(P.LBGError):
        P.image_blocks(dev(np.zeros((1, 34, 34), np.float32)), 17)  # b * b > 256
