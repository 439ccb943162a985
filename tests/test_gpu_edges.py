"""Degenerate and extreme cases across the GPU paths, against the oracle or
against what the definition fixes exactly.

  * an all-zero mask gives all-zero outputs on every path;
  * a 1x1 mask c scales the block by c (H = c I up to the FP64 rounding of
    the two transforms, which leaves off-diagonal entries below N eps64);
    with c a power of two the diagonal product is exact, so each output is
    c X rounded once, plus at most that residue times the block's sum |X|;
  * the largest mask a block size allows (2N + 1 per side, reaching the
    far edge of the block from every pixel) on the block-local filter (the
    builder is tested at that size with random masks elsewhere);
  * filtered pixels that leave [0, 255] saturate (a mask of sum 2 doubles
    the bright pixels; a negative mask drives them below zero).
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
FP32, SPLIT = 0, 1
TOL = {FP32: 2e-3, SPLIT: 5e-3}


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def coeffs(seed, h, w, N):
    px = oracle.tile_u8(syn.image_u8(seed, h, w), N)
    return px, oracle.coeffs_fp32(px)


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_zero_mask_gives_zero_on_every_path(dctf, N):
    _, X32 = coeffs(60 + N, 4 * N, 6 * N, N)
    op = dctf.dctf_build_operator(np.zeros((3, 3)), N, R)
    X = dev(X32.reshape(-1))
    for prec in (FP32, SPLIT):
        Y = torch.full_like(X, 7.0)
        dctf.dctf_filter_blocks(op, prec, X, Y)
        torch.cuda.synchronize()
        assert float(Y.abs().max()) == 0.0, prec
        if N <= 16:
            pix = torch.full((X.numel(),), 9, dtype=torch.uint8, device="cuda")
            dctf.dctf_filter_blocks_u8(op, prec, X, pix)
            torch.cuda.synchronize()
            assert int(pix.max()) == 0
    X64 = X.double()
    Y64 = torch.full_like(X64, 3.0)
    dctf.dctf_filter_blocks_f64(op, X64, Y64)
    torch.cuda.synchronize()
    assert float(Y64.abs().max()) == 0.0


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
@pytest.mark.parametrize("border", [Z, R])
def test_one_by_one_mask_scales_exactly(dctf, N, border):
    _, X32 = coeffs(70 + N, 5 * N, 4 * N, N)
    op = dctf.dctf_build_operator(np.array([[0.5]]), N, border)
    H = dctf.dctf_operator_fp64(op)
    # the builder's FP64 residue: sums of N products of unit-size terms
    off = np.abs(H - 0.5 * np.eye(N * N)).max()
    assert off <= N * np.finfo(np.float64).eps, off
    X = dev(X32.reshape(-1))
    Y = torch.empty_like(X)
    dctf.dctf_filter_blocks(op, FP32, X, Y)
    torch.cuda.synchronize()
    got = Y.cpu().numpy().reshape(X32.shape).astype(np.float64)
    want = 0.5 * X32.astype(np.float64)
    # FP32 rounding of the operator keeps the residue's size (up to 2^-24)
    resid = 1.01 * off * np.abs(X32).astype(np.float64).sum(axis=(-2, -1), keepdims=True)
    bound = np.abs(want) * 2.0 ** -24 + 2.0 * resid
    assert (np.abs(got - want) <= bound).all()
    # where the block's own term dominates the residue, the result is exact
    big = np.abs(want) >= 2.0 ** 26 * resid
    assert big.mean() > 0.9 and np.array_equal(got[big], want[big])


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,border", [(8, Z), (8, R), (16, Z), (16, R)])
def test_largest_mask_on_the_filter(dctf, N, border, prec):
    # a broad positive mask (sum 1): every output reads the whole block, and
    # the outputs stay in the pixel range (a random mask of this size would
    # amplify the noise by orders of magnitude, beyond what FP32 resolves to 2e-3)
    K = 2 * N + 1
    W = syn.gaussian_mask(K, sigma=N / 2.0)
    px, X32 = coeffs(80 + N, 6 * N, 5 * N, N)
    op = dctf.dctf_build_operator(W, N, border)
    X = dev(X32.reshape(-1))
    Y = torch.empty_like(X)
    dctf.dctf_filter_blocks(op, prec, X, Y)
    torch.cuda.synchronize()
    Yref, _, _ = oracle.filter_pixels(px, W, border)
    err = np.abs(Y.cpu().numpy().reshape(Yref.shape) - Yref).max()
    assert err <= TOL[prec], err


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [8, 16])
def test_saturating_pixels(dctf, N, prec):
    px, X32 = coeffs(90 + N, 8 * N, 8 * N, N)
    X = dev(X32.reshape(-1))
    pix = torch.empty(X.numel(), dtype=torch.uint8, device="cuda")
    for W in (2.0 * syn.gaussian_mask(3), -syn.box_mask(3)):
        op = dctf.dctf_build_operator(W, N, R)
        dctf.dctf_filter_blocks_u8(op, prec, X, pix)
        torch.cuda.synchronize()
        _, u8, nh = oracle.filter_coeffs_to_pixels(X32.astype(np.float64), W, R)
        got = pix.cpu().numpy().reshape(u8.shape)
        assert np.array_equal(got[~nh], u8[~nh])
        # the masks do push pixels out of range on both sides
        assert (u8 == 255).any() or (u8 == 0).any()


@pytest.mark.parametrize("N", [8, 16])
def test_u8_conversion_saturates_and_nan_gives_zero(dctf, N):
    """The packed byte conversion of the verify kernels: blocks whose only
    coefficient is DC = N * v hold the pixel v everywhere; out-of-range values
    saturate to 0 or 255, NaN converts to 0 (the library's stated rule)."""
    vals = [256.0, 300.0, 1e9, float("inf"), -0.5, -300.0, float("-inf"), float("nan"), 254.6, 0.4, 127.2, 12.49]
    want = [255, 255, 255, 255, 0, 0, 0, 0, 255, 0, 127, 12]
    Y = torch.zeros(len(vals), N * N, dtype=torch.float32)
    Y[:, 0] = torch.tensor(vals) * N
    pix = torch.empty(len(vals) * N * N, dtype=torch.uint8, device="cuda")
    dctf.dctf_idct_u8_verify(N, Y.reshape(-1).cuda(), pix)
    torch.cuda.synchronize()
    got = pix.cpu().numpy().reshape(len(vals), N * N)
    for k, w in enumerate(want):
        assert (got[k] == w).all(), (vals[k], got[k][:4], w)
