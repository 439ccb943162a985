"""GPU parity of the FP64 filter against the FP64 oracle.

Both sides are FP64 and differ only in summation order, so the bound is
that of a 64-term FP64 dot product: |error| <= 64 u sum_k |H_rk| |X_k| with
u = 2^-53, about 1e-11 for these coefficients (|X| <= ~2100, sum_k |H_rk|
<= ~20 for sum-1 masks with entries up to 1).  The tests use 1e-9.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
TOL = 1e-9


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def gpu_f64(dctf, op, X):
    Xd = torch.from_numpy(np.ascontiguousarray(X.reshape(-1))).cuda()
    Y = torch.empty_like(Xd)
    dctf.dctf_filter_blocks_f64(op, Xd, Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy().reshape(X.shape)


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N,h,w,mask", [(8, 64, 64, "box3"), (8, 512, 512, "asym5"), (8, 136, 200, "rand7"),
                                        (4, 96, 88, "rand3x5"), (2, 64, 48, "box3"), (8, 72, 40, "rand17")])
def test_fp64_filter_matches_oracle(dctf, N, h, w, mask, border):
    W = {"box3": syn.box_mask(3), "asym5": syn.asym_mask_5x5(),
         "rand7": syn.random_mask(np.random.default_rng(4), 7, 7),
         "rand3x5": syn.random_mask(np.random.default_rng(N), 3, 5),
         "rand17": syn.random_mask(np.random.default_rng(8), 17, 17)}[mask]
    px = oracle.tile_u8(syn.image_u8(21, h, w), N)
    X = oracle.dct_pixels(px)                      # FP64 coefficients, no rounding
    op = dctf.dctf_build_operator(W, N, border)
    Y = gpu_f64(dctf, op, X)
    Yref = oracle.filter_coeffs(X, W, border)
    assert np.abs(Y - Yref).max() <= TOL
    u8, nh = oracle.idct_u8(Y)
    _, u8ref, nhref = oracle.filter_pixels(px, W, border)
    out = ~(nh | nhref)
    assert np.array_equal(u8[out], u8ref[out])


def test_fp64_ragged_counts_are_prefix_identical(dctf):
    N = 8
    px = oracle.tile_u8(syn.image_u8(22, 16 * N, 17 * N), N)
    X = oracle.dct_pixels(px)[:257]
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), N, R)
    full = gpu_f64(dctf, op, X)
    assert np.abs(full - oracle.filter_coeffs(X, syn.asym_mask_5x5(), R)).max() <= TOL
    for B in (1, 15, 16, 17, 33, 200):
        assert np.array_equal(gpu_f64(dctf, op, X[:B]), full[:B]), B


def test_fp64_full_size_sampled(dctf):
    """4,194,304 8x8 blocks in one launch (the 64-image workload's size):
    sampled outputs against the oracle."""
    N, B = 8, 4194304
    rng = np.random.default_rng(3)
    base = oracle.dct_pixels(oracle.tile_u8(syn.image_u8(23, 256, 256), N))   # 1024 blocks
    X = torch.from_numpy(np.ascontiguousarray(base.reshape(-1))).cuda().repeat(B // 1024)
    X += torch.arange(B, device="cuda", dtype=torch.float64).repeat_interleave(64) * 1e-6
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), N, Z)
    Y = torch.empty_like(X)
    dctf.dctf_filter_blocks_f64(op, X, Y)
    torch.cuda.synchronize()
    idx = np.concatenate([rng.integers(0, B, size=2000), [0, B - 1]])
    ti = torch.from_numpy(idx).cuda()
    Xs = X.view(B, N, N)[ti].cpu().numpy()
    Ys = Y.view(B, N, N)[ti].cpu().numpy()
    assert np.abs(Ys - oracle.filter_coeffs(Xs, syn.asym_mask_5x5(), Z)).max() <= TOL
    del X, Y
    torch.cuda.empty_cache()


def test_fp64_argument_errors(dctf):
    lib = dctf.raw_library()
    op16 = dctf.dctf_build_operator(syn.box_mask(3), 16, Z)
    op8 = dctf.dctf_build_operator(syn.box_mask(3), 8, Z)
    X = torch.zeros(256 * 2, dtype=torch.float64, device="cuda")
    Y = torch.zeros(256 * 2, dtype=torch.float64, device="cuda")
    assert lib.dctf_filter_blocks_f64(op16.handle, X.data_ptr(), Y.data_ptr(), 1, None) == -2
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr(), Y.data_ptr(), 0, None) == 0
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr(), Y.data_ptr(), -1, None) == -1
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr(), X.data_ptr() + 256, 1, None) == -1
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr() + 8, Y.data_ptr(), 1, None) == -1
