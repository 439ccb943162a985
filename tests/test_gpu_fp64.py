"""GPU parity of the FP64 filter against the FP64 oracle.

Both sides are FP64 and differ only in summation order, so the bound is
that of an N^2-term FP64 dot product: |error| <= N^2 u sum_k |H_rk| |X_k|
with u = 2^-53; at N = 8 about 1e-11 for these coefficients (|X| <= ~2100,
sum_k |H_rk| <= ~20 for sum-1 masks with entries up to 1), at N = 16 and 32
(DC up to 4096, 256 and 1024 terms) a few 1e-10 at worst.  The tests use
1e-9 (N <= 16) and 4e-9 (N = 32).
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
TOL = 1e-9
TOL_N = {2: 1e-9, 4: 1e-9, 8: 1e-9, 16: 1e-9, 32: 4e-9}


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
                                        (4, 96, 88, "rand3x5"), (2, 64, 48, "box3"), (8, 72, 40, "rand17"),
                                        (16, 168, 232, "rand7"), (16, 96, 80, "rand33"), (32, 200, 136, "asym5"),
                                        (32, 96, 64, "rand7")])
def test_fp64_filter_matches_oracle(dctf, N, h, w, mask, border):
    W = {"box3": syn.box_mask(3), "asym5": syn.asym_mask_5x5(),
         "rand7": syn.random_mask(np.random.default_rng(4), 7, 7),
         "rand3x5": syn.random_mask(np.random.default_rng(N), 3, 5),
         "rand17": syn.random_mask(np.random.default_rng(8), 17, 17),
         "rand33": syn.random_mask(np.random.default_rng(9), 33, 33)}[mask]
    px = oracle.tile_u8(syn.image_u8(21, h, w), N)
    X = oracle.dct_pixels(px)                      # FP64 coefficients, no rounding
    op = dctf.dctf_build_operator(W, N, border)
    Y = gpu_f64(dctf, op, X)
    Yref = oracle.filter_coeffs(X, W, border)
    assert np.abs(Y - Yref).max() <= TOL_N[N]
    u8, nh = oracle.idct_u8(Y)
    _, u8ref, nhref = oracle.filter_pixels(px, W, border)
    out = ~(nh | nhref)
    assert np.array_equal(u8[out], u8ref[out])


@pytest.mark.parametrize("N,nb", [(8, 257), (16, 131), (32, 70)])
def test_fp64_ragged_counts_are_prefix_identical(dctf, N, nb):
    px = oracle.tile_u8(syn.image_u8(22, 12 * N, 23 * N), N)
    X = oracle.dct_pixels(px)[:nb]
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), N, R)
    full = gpu_f64(dctf, op, X)
    assert np.abs(full - oracle.filter_coeffs(X, syn.asym_mask_5x5(), R)).max() <= TOL_N[N]
    for B in (1, 15, 16, 17, 31, 32, 33, 65, nb - 1):
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


@pytest.mark.parametrize("N,frames,h,w", [(16, 32, 2160, 3840), (32, 32, 2160, 3840)])
def test_fp64_streamed_full_size_sampled(dctf, N, frames, h, w):
    """The N = 16 / N = 32 frames workloads (1,036,800 / 261,120 blocks) in
    FP64, one launch each; sampled outputs against the oracle."""
    nb = ((h + N - 1) // N) * (w // N)
    B = frames * nb
    X32 = torch.empty(B * N * N, dtype=torch.float32, device="cuda")
    for f in range(frames):
        dctf.dctf_forward_dct_u8(torch.from_numpy(syn.image_u8(3000 + f, h, w)).cuda(), N,
                                 X32[f * nb * N * N:(f + 1) * nb * N * N])
    X = X32.double()
    del X32
    W = syn.random_mask(np.random.default_rng(7), 7, 7)
    op = dctf.dctf_build_operator(W, N, Z)
    Y = torch.empty_like(X)
    dctf.dctf_filter_blocks_f64(op, X, Y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.integers(0, B, size=120), [0, B - 1]])
    ti = torch.from_numpy(idx).cuda()
    Xs = X.view(B, N, N)[ti].cpu().numpy()
    Ys = Y.view(B, N, N)[ti].cpu().numpy()
    assert np.abs(Ys - oracle.filter_coeffs(Xs, W, Z)).max() <= TOL_N[N]
    del X, Y
    torch.cuda.empty_cache()


def test_fp64_argument_errors(dctf):
    lib = dctf.raw_library()
    op16 = dctf.dctf_build_operator(syn.box_mask(3), 16, Z)
    op8 = dctf.dctf_build_operator(syn.box_mask(3), 8, Z)
    X = torch.zeros(256 * 2, dtype=torch.float64, device="cuda")
    Y = torch.ones(256 * 2, dtype=torch.float64, device="cuda")
    assert lib.dctf_filter_blocks_f64(op16.handle, X.data_ptr(), Y.data_ptr(), 1, None) == 0
    torch.cuda.synchronize()
    assert float(Y[:256].abs().max()) == 0.0 and float(Y[256:].min()) == 1.0   # one block written
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr(), Y.data_ptr(), 0, None) == 0
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr(), Y.data_ptr(), -1, None) == -1
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr(), X.data_ptr() + 256, 1, None) == -1
    assert lib.dctf_filter_blocks_f64(op8.handle, X.data_ptr() + 8, Y.data_ptr(), 1, None) == -1


def test_fp64_batch_matches_single_calls(dctf):
    """FP64 jobs of N = 4, 8, 16 and 32 in one call equal the single-job
    FP64 filter bit for bit; overlapping outputs are rejected."""
    rng = np.random.default_rng(61)
    jobs, want = [], []
    for k, (N, B) in enumerate(((4, 300), (8, 5000), (16, 700), (32, 90), (8, 1))):
        W = syn.random_mask(rng, 5, 5) if N >= 4 else syn.box_mask(3)
        op = dctf.dctf_build_operator(W, N, k % 2)
        X = torch.randn(B * N * N, dtype=torch.float64, device="cuda") * 40
        Y = torch.full_like(X, float("nan"))
        Wt = torch.empty_like(X)
        dctf.dctf_filter_blocks_f64(op, X, Wt)
        jobs.append((op, X, Y))
        want.append(Wt)
    dctf.dctf_filter_batch_f64(jobs)
    torch.cuda.synchronize()
    for (_, _, Y), Wt in zip(jobs, want):
        assert torch.equal(Y, Wt)
    op, X, Y = jobs[1]
    with pytest.raises(dctf.DctfError):
        dctf.dctf_filter_batch_f64([(op, X, Y), (op, X, Y)])   # two jobs write the same memory
