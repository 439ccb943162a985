"""GPU tests of the parity-class filter (N = 16 and 32, masks mirror-symmetric
on both axes): H_dct splits into four (N^2/4) x (N^2/4) operators, one per
parity class (u % 2, v % 2) of the coefficients, and
dctf_filter_blocks_parity filters through them.

The class operators come from the FP64 H_dct, whose coupling between
classes is zero to rounding (pinned on the oracle by
test_doubly_symmetric_mask_decouples_parity_classes).  Here: which
operators have the classes; the filter against the FP64 oracle at the
dense path's tolerances (FP32 2e-3, split-BF16 5e-3) on natural-image
content, ragged block counts and both borders; agreement with
dctf_filter_blocks; sampled outputs of 32 frames of 3840 x 2160; and the
argument errors.  Each test runs at both block sizes.
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


def sym(A):
    """A averaged with its mirror images, exactly symmetric (each sum pairs
    the same two terms in either order)."""
    B = A + A[::-1]
    return (B + B[:, ::-1]) / 4


RNG = np.random.default_rng(71)
MASKS = {"gauss7": syn.gaussian_mask(7, sigma=1.5), "box3": syn.box_mask(3),
         "sym5": sym(RNG.uniform(-1, 1, (5, 5))), "sym7": sym(RNG.uniform(-1, 1, (7, 7))),
         "row1x9": sym(RNG.uniform(-1, 1, (1, 9))), "col9x1": sym(RNG.uniform(-1, 1, (9, 1))),
         "gauss33": syn.gaussian_mask(33, sigma=5.0), "delta1": np.ones((1, 1)),
         "laplace3": np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])}


def natural_coeffs(B, seed, N):
    """Seeded coefficients whose spread falls with frequency as in natural
    images (the content the split-BF16 bound is stated for), DC near 128 N."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    u = torch.arange(N, device="cuda", dtype=torch.float32)
    decay = (40.0 / (1.0 + u.view(N, 1) + u.view(1, N))).reshape(-1)
    X = torch.randn(B, N * N, device="cuda", generator=gen) * decay
    X[:, 0] += 128.0 * N
    return X.reshape(-1)


def test_which_operators_have_classes(dctf):
    A = np.random.default_rng(3).uniform(-1, 1, (7, 7))
    # the four-term average differs from its mirrors by rounding: still symmetric
    near = (A + A[::-1] + A[:, ::-1] + A[::-1, ::-1]) / 4
    assert not np.array_equal(near, near[::-1]) or not np.array_equal(near, near[:, ::-1])
    off = sym(A).copy()
    off[0, 1] += 1e-9
    for N in (16, 32):
        for W in list(MASKS.values()) + [near]:
            assert dctf.dctf_operator_parity_classes(dctf.dctf_build_operator(W, N, R)) == 4
        for W in ((A + A[:, ::-1]) / 2, (A + A[::-1]) / 2, A, off, np.ones((4, 4)) / 16, np.ones((3, 4)) / 12):
            assert dctf.dctf_operator_parity_classes(dctf.dctf_build_operator(W, N, R)) == 1
    for n in (2, 4, 8):
        assert dctf.dctf_operator_parity_classes(dctf.dctf_build_operator(syn.box_mask(3), n, Z)) == 1


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("mask", sorted(MASKS))
@pytest.mark.parametrize("N", [16, 32])
def test_parity_filter_matches_oracle(dctf, N, mask, border, prec):
    W = MASKS[mask]
    op = dctf.dctf_build_operator(W, N, border)
    B = 16 * 37 + 5   # several tiles per workgroup, ragged tail
    X = natural_coeffs(B, 100 + len(mask) + border + N, N)
    Y = torch.full_like(X, float("nan"))
    dctf.dctf_filter_blocks_parity(op, prec, X, Y)
    D = torch.empty_like(X)
    dctf.dctf_filter_blocks(op, prec, X, D)
    torch.cuda.synchronize()
    X64 = X.double().cpu().numpy().reshape(B, N, N)
    want = oracle.filter_coeffs(X64, W, border).reshape(-1)
    got = Y.cpu().numpy()
    assert np.isfinite(got).all()
    assert np.abs(got - want).max() <= TOL[prec]
    assert np.abs(got - D.cpu().numpy()).max() <= 2 * TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [16, 32])
def test_parity_filter_small_and_empty(dctf, N, prec):
    """B = 0 writes nothing; B = 1, 15, 16, 17, 32, 33 (a partial tile, whole
    tiles, whole tiles and a block): only the first B blocks are written."""
    W = MASKS["gauss7"]
    op = dctf.dctf_build_operator(W, N, R)
    X = natural_coeffs(40, 9, N)
    for B in (0, 1, 15, 16, 17, 32, 33):
        Y = torch.full((40 * N * N,), 7.0, device="cuda")
        dctf.dctf_filter_blocks_parity(op, prec, X[:B * N * N], Y[:B * N * N])
        torch.cuda.synchronize()
        got = Y.cpu().numpy()
        if B:
            want = oracle.filter_coeffs(X[:B * N * N].double().cpu().numpy().reshape(B, N, N), W, R).reshape(-1)
            assert np.abs(got[:B * N * N] - want).max() <= TOL[prec]
        assert (got[B * N * N:] == 7.0).all()


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [16, 32])
def test_parity_filter_full_frames_sampled(dctf, N, prec):
    """32 frames of 3840 x 2160 (1,036,800 blocks at N = 16, 257,280 at
    N = 32), every workgroup over many tiles: sampled outputs against the
    oracle, and the first and last blocks."""
    B = 32 * (2160 // N) * (3840 // N)
    W = MASKS["gauss7"]
    op = dctf.dctf_build_operator(W, N, Z)
    X = natural_coeffs(B, 77 + N, N)
    Y = torch.full_like(X, float("nan"))
    dctf.dctf_filter_blocks_parity(op, prec, X, Y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(78)
    bi = np.concatenate([rng.integers(0, B, 4000), [0, 0, B - 1, B - 1]])
    ci = np.concatenate([rng.integers(0, N * N, 4000), [0, N * N - 1, 0, N * N - 1]])
    Xs = X.view(B, N * N)[torch.from_numpy(bi).cuda()].cpu().numpy()
    want = oracle.filter_coeffs_sampled(Xs, W, Z, np.arange(len(bi)), ci)
    got = Y.view(B, N * N)[torch.from_numpy(bi).cuda(), torch.from_numpy(ci).cuda()].cpu().numpy()
    assert np.abs(got - want).max() <= TOL[prec]
    assert not torch.isnan(Y).any()


@pytest.mark.parametrize("N", [16, 32])
def test_parity_filter_argument_errors(dctf, N):
    lib = dctf.raw_library()
    X = torch.zeros(4 * N * N, dtype=torch.float32, device="cuda")
    Y = torch.zeros(4 * N * N, dtype=torch.float32, device="cuda")
    op = dctf.dctf_build_operator(MASKS["box3"], N, Z)
    asym = dctf.dctf_build_operator(np.arange(9.0).reshape(3, 3) / 36, N, Z)
    op8 = dctf.dctf_build_operator(MASKS["box3"], 8, Z)
    f = lib.dctf_filter_blocks_parity
    assert f(op.handle, SPLIT, X.data_ptr(), Y.data_ptr(), 4, None) == 0
    assert f(op.handle, 2, X.data_ptr(), Y.data_ptr(), 4, None) == -1                   # precision
    assert f(op.handle, SPLIT, X.data_ptr(), X.data_ptr(), 4, None) == -1               # in place
    assert f(op.handle, SPLIT, X.data_ptr() + 4, Y.data_ptr(), 3, None) == -1           # alignment
    assert f(asym.handle, SPLIT, X.data_ptr(), Y.data_ptr(), 4, None) == -2             # no classes
    assert f(op8.handle, SPLIT, X.data_ptr(), Y.data_ptr(), 4, None) == -2
