"""GPU tests of the factored (paper-form) operator and filter.

The mask is decomposed into rank-one terms and the builder forms the N x N
DCT-domain factors P_r, Q_r (Sec. II.B-C, eq. 8-12, 20).  Their Kronecker
sum must be the dense operator of the FP64 oracle (the plain definition,
probed column by column), and the factored FP32 filter must meet the FP32
coefficient tolerance against the oracle's filter.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
TOL_FP32 = 2e-3


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rng_masks():
    rng = np.random.default_rng(31)
    return {
        "box3": (syn.box_mask(3), 1),
        "gauss7": (syn.gaussian_mask(7), 1),
        "row1x5": (rng.uniform(-1, 1, (1, 5)), 1),
        "col5x1": (rng.uniform(-1, 1, (5, 1)), 1),
        "outer5x3": (np.outer(rng.uniform(-1, 1, 5), rng.uniform(-1, 1, 3)), 1),
        "delta": (syn.delta_mask(3, 3, 1, -1), 1),
        "magic3": (syn.magic_square_3(), 3),
        "sym5": (syn.random_mask(rng, 5, 5, symmetric=True), 3),
        "asym5": (syn.asym_mask_5x5(), 5),
        "asym7": (syn.random_mask(rng, 7, 7), 7),
        "zero3": (np.zeros((3, 3)), 1),
    }


@pytest.mark.parametrize("name", sorted(rng_masks()))
def test_rank_of_mask(dctf, name):
    W, want = rng_masks()[name]
    op = dctf.dctf_build_operator(W, 16, Z)
    assert dctf.dctf_operator_rank(op) == want


FACTOR_CASES = [(N, name, b) for N in (2, 4, 8, 16) for name in ("gauss7", "magic3", "sym5", "asym5", "row1x5")
                for b in (Z, R)]


@pytest.mark.parametrize("N,name,border", FACTOR_CASES)
def test_kronecker_sum_is_the_oracle_operator(dctf, N, name, border):
    W, _ = rng_masks()[name]
    if max(W.shape) > 2 * N + 1:
        pytest.skip("mask wider than 2N+1")
    op = dctf.dctf_build_operator(W, N, border)
    P, Q = dctf.dctf_operator_factors_fp64(op)
    H = sum(np.kron(P[r], Q[r]) for r in range(P.shape[0]))
    Href = oracle.operator_probe(N, W, border)
    assert np.abs(H - Href).max() <= 1e-12
    # and the dense image built beside it
    assert np.abs(dctf.dctf_operator_fp64(op) - H).max() <= 1e-12


def test_widest_mask_factors(dctf):
    rng = np.random.default_rng(5)
    W = rng.uniform(-1, 1, (33, 33))
    op = dctf.dctf_build_operator(W, 16, R)
    P, Q = dctf.dctf_operator_factors_fp64(op)
    assert P.shape[0] == 33
    H = sum(np.kron(P[r], Q[r]) for r in range(P.shape[0]))
    assert np.abs(H - oracle.operator_probe(16, W, R)).max() <= 1e-11


def factored(dctf, op, X32):
    X = dev(X32.reshape(-1))
    Y = torch.full_like(X, float("nan"))
    dctf.dctf_filter_blocks_factored(op, X, Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy().reshape(X32.shape)


@pytest.mark.parametrize("name,border", [("gauss7", Z), ("gauss7", R), ("box3", R), ("sym5", R), ("asym5", Z),
                                         ("asym7", Z), ("magic3", R), ("col5x1", Z), ("outer5x3", R)])
def test_factored_filter_matches_oracle(dctf, name, border):
    W, _ = rng_masks()[name]
    px = oracle.tile_u8(syn.image_u8(40, 272, 208), 16)      # 17 x 13 = 221 blocks (ragged tail of U = 4)
    X32 = oracle.coeffs_fp32(px)
    op = dctf.dctf_build_operator(W, 16, border)
    Y = factored(dctf, op, X32)
    Yref = oracle.filter_coeffs(X32, W, border)
    assert np.abs(Y.astype(np.float64) - Yref).max() <= TOL_FP32
    # same block results as the dense FP32 path, up to FP32 rounding
    Xd = dev(X32.reshape(-1))
    Yd = torch.empty_like(Xd)
    dctf.dctf_filter_blocks(op, 0, Xd, Yd)
    torch.cuda.synchronize()
    assert np.abs(Yd.cpu().numpy().reshape(Y.shape) - Y).max() <= TOL_FP32


def test_factored_large_sampled_and_prefix_identity(dctf):
    """Many blocks (every wave strides over several iterations), checked on
    sampled outputs; a prefix run gives bit-identical blocks."""
    B = 300_003
    X32 = syn.coeff_like_fp32(8, B, 16)
    W = syn.gaussian_mask(5)
    op = dctf.dctf_build_operator(W, 16, R)
    Y = factored(dctf, op, X32)
    rng = np.random.default_rng(2)
    bi = np.concatenate([rng.integers(0, B, 3000), np.arange(B - 8, B)])
    ci = rng.integers(0, 256, bi.size)
    ref = oracle.filter_coeffs_sampled(X32, W, R, bi, ci)
    got = Y.reshape(B, 256)[bi, ci].astype(np.float64)
    assert np.abs(got - ref).max() <= TOL_FP32
    for k in (1, 3, 5, 4097):
        assert np.array_equal(factored(dctf, op, X32[:k]), Y[:k]), k


def test_factored_errors(dctf):
    op8 = dctf.dctf_build_operator(syn.box_mask(3), 8, Z)
    x = torch.zeros(64 * 4, device="cuda")
    with pytest.raises(dctf.DctfError) as e:
        dctf.dctf_filter_blocks_factored(op8, x, torch.zeros_like(x))
    assert e.value.status == dctf.DCTF_EUNSUPPORTED
    big = dctf.dctf_build_operator(np.random.default_rng(9).uniform(-1, 1, (9, 9)), 16, Z)
    assert dctf.dctf_operator_rank(big) == 9
    x16 = torch.zeros(256 * 4, device="cuda")
    with pytest.raises(dctf.DctfError) as e:
        dctf.dctf_filter_blocks_factored(big, x16, torch.zeros_like(x16))
    assert e.value.status == dctf.DCTF_EUNSUPPORTED
    op = dctf.dctf_build_operator(syn.box_mask(3), 16, Z)
    with pytest.raises(dctf.DctfError):          # in-place
        dctf.dctf_filter_blocks_factored(op, x16, x16)
    with pytest.raises(dctf.DctfError):          # misaligned
        dctf.dctf_filter_blocks_factored(op, x16[1:257], torch.zeros(256, device="cuda"))
    empty = torch.empty(0, device="cuda")
    dctf.dctf_filter_blocks_factored(op, empty, empty)   # B = 0: no-op


# ---------------------------------------------------------------- N = 32

@pytest.mark.parametrize("name,border", [("gauss7", Z), ("asym5", R), ("magic3", Z), ("row1x5", R)])
def test_kronecker_sum_is_the_oracle_operator_n32(dctf, name, border):
    W, _ = rng_masks()[name]
    op = dctf.dctf_build_operator(W, 32, border)
    P, Q = dctf.dctf_operator_factors_fp64(op)
    H = sum(np.kron(P[r], Q[r]) for r in range(P.shape[0]))
    assert np.abs(H - oracle.operator_probe(32, W, border)).max() <= 1e-12


@pytest.mark.parametrize("name,border", [("gauss7", Z), ("box3", R), ("asym5", Z), ("asym7", R), ("magic3", R),
                                         ("outer5x3", Z), ("rank8", R)])
def test_factored_filter_n32_matches_oracle(dctf, name, border):
    """32 x 32 blocks (two chained quadrant products per rank term, ranks 1
    to 8) against the oracle's filter and the dense FP32 path; 15 blocks
    leave a ragged tail of the two-block units."""
    if name == "rank8":
        W = syn.random_mask(np.random.default_rng(8), 8, 8)
    else:
        W, _ = rng_masks()[name]
    px = oracle.tile_u8(syn.image_u8(41, 160, 96), 32)          # 5 x 3 = 15 blocks
    X32 = oracle.coeffs_fp32(px)
    op = dctf.dctf_build_operator(W, 32, border)
    assert dctf.dctf_operator_rank(op) <= 8
    Y = factored(dctf, op, X32)
    Yref = oracle.filter_coeffs(X32, W, border)
    assert np.abs(Y.astype(np.float64) - Yref).max() <= TOL_FP32
    Xd = dev(X32.reshape(-1))
    Yd = torch.empty_like(Xd)
    dctf.dctf_filter_blocks(op, 0, Xd, Yd)
    torch.cuda.synchronize()
    assert np.abs(Yd.cpu().numpy().reshape(Y.shape) - Y).max() <= TOL_FP32


def test_factored_n32_many_blocks_prefix_identity(dctf):
    """Every wave strides over several units: sampled outputs against the
    oracle, and a prefix run bit-identical."""
    B = 40_001
    X32 = syn.coeff_like_fp32(9, B, 32)
    W = syn.random_mask(np.random.default_rng(3), 5, 5)
    op = dctf.dctf_build_operator(W, 32, Z)
    Y = factored(dctf, op, X32)
    rng = np.random.default_rng(4)
    bi = np.concatenate([rng.integers(0, B, 200), np.arange(B - 3, B)])
    ref = oracle.filter_coeffs(X32[bi].astype(np.float64), W, Z)
    assert np.abs(Y[bi].astype(np.float64) - ref).max() <= TOL_FP32
    Yp = factored(dctf, op, X32[:777])
    assert np.array_equal(Yp, Y[:777])
