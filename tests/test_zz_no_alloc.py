"""GPU test of dctf_filter_batch_noalloc: the same results as
dctf_filter_batch (bit for bit) on two calls in a row, the second with a
smaller input, through the C ABI; and a table beyond the fixed scratch array
is rejected before anything runs."""
import numpy as np
import pytest
import torch

import synthetic as syn

pytestmark = pytest.mark.gpu
FP32, SPLIT = 0, 1


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def jobs_of(dctf, rng, njobs, max_blocks, ops):
    out = []
    for _ in range(njobs):
        op = ops[int(rng.integers(0, len(ops)))]
        B = int(rng.integers(1, max_blocks))
        X = torch.randn(B * op.N * op.N, device="cuda") * 60
        out.append((op, X, torch.full_like(X, float("nan"))))
    return out


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_noalloc_matches_filter_batch(dctf, prec):
    rng = np.random.default_rng(41)
    ops = dctf.dctf_build_operators([(syn.random_mask(rng, k, k), N, b) for N in (8, 16) for k in (3, 5)
                                     for b in (0, 1)])
    for njobs, max_blocks in ((40, 20000), (7, 500)):    # the second call is smaller
        jobs = jobs_of(dctf, rng, njobs, max_blocks, ops)
        want = []
        for op, X, _ in jobs:
            want.append(torch.empty_like(X))
        dctf.dctf_filter_batch([(op, X, W) for (op, X, _), W in zip(jobs, want)], prec)
        dctf.dctf_filter_batch_noalloc(jobs, prec)
        for (_, _, Y), W in zip(jobs, want):
            assert torch.equal(Y, W)


def test_noalloc_rejects_a_table_beyond_the_scratch(dctf):
    """One job descriptor is 40 bytes: 20,000 one-block jobs fit the 1 MiB
    array (and match dctf_filter_batch), 27,000 do not (rejected, nothing
    written)."""
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), 8, 1)
    X = torch.randn(27000 * 64, device="cuda") * 50
    Y = torch.full_like(X, float("nan"))
    W = torch.empty_like(X)
    n = 20000
    jobs = [(op, X[64 * i:64 * (i + 1)], Y[64 * i:64 * (i + 1)]) for i in range(n)]
    dctf.dctf_filter_batch([(op, X[64 * i:64 * (i + 1)], W[64 * i:64 * (i + 1)]) for i in range(n)], SPLIT)
    dctf.dctf_filter_batch_noalloc(jobs, SPLIT)
    assert torch.equal(Y[:64 * n], W[:64 * n])
    Y.fill_(float("nan"))
    big = [(op, X[64 * i:64 * (i + 1)], Y[64 * i:64 * (i + 1)]) for i in range(27000)]
    with pytest.raises(dctf.DctfError) as e:
        dctf.dctf_filter_batch_noalloc(big, SPLIT)
    assert e.value.status == dctf.DCTF_EINVAL
    torch.cuda.synchronize()
    assert torch.isnan(Y).all()


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_noalloc_with_jobs_of_every_block_size(dctf, prec):
    """Jobs of N = 4 and 32 (one launch each, no table entry) beside N = 8
    and 16: the same results as dctf_filter_batch, and a call of only such
    jobs runs them with an empty table."""
    rng = np.random.default_rng(43)
    ops = dctf.dctf_build_operators([(syn.random_mask(rng, 3, 3), N, 1) for N in (4, 8, 16, 32)])
    for njobs, max_blocks in ((12, 3000), (5, 200)):
        jobs = jobs_of(dctf, rng, njobs, max_blocks, ops)
        want = [torch.empty_like(X) for _, X, _ in jobs]
        dctf.dctf_filter_batch([(op, X, W) for (op, X, _), W in zip(jobs, want)], prec)
        dctf.dctf_filter_batch_noalloc(jobs, prec)
        for (_, _, Y), W in zip(jobs, want):
            assert torch.equal(Y, W)
    side_only = jobs_of(dctf, rng, 3, 500, [ops[0], ops[3]])
    dctf.dctf_filter_batch_noalloc(side_only, prec)
    for op, X, Y in side_only:
        W = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, W)
        torch.cuda.synchronize()
        assert torch.equal(Y, W)
