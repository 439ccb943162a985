"""Concurrent use of the library: one operator filtering (dense and parity-class) on several streams
at once, calls from several host threads (ctypes releases the GIL, so the
calls overlap), and operators built concurrently.  Every result must be
bit-identical to the same call made alone on one stream.
"""
import threading

import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
FP32, SPLIT = 0, 1


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def inputs(n, N, side, seed0):
    out = []
    for i in range(n):
        px = oracle.tile_u8(syn.image_u8(seed0 + i, side, side), N)
        out.append(torch.from_numpy(oracle.coeffs_fp32(px).reshape(-1)).cuda())
    return out


@pytest.mark.parametrize("N", [8, 16])
def test_one_operator_on_several_streams(dctf, N):
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), N, R)
    Xs = inputs(4, N, 512, 700)
    ref = {}
    for prec in (FP32, SPLIT):
        for i, X in enumerate(Xs):
            ref[prec, i] = dctf.filter_blocks(op, X, prec)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in Xs]
    outs = {}
    for rep in range(3):
        for prec in (FP32, SPLIT):
            for i, (X, s) in enumerate(zip(Xs, streams)):
                Y = torch.empty_like(X)
                with torch.cuda.stream(s):
                    dctf.dctf_filter_blocks(op, prec, X, Y, s)
                outs[rep, prec, i] = Y
    torch.cuda.synchronize()
    for (rep, prec, i), Y in outs.items():
        assert torch.equal(Y, ref[prec, i]), (rep, prec, i)


@pytest.mark.parametrize("N", [16, 32])
def test_parity_filter_on_several_streams(dctf, N):
    """The parity-class filter of one symmetric operator on four streams at
    once: each result bit-identical to the same call alone."""
    op = dctf.dctf_build_operator(syn.gaussian_mask(7, sigma=1.5), N, R)
    assert dctf.dctf_operator_parity_classes(op) == 4
    Xs = inputs(4, N, 512, 740)
    ref = {}
    for prec in (FP32, SPLIT):
        for i, X in enumerate(Xs):
            Y = torch.empty_like(X)
            dctf.dctf_filter_blocks_parity(op, prec, X, Y)
            ref[prec, i] = Y
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in Xs]
    outs = {}
    for rep in range(3):
        for prec in (FP32, SPLIT):
            for i, (X, s) in enumerate(zip(Xs, streams)):
                Y = torch.empty_like(X)
                with torch.cuda.stream(s):
                    dctf.dctf_filter_blocks_parity(op, prec, X, Y, s)
                outs[rep, prec, i] = Y
    torch.cuda.synchronize()
    for (rep, prec, i), Y in outs.items():
        assert torch.equal(Y, ref[prec, i]), (rep, prec, i)


def test_calls_from_several_host_threads(dctf):
    N = 8
    ops = [dctf.dctf_build_operator(m, N, b) for m in (syn.asym_mask_5x5(), syn.gaussian_mask(3))
           for b in (Z, R)]
    Xs = inputs(4, N, 256, 720)
    ref = {}
    for t in range(4):
        for prec in (FP32, SPLIT):
            ref[t, prec] = dctf.filter_blocks(ops[t], Xs[t], prec)
    torch.cuda.synchronize()
    errors, results = [], {}

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for it in range(20):
                    prec = (FP32, SPLIT)[it % 2]
                    Y = torch.empty_like(Xs[t])
                    dctf.dctf_filter_blocks(ops[t], prec, Xs[t], Y, s)
                    results[t, it] = (prec, Y)
            s.synchronize()
        except Exception as e:   # reported below, on the test's thread
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    assert len(results) == 80
    for (t, it), (prec, Y) in results.items():
        assert torch.equal(Y, ref[t, prec]), (t, it)


def test_operators_built_concurrently(dctf):
    masks = [syn.random_mask(np.random.default_rng(40 + k), 5, 5) for k in range(8)]
    built = [None] * len(masks)
    errors = []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            built[k] = dctf.dctf_build_operator(masks[k], 8, k % 2, s)
            s.synchronize()
        except Exception as e:
            errors.append((k, repr(e)))

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(masks))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for k, op in enumerate(built):
        H = dctf.dctf_operator_fp64(op)
        assert np.abs(H - oracle.operator_probe(8, masks[k], k % 2)).max() <= 1e-12, k
