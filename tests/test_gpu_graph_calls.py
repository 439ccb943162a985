"""Single calls captured into a HIP graph (torch.cuda.graph on the capture
stream) and replayed: the block filter (N = 8, 16, 32), the parity-class filter (N = 16, 32),
the one-pass uint8 filter, the raster pixel output and the multi-image
forward DCT.  Each replay follows eager work that overwrites the outputs,
and must reproduce the eager result bit for bit (the calls enqueue kernel
launches only: no allocation, memset or synchronisation inside)."""
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


def replay_matches(fn, outs):
    """Eager run, capture, then three replays, each after the outputs were
    overwritten eagerly; every replay must equal the eager result."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(s)            # warm-up (first-call queries happen outside the capture)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for r in range(3):
        for o in outs:
            o.fill_(13 + r) if o.dtype == torch.uint8 else o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, ref):
            assert torch.equal(o, e), r


@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_filter_blocks_in_a_graph(dctf, N, prec):
    op = dctf.dctf_build_operator(syn.random_mask(np.random.default_rng(3), 5, 5), N, 1)
    X = torch.randn(3001 * N * N, device="cuda") * 20
    Y = torch.empty_like(X)
    replay_matches(lambda s: dctf.dctf_filter_blocks(op, prec, X, Y, s), [Y])


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_parity_filter_in_a_graph(dctf, N, prec):
    op = dctf.dctf_build_operator(syn.gaussian_mask(7, sigma=1.5), N, 0)
    X = torch.randn(2003 * N * N, device="cuda") * 20
    Y = torch.empty_like(X)
    replay_matches(lambda s: dctf.dctf_filter_blocks_parity(op, prec, X, Y, s), [Y])


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_pixel_paths_in_a_graph(dctf, prec):
    """Forward DCT of several images in one launch, their filtered pixels into
    raster images, and the one-pass uint8 filter, all in one graph."""
    n, h, w = 3, 200, 264
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), 8, 1)
    imgs = torch.from_numpy(np.stack([syn.image_u8(40 + i, h, w) for i in range(n)])).cuda()
    nb = -(-h // 8) * -(-w // 8)
    X = torch.empty(n * nb * 64, dtype=torch.float32, device="cuda")
    two = torch.empty((n, h, w), dtype=torch.uint8, device="cuda")
    one = torch.empty((n, h, w), dtype=torch.uint8, device="cuda")

    def fn(s):
        dctf.dctf_forward_dct_u8_images(imgs, 8, X, s)
        dctf.dctf_filter_blocks_u8_raster(op, prec, X, h, w, two, s)
        dctf.dctf_filter_u8_raster(op, prec, imgs, h, w, one, s)

    replay_matches(fn, [X, two, one])
