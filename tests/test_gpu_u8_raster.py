"""GPU tests of the one-pass uint8 path: uint8 images in, filtered uint8
images out (N = 8), through the pixel-to-pixel operator (forward DCT,
DCT-domain filter and inverse DCT as one matrix).

The builder's FP64 pixel-to-pixel operator must equal the oracle's spatial
filter probed with unit pixel blocks (the block-local correlation the
DCT-domain operator is the orthogonal similarity of) to 1e-12; the filtered
images must equal the oracle's uint8 of the spatially filtered blocks
outside the 1e-3 band around .5, in both precisions; several images in one
call must equal one call per image; and the result must agree with the
two-pass route (forward DCT, then filtered pixels into a raster image)
except at near-1/2 pixels.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
FP32, SPLIT = 0, 1
N = 8


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def untile(blocks, h, w):
    bh, bw = -(-h // N), -(-w // N)
    return blocks.reshape(bh, bw, N, N).transpose(0, 2, 1, 3).reshape(bh * N, bw * N)[:h, :w]


MASKS = {"box3": syn.box_mask(3), "asym5": syn.asym_mask_5x5(),
         "rand7": syn.random_mask(np.random.default_rng(17), 7, 7),
         "gauss17": syn.gaussian_mask(17, sigma=3.0), "row1x5": syn.random_mask(np.random.default_rng(18), 1, 5)}


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("mask", sorted(MASKS))
def test_pixpix_operator_is_the_spatial_filter(dctf, mask, border):
    W = MASKS[mask]
    op = dctf.dctf_build_operator(W, N, border)
    H = dctf.dctf_operator_pixpix_fp64(op)
    E = np.eye(N * N).reshape(N * N, N, N)
    probe = oracle.filter_spatial(E, W, border).reshape(N * N, N * N).T
    assert np.abs(H - probe).max() <= 1e-12


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("h,w,mask,border", [(77, 131, "asym5", R), (64, 64, "box3", Z), (1, 1, "rand7", R),
                                             (5, 300, "gauss17", Z), (203, 3, "row1x5", R), (512, 520, "rand7", Z)])
def test_u8_raster_matches_oracle(dctf, h, w, mask, border, prec):
    W = MASKS[mask]
    img = syn.image_u8(500 + h + w, h, w)
    op = dctf.dctf_build_operator(W, N, border)
    pitch = (w + 3) // 4 * 4 + 4
    src = torch.zeros((h, pitch), dtype=torch.uint8, device="cuda")
    src[:, :w] = torch.from_numpy(img).cuda()
    dst = torch.full((h + 1, pitch + 8), 99, dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_u8_raster(op, prec, src[:, :w], h, w, dst[:h, :w])
    torch.cuda.synchronize()
    got = dst.cpu().numpy()
    px = oracle.tile_u8(img, N)
    _, u8, nh = oracle.filter_pixels(px, W, border)
    ref, band = untile(u8, h, w), untile(nh, h, w)
    assert np.array_equal(got[:h, :w][~band], ref[~band])
    assert np.abs(got[:h, :w][band].astype(int) - ref[band].astype(int)).max(initial=0) <= 1
    assert (got[:h, w:] == 99).all() and (got[h:] == 99).all()


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_u8_raster_many_images_and_two_pass_route(dctf, prec):
    """Four images in one call equal one call each; and the one-pass result
    agrees with the forward DCT followed by the filtered raster output,
    except at pixels within the 1/2 band (either rounding)."""
    h, w, n = 130, 204, 4
    W = MASKS["asym5"]
    op = dctf.dctf_build_operator(W, N, R)
    imgs = np.stack([syn.image_u8(520 + i, h, w) for i in range(n)])
    src = torch.from_numpy(imgs).cuda()
    dst = torch.zeros((n, h, w), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_u8_raster(op, prec, src, h, w, dst)
    one = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
    nb = -(-h // N) * -(-w // N)
    X = torch.empty(nb * N * N, dtype=torch.float32, device="cuda")
    two = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
    for i in range(n):
        dctf.dctf_filter_u8_raster(op, prec, src[i], h, w, one)
        torch.cuda.synchronize()
        assert torch.equal(dst[i], one), i
        dctf.dctf_forward_dct_u8(src[i], N, X)
        dctf.dctf_filter_blocks_u8_raster(op, prec, X, h, w, two)
        torch.cuda.synchronize()
        _, _, nh = oracle.filter_pixels(oracle.tile_u8(imgs[i], N), W, R)
        band = untile(nh, h, w)
        a, b = one.cpu().numpy(), two.cpu().numpy()
        assert np.array_equal(a[~band], b[~band]), i
        assert np.abs(a.astype(int) - b.astype(int)).max() <= 1


def test_u8_raster_argument_errors(dctf):
    lib = dctf.raw_library()
    op = dctf.dctf_build_operator(syn.box_mask(3), N, Z)
    a = torch.zeros(64 * 64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64 * 64, dtype=torch.uint8, device="cuda")
    f = lib.dctf_filter_u8_raster
    pa, pb = a.data_ptr(), b.data_ptr()
    assert f(op.handle, FP32, pa, 16, 0, 16, 16, 1, pb, 16, 0, None) == 0
    assert f(op.handle, 3, pa, 16, 0, 16, 16, 1, pb, 16, 0, None) == -1              # precision
    assert f(op.handle, FP32, pa, 18, 0, 16, 16, 1, pb, 16, 0, None) == -1           # in pitch % 4
    assert f(op.handle, FP32, pa, 16, 0, 16, 16, 1, pb, 12, 0, None) == -1           # out pitch < w
    assert f(op.handle, FP32, pa, 16, 256, 16, 16, 2, pb, 16, 200, None) == -1       # out images overlap
    assert f(op.handle, FP32, pa, 16, 0, 16, 16, 1, pa + 64, 16, 0, None) == -1      # in / out overlap
    assert f(op.handle, FP32, pa + 1, 16, 0, 16, 16, 1, pb, 16, 0, None) == -1       # alignment
    assert f(op.handle, FP32, pa, 16, 0, 0, 16, 1, pb, 16, 0, None) == 0             # no-op
    op16 = dctf.dctf_build_operator(syn.box_mask(3), 16, Z)
    assert f(op16.handle, FP32, pa, 16, 0, 16, 16, 1, pb, 16, 0, None) == -2
    with pytest.raises(dctf.DctfError):
        dctf.dctf_operator_pixpix_fp64(op16)
