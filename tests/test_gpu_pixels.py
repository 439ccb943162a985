"""GPU parity of the pixel-output path (filter, inverse DCT and uint8 in one
pass) and of the JPEG-style quantised input, against the FP64 oracle.

The builder's FP64 pixel-domain operator G must match the oracle's probe
G[:, k] = filter(IDCT(e_k)) to 1e-12.  Pixels must equal the oracle's uint8
of filter(IDCT(X)) exactly, except pixels within 1e-3 of a .5 boundary
(counted separately); X is the FP32 input the kernel reads (or the
dequantised integers), taken exactly in FP64.
"""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def image_case(seed, h, w, N):
    px = oracle.tile_u8(syn.image_u8(seed, h, w), N)
    return px, oracle.coeffs_fp32(px)


def gpu_px(dctf, op, X32, prec):
    X = dev(X32.reshape(-1))
    pix = torch.empty(X.numel(), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_blocks_u8(op, prec, X, pix)
    torch.cuda.synchronize()
    return pix.cpu().numpy().reshape(X32.shape)


def gpu_qpx(dctf, op, qc, q, dc, prec):
    Q = dev(qc.reshape(-1))
    pix = torch.empty(Q.numel(), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_quantized_u8(op, prec, Q, dev(q.astype(np.float32).reshape(-1)), dc, pix)
    torch.cuda.synchronize()
    return pix.cpu().numpy().reshape(qc.shape)


def assert_u8_exact(pix, X64, W, border):
    _, u8, nh = oracle.filter_coeffs_to_pixels(X64, W, border)
    outside = ~nh
    bad = int((pix[outside] != u8[outside]).sum())
    assert bad == 0, "%d uint8 mismatches outside the 1/2 band" % bad
    # inside the band either rounding is accepted: at most one apart
    assert np.abs(pix[nh].astype(int) - u8[nh].astype(int)).max(initial=0) <= 1
    return int(nh.sum())


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N,kh,kw", [(2, 3, 3), (4, 3, 5), (8, 3, 3), (8, 5, 5), (8, 7, 7), (8, 1, 5),
                                     (16, 7, 7), (16, 4, 4), (16, 33, 33)])
def test_pixel_operator_matches_oracle_probe(dctf, N, kh, kw, border):
    W = np.random.default_rng(7 * N + kh + 3 * kw).uniform(-1, 1, size=(kh, kw))
    op = dctf.dctf_build_operator(W, N, border)
    G = dctf.dctf_operator_pixel_fp64(op)
    assert np.abs(G - oracle.pixel_operator_probe(N, W, border)).max() <= 1e-12
    # the DCT-domain operator of the same build is unaffected
    assert np.abs(dctf.dctf_operator_fp64(op) - oracle.operator_probe(N, W, border)).max() <= 1e-12


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,h,w,mask,border", [
    (8, 64, 64, "box3", Z),
    (8, 512, 512, "gauss3", Z),
    (8, 512, 512, "asym5", R),
    (8, 200, 136, "magic", R),
    (16, 344, 520, "rand7", Z),
    (16, 344, 520, "rand7", R),
    (4, 96, 88, "rand3x5", R),
    (2, 64, 48, "box3", Z),
])
def test_filtered_pixels_match_oracle(dctf, N, h, w, mask, border, prec):
    W = {"box3": syn.box_mask(3), "gauss3": syn.gaussian_mask(3), "asym5": syn.asym_mask_5x5(),
         "magic": syn.magic_square_3(True), "rand7": syn.random_mask(np.random.default_rng(4), 7, 7),
         "rand3x5": syn.random_mask(np.random.default_rng(N), 3, 5)}[mask]
    px, X = image_case(11, h, w, N)
    op = dctf.dctf_build_operator(W, N, border)
    pix = gpu_px(dctf, op, X, prec)
    near = assert_u8_exact(pix, X.astype(np.float64), W, border)
    print("N=%d %s border=%d prec=%d near-1/2 pixels: %d of %d" % (N, mask, border, prec, near, pix.size))


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [8, 16])
def test_pixels_ragged_counts_are_prefix_identical(dctf, N, prec):
    px, X = image_case(6, 16 * N, 17 * N, N)
    X = X[:257]
    W = syn.random_mask(np.random.default_rng(9), 5, 5)
    op = dctf.dctf_build_operator(W, N, R)
    full = gpu_px(dctf, op, X, prec)
    assert_u8_exact(full, X.astype(np.float64), W, R)
    for B in (1, 15, 16, 17, 31, 33, 100, 255):
        assert np.array_equal(gpu_px(dctf, op, X[:B], prec), full[:B]), B


def quant_case(seed, h, w, N):
    px = oracle.tile_u8(syn.image_u8(seed, h, w), N)
    q = syn.quant_table(N)
    dc = 128.0 * N
    qc = syn.quantize(oracle.dct_pixels(px), q, dc)
    return qc, q, dc


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,border", [(8, R), (8, Z), (16, R), (4, Z), (2, R)])
def test_quantized_input_matches_oracle(dctf, N, border, prec):
    qc, q, dc = quant_case(12, 256 if N >= 8 else 64, 320 if N >= 8 else 96, N)
    W = syn.random_mask(np.random.default_rng(31), 5, 5, symmetric=True)
    op = dctf.dctf_build_operator(W, N, border)
    pix = gpu_qpx(dctf, op, qc, q, dc, prec)
    assert_u8_exact(pix, oracle.dequantize(qc, q, dc), W, border)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [8, 16])
def test_quantized_ragged_counts_are_prefix_identical(dctf, N, prec):
    qc, q, dc = quant_case(13, 16 * N, 17 * N, N)
    qc = qc[:257]
    W = syn.gaussian_mask(5, 1.2)
    op = dctf.dctf_build_operator(W, N, R)
    full = gpu_qpx(dctf, op, qc, q, dc, prec)
    assert_u8_exact(full, oracle.dequantize(qc, q, dc), W, R)
    for B in (1, 15, 16, 17, 33, 200):
        assert np.array_equal(gpu_qpx(dctf, op, qc[:B], q, dc, prec), full[:B]), B


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_full_size_sampled(dctf, prec):
    """The 64-image workload's size (4,194,304 8x8 blocks) in one launch, the
    launch the benchmark times: sampled blocks against the oracle."""
    N, side, images = 8, 2048, 64
    nb = (side // N) ** 2
    X = torch.empty(images * nb * N * N, dtype=torch.float32, device="cuda")
    for i in range(images):
        dctf.dctf_forward_dct_u8(torch.from_numpy(syn.image_u8(1000 + i, side, side)).cuda(), N,
                                 X[i * nb * N * N:(i + 1) * nb * N * N])
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_operator(W, N, R)
    pix = torch.empty(X.numel(), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_blocks_u8(op, prec, X, pix)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    blocks = np.concatenate([rng.integers(0, images * nb, size=3000), [0, images * nb - 1]])
    Xs = X.view(-1, N, N)[torch.from_numpy(blocks).cuda()].cpu().numpy().astype(np.float64)
    got = pix.view(-1, N, N)[torch.from_numpy(blocks).cuda()].cpu().numpy()
    assert_u8_exact(got, Xs, W, R)
    del X, pix
    torch.cuda.empty_cache()


def test_pixel_entry_points_reject_bad_arguments(dctf):
    op = dctf.dctf_build_operator(syn.box_mask(3), 8, Z)
    lib = dctf.raw_library()
    X = torch.zeros(64 * 4, dtype=torch.float32, device="cuda")
    pix = torch.zeros(64 * 4 + 16, dtype=torch.uint8, device="cuda")
    P = lambda t, off=0: t.data_ptr() + off
    assert lib.dctf_filter_blocks_u8(op.handle, 0, P(X), P(pix), 0, None) == 0          # no-op
    assert lib.dctf_filter_blocks_u8(op.handle, 0, P(X), P(pix), -1, None) == -1
    assert lib.dctf_filter_blocks_u8(op.handle, 2, P(X), P(pix), 4, None) == -1          # prec
    assert lib.dctf_filter_blocks_u8(op.handle, 0, P(X), P(pix, 1), 4, None) == -1       # misaligned
    assert lib.dctf_filter_blocks_u8(op.handle, 0, P(X), P(X, 64), 1, None) == -1        # overlap
    assert lib.dctf_filter_blocks_u8(op.handle, 0, None, P(pix), 4, None) == -1
    Q = torch.zeros(64 * 4, dtype=torch.int16, device="cuda")
    qt = torch.ones(64, dtype=torch.float32, device="cuda")
    f = ctypes_float(0.0)
    assert lib.dctf_filter_quantized_u8(op.handle, 0, P(Q), None, f, P(pix), 4, None) == -1
    assert lib.dctf_filter_quantized_u8(op.handle, 0, P(Q), P(qt), ctypes_float(float("nan")), P(pix), 4,
                                        None) == -1
    assert lib.dctf_filter_quantized_u8(op.handle, 0, P(Q), P(qt), f, P(pix), 4, None) == 0
    torch.cuda.synchronize()
    assert int(pix[:256].max()) == 0          # zeros in -> zeros out


def ctypes_float(v):
    import ctypes
    return ctypes.c_float(v)


# ------------------------------------------------------------ raster output

def untile(blocks, h, w, N):
    """[Bh * Bw, N, N] blocks in raster order -> the h x w image they tile."""
    bh, bw = -(-h // N), -(-w // N)
    img = blocks.reshape(bh, bw, N, N).transpose(0, 2, 1, 3).reshape(bh * N, bw * N)
    return img[:h, :w]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,h,w,border", [(8, 77, 131, R), (8, 64, 64, Z), (8, 1, 1, Z), (8, 5, 300, R),
                                          (8, 203, 3, Z), (16, 77, 131, Z), (16, 160, 48, R), (16, 17, 1, R),
                                          (4, 30, 41, R), (2, 9, 7, Z)])
def test_raster_output_matches_blocks_and_oracle(dctf, N, h, w, border, prec):
    """Raster pixels equal the block-ordered pixels of the same call put in
    their places (bit for bit) and the oracle's uint8 outside the 1/2 band;
    the image is a column slice of a wider buffer, whose other bytes must stay
    untouched."""
    img = syn.image_u8(300 + h + w + N, h, w)
    px = oracle.tile_u8(img, N)
    X32 = oracle.coeffs_fp32(px)
    W = syn.asym_mask_5x5() if N >= 4 else syn.box_mask(3)
    op = dctf.dctf_build_operator(W, N, border)
    blocks = gpu_px(dctf, op, X32, prec)
    pitch = (w + 7) // 4 * 4 + 8
    buf = torch.full((h + 2, pitch), 77, dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_blocks_u8_raster(op, prec, dev(X32.reshape(-1)), h, w, buf[:, :w])
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    assert np.array_equal(got[:h, :w], untile(blocks, h, w, N))
    assert (got[:h, w:] == 77).all() and (got[h:] == 77).all()
    _, u8, nh = oracle.filter_coeffs_to_pixels(X32.astype(np.float64), W, border)
    ref, band = untile(u8, h, w, N), untile(nh, h, w, N)
    assert np.array_equal(got[:h, :w][~band], ref[~band])


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [8, 16])
def test_quantized_raster_output(dctf, N, prec):
    h, w = 200, 136
    img = syn.image_u8(310 + N, h, w)
    px = oracle.tile_u8(img, N)
    q = syn.quant_table(N)
    qc = syn.quantize(oracle.dct_pixels(px), q, 128.0 * N)
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_operator(W, N, R)
    blocks = gpu_qpx(dctf, op, qc, q, 128.0 * N, prec)
    out = torch.full((h, w), 0, dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_quantized_u8_raster(op, prec, dev(qc.reshape(-1)), dev(q.astype(np.float32).reshape(-1)),
                                         128.0 * N, h, w, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), untile(blocks, h, w, N))


def test_raster_many_images_in_one_call(dctf):
    """Three ragged images in one call, written into a 3-D buffer whose
    images and rows are padded: equal to one call per image, padding
    untouched; the same through the quantised input."""
    N, h, w, n = 8, 45, 70, 3
    imgs = [syn.image_u8(330 + i, h, w) for i in range(n)]
    X32 = np.concatenate([oracle.coeffs_fp32(oracle.tile_u8(im, N)) for im in imgs])
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), N, R)
    X = dev(X32.reshape(-1))
    for prec in (FP32, SPLIT):
        buf = torch.full((n, h + 3, 76), 55, dtype=torch.uint8, device="cuda")
        dctf.dctf_filter_blocks_u8_raster(op, prec, X, h, w, buf[:, :, :w])
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        per = X32.shape[0] // n
        for i in range(n):
            one = torch.zeros((h, 72), dtype=torch.uint8, device="cuda")   # row pitch a multiple of 4
            dctf.dctf_filter_blocks_u8_raster(op, prec, dev(X32[i * per:(i + 1) * per].reshape(-1)), h, w,
                                              one[:, :w])
            torch.cuda.synchronize()
            assert np.array_equal(got[i, :h, :w], one[:, :w].cpu().numpy()), (prec, i)
        assert (got[:, :h, w:] == 55).all() and (got[:, h:] == 55).all()


def test_raster_argument_errors(dctf):
    N = 8
    op = dctf.dctf_build_operator(syn.box_mask(3), N, Z)
    lib = dctf.raw_library()
    X = torch.zeros(8 * 64, dtype=torch.float32, device="cuda")
    img = torch.zeros(64 * 64, dtype=torch.uint8, device="cuda")
    p = img.data_ptr()
    f = lib.dctf_filter_blocks_u8_raster
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 1, p, 16, 0, None) == 0
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 2, p, 16, 256, None) == 0        # two images
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 2, p, 16, 200, None) == -1       # images overlap
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 2, p, 16, 258, None) == -1       # stride % 4
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 1, p, 18, 0, None) == -1         # pitch % 4
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 1, p, 12, 0, None) == -1         # pitch < w
    assert f(op.handle, FP32, X.data_ptr(), -1, 16, 1, p, 16, 0, None) == -1
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, -1, p, 16, 0, None) == -1
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 1, p + 2, 16, 0, None) == -1     # alignment
    assert f(op.handle, FP32, X.data_ptr(), 0, 16, 1, p, 16, 0, None) == 0           # no-op
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 0, p, 16, 0, None) == 0          # no-op
    # the input overlapping the image
    assert f(op.handle, FP32, X.data_ptr(), 16, 16, 1, X.data_ptr(), 16, 0, None) == -1
    op32 = dctf.dctf_build_operator(syn.box_mask(3), 32, Z)
    assert f(op32.handle, FP32, X.data_ptr(), 8, 8, 1, p, 16, 0, None) == -2
