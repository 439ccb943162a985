"""Inputs past 2^31 elements (and past 4 GiB): every entry point indexes
blocks with 64-bit offsets, so blocks beyond those boundaries must come out
as right as the first ones.  Each case fills one launch with more than 2^31
elements (8.6 GB of FP32, 17 GB of FP64) and checks sampled blocks, the
blocks on either side of each boundary among them, against the oracle.

Inputs: the coefficient blocks of a 512 x 512 image of the synthetic recipe,
placed by a hash of the block's position and given a hashed DC shift, so
that a block read from a wrapped 32-bit offset would be a different block.
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
TOL_F64 = 1e-9


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


@pytest.fixture(autouse=True)
def release_memory():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def position_hash(B):
    b = torch.arange(B, device="cuda", dtype=torch.int64)
    return (b * 2654435761) % 1000003


def big_coeffs(N, B, seed):
    """FP32 coefficients of B blocks (flat, block-contiguous)."""
    base = oracle.coeffs_fp32(oracle.tile_u8(syn.image_u8(seed, 512, 512), N)).reshape(-1, N * N)
    base = torch.from_numpy(np.ascontiguousarray(base)).cuda()
    h = position_hash(B)
    X = base[h % base.shape[0]]
    X[:, 0] += (h % 1024).to(torch.float32) * 0.25 - 128.0
    del h
    return X.reshape(-1)


def boundary_blocks(nn, B, elem_bytes, seed, n=1500):
    """Random blocks plus those on either side of element 2^31 and of byte
    offsets 2^31 and 2^32, and the first and last blocks."""
    marks = [0, 1, B - 2, B - 1]
    for e in (2 ** 31 // nn, 2 ** 31 // (nn * elem_bytes), 2 ** 32 // (nn * elem_bytes)):
        marks += [e - 1, e, e + 1]
    marks = [m for m in marks if 0 <= m < B]
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, B, n), marks]))


def sample(T, N, idx):
    return T.view(-1, N, N)[torch.from_numpy(idx).cuda()].cpu().numpy()


def assert_u8_exact(pix, X64, W, border):
    _, u8, nh = oracle.filter_coeffs_to_pixels(X64, W, border)
    assert int((pix[~nh] != u8[~nh]).sum()) == 0
    assert np.abs(pix[nh].astype(int) - u8[nh].astype(int)).max(initial=0) <= 1


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,B", [(8, 2 ** 25 + 37), (16, 2 ** 23 + 5), (32, 2 ** 21 + 3)])
def test_filter_blocks_past_2_31(dctf, N, B, prec):
    W = syn.random_mask(np.random.default_rng(9), 5, 5)
    op = dctf.dctf_build_operator(W, N, R)
    X = big_coeffs(N, B, 51)
    assert X.numel() > 2 ** 31
    Y = torch.empty_like(X)
    idx = boundary_blocks(N * N, B, 4, 100 + N)
    ref = oracle.filter_coeffs(sample(X, N, idx), W, R)
    for v in range(dctf.dctf_variant_count(N, prec)):
        dctf.dctf_set_variant(N, prec, v)
        try:
            Y.fill_(float("nan"))
            dctf.dctf_filter_blocks(op, prec, X, Y)
            torch.cuda.synchronize()
            err = np.abs(sample(Y, N, idx) - ref).max()
            assert err <= TOL[prec], (dctf.dctf_variant_name(N, prec, v), err)
        finally:
            dctf.dctf_set_variant(N, prec, 0)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [16, 32])
def test_parity_classes_past_2_31(dctf, N, prec):
    """The parity-class filter (a mirror-symmetric 7x7 Gaussian) over more
    than 2^31 elements: the blocks on either side of each boundary and
    random ones against the oracle."""
    B = 2 ** 31 // (N * N) + 5
    W = syn.gaussian_mask(7, sigma=1.5)
    op = dctf.dctf_build_operator(W, N, R)
    assert dctf.dctf_operator_parity_classes(op) == 4
    X = big_coeffs(N, B, 53)
    assert X.numel() > 2 ** 31
    Y = torch.full_like(X, float("nan"))
    dctf.dctf_filter_blocks_parity(op, prec, X, Y)
    torch.cuda.synchronize()
    idx = boundary_blocks(N * N, B, 4, 117)
    err = np.abs(sample(Y, N, idx) - oracle.filter_coeffs(sample(X, N, idx), W, R)).max()
    assert err <= TOL[prec], err


def test_factored_past_2_31(dctf):
    N, B = 16, 2 ** 23 + 5
    W = syn.gaussian_mask(5)
    op = dctf.dctf_build_operator(W, N, R)
    X = big_coeffs(N, B, 52)
    Y = torch.full_like(X, float("nan"))
    dctf.dctf_filter_blocks_factored(op, X, Y)
    torch.cuda.synchronize()
    idx = boundary_blocks(N * N, B, 4, 7)
    assert np.abs(sample(Y, N, idx) - oracle.filter_coeffs(sample(X, N, idx), W, R)).max() <= TOL[FP32]


def test_fp64_past_2_31(dctf):
    N, B = 8, 2 ** 25 + 37
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_operator(W, N, Z)
    X = big_coeffs(N, B, 53).double()
    torch.cuda.empty_cache()
    Y = torch.full_like(X, float("nan"))
    dctf.dctf_filter_blocks_f64(op, X, Y)
    torch.cuda.synchronize()
    idx = boundary_blocks(N * N, B, 8, 8)
    assert np.abs(sample(Y, N, idx) - oracle.filter_coeffs(sample(X, N, idx), W, Z)).max() <= TOL_F64


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,B", [(8, 2 ** 25 + 37), (16, 2 ** 23 + 5)])
def test_pixels_past_2_31(dctf, N, B, prec):
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_operator(W, N, R)
    X = big_coeffs(N, B, 54)
    pix = torch.empty(X.numel(), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_blocks_u8(op, prec, X, pix)
    torch.cuda.synchronize()
    idx = boundary_blocks(N * N, B, 1, 9)
    assert_u8_exact(sample(pix, N, idx), sample(X, N, idx).astype(np.float64), W, R)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_quantized_pixels_past_2_31(dctf, prec):
    N, B = 8, 2 ** 25 + 37
    px = oracle.tile_u8(syn.image_u8(55, 512, 512), N)
    q = syn.quant_table(N)
    dc = 128.0 * N
    base = torch.from_numpy(np.ascontiguousarray(syn.quantize(oracle.dct_pixels(px), q, dc).reshape(-1, N * N)))
    h = position_hash(B)
    qc = base.cuda()[h % base.shape[0]]
    qc[:, 0] += ((h % 33) - 16).to(torch.int16)
    del h
    qc = qc.reshape(-1)
    W = syn.random_mask(np.random.default_rng(31), 5, 5, symmetric=True)
    op = dctf.dctf_build_operator(W, N, Z)
    pix = torch.empty(qc.numel(), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_quantized_u8(op, prec, qc, torch.from_numpy(q.astype(np.float32).reshape(-1)).cuda(), dc, pix)
    torch.cuda.synchronize()
    idx = boundary_blocks(N * N, B, 2, 10)
    assert_u8_exact(sample(pix, N, idx), oracle.dequantize(sample(qc, N, idx), q, dc), W, Z)


@pytest.mark.parametrize("N,B", [(8, 2 ** 25 + 37), (16, 2 ** 23 + 5), (32, 2 ** 21 + 3)])
def test_verify_past_2_31(dctf, N, B):
    """Pixels of sampled blocks against the oracle; then an expected image
    that differs in chosen pixels (all past the 2^31 boundary, none in the
    1/2 band) must give exactly that many mismatches."""
    Y = big_coeffs(N, B, 56)
    pix = torch.empty(Y.numel(), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    dctf.dctf_idct_u8_verify(N, Y, pix, None, cnt)
    torch.cuda.synchronize()
    assert int(cnt[0]) == 0
    idx = boundary_blocks(N * N, B, 1, 11)
    u8, nh = oracle.idct_u8(sample(Y, N, idx))
    got = sample(pix, N, idx)
    assert np.array_equal(got[~nh], u8[~nh])
    # plant differences at oracle-checked pixels outside the band, past 2^31
    flat = (idx[:, None] * N * N + np.arange(N * N)[None, :])[~nh.reshape(len(idx), -1)]
    flat = flat[flat >= 2 ** 31]
    chosen = np.random.default_rng(12).choice(flat, size=min(97, flat.size), replace=False)
    assert chosen.size > 50
    expected = pix.clone()
    ti = torch.from_numpy(chosen).cuda()
    expected[ti] = expected[ti] ^ 1
    cnt.zero_()
    pix2 = torch.empty_like(pix)
    dctf.dctf_idct_u8_verify(N, Y, pix2, expected, cnt)
    torch.cuda.synchronize()
    assert int(cnt[0]) == chosen.size
    assert torch.equal(pix2, pix)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_image_level_past_2_31(dctf, prec):
    """513 images of 256 x 256 blocks: image 256 starts at byte 2^32 and
    image 512 at element 2^31.  Windows around sampled interior blocks of
    the images on either side of those boundaries, and the corners of the
    last image, against the oracle."""
    N, Bh, Bw, nimg = 8, 256, 256, 513
    nb = Bh * Bw
    X = big_coeffs(N, nimg * nb, 57)
    Y = torch.full_like(X, float("nan"))
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_image_operator(W, N, R)
    dctf.dctf_filter_image(op, prec, X, Y, Bh, Bw)
    torch.cuda.synchronize()
    Xb = X.view(nimg, Bh, Bw, N, N)
    Yb = Y.view(nimg, Bh, Bw, N, N)
    rng = np.random.default_rng(13)
    worst = 0.0
    for img in (0, 255, 256, 511, 512):
        for _ in range(6):
            r, c = int(rng.integers(2, Bh - 2)), int(rng.integers(2, Bw - 2))
            win = Xb[img, r - 2:r + 3, c - 2:c + 3].cpu().numpy().astype(np.float64).reshape(-1, N, N)
            ref = oracle.filter_image_coeffs(win, 5, 5, W, R).reshape(5, 5, N, N)[2, 2]
            worst = max(worst, np.abs(Yb[img, r, c].cpu().numpy() - ref).max())
    full = oracle.filter_image_coeffs(Xb[nimg - 1].cpu().numpy().astype(np.float64).reshape(-1, N, N), Bh, Bw,
                                      W, R).reshape(Bh, Bw, N, N)
    got = Yb[nimg - 1].cpu().numpy()
    for r, c in ((0, 0), (0, Bw - 1), (Bh - 1, 0), (Bh - 1, Bw - 1), (0, 100), (Bh - 1, 7), (50, 0),
                 (200, Bw - 1)):
        worst = max(worst, np.abs(got[r, c] - full[r, c]).max())
    assert worst <= TOL[prec], worst


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("layout", ["n8", "n16", "mixed"])
def test_batch_past_2_31(dctf, layout, prec):
    """The persistent batch kernels with a job of more than 2^31 elements:
    N = 8 alone, N = 16 alone, and an N = 8 one behind a small N = 16 job."""
    W8 = syn.random_mask(np.random.default_rng(14), 5, 5)
    W16 = syn.gaussian_mask(7)
    op8 = dctf.dctf_build_operator(W8, 8, R)
    op16 = dctf.dctf_build_operator(W16, 16, Z)
    jobs, checks = [], []
    if layout in ("n16", "mixed"):
        B16 = 2 ** 23 + 5 if layout == "n16" else 3001
        X16 = big_coeffs(16, B16, 58)
        Y16 = torch.full_like(X16, float("nan"))
        jobs.append((op16, X16, Y16))
        checks.append((X16, Y16, 16, B16, W16, Z))
    if layout in ("n8", "mixed"):
        B8 = 2 ** 25 + 37
        X8 = big_coeffs(8, B8, 59)
        Y8 = torch.full_like(X8, float("nan"))
        jobs.append((op8, X8, Y8))
        checks.append((X8, Y8, 8, B8, W8, R))
    dctf.dctf_filter_batch(jobs, prec)
    torch.cuda.synchronize()
    for X, Y, N, B, W, border in checks:
        idx = boundary_blocks(N * N, B, 4, 15 + N)
        err = np.abs(sample(Y, N, idx) - oracle.filter_coeffs(sample(X, N, idx), W, border)).max()
        assert err <= TOL[prec], (layout, N, err)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("h,w,pitch,nimg", [(4096, 4096, 4096, 130), (4093, 4094, 4096, 129)])
def test_u8_raster_past_2_31(dctf, h, w, pitch, nimg, prec):
    """uint8 images to filtered uint8 images in one pass, the images spanning
    more than 2^31 bytes (the kernel's 64-bit address path): bit-identical to
    calls over parts of fewer than 2^31 bytes (its 32-bit buffer path), and
    equal to the oracle on sampled blocks, among them the blocks that hold
    byte 2^31 of the input and of the output, outside the 1/2 band."""
    N = 8
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_operator(W, N, R)
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    src = torch.randint(0, 256, (nimg, h, pitch), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros((nimg, h, pitch), dtype=torch.uint8, device="cuda")
    dctf.dctf_filter_u8_raster(op, prec, src[:, :, :w], h, w, dst[:, :, :w])
    part = torch.zeros((64, h, pitch), dtype=torch.uint8, device="cuda")
    for i0 in range(0, nimg, 64):
        n = min(64, nimg - i0)
        dctf.dctf_filter_u8_raster(op, prec, src[i0:i0 + n, :, :w], h, w, part[:n, :, :w])
        torch.cuda.synchronize()
        assert torch.equal(part[:n, :, :w], dst[i0:i0 + n, :, :w]), i0
    del part
    bh, bw = -(-h // N), -(-w // N)
    at = divmod(2 ** 31, h * pitch)
    mark = (at[0], at[1] // pitch // N, min(at[1] % pitch, w - 1) // N)
    rng = np.random.default_rng(7)
    blocks = {mark, (nimg - 1, bh - 1, bw - 1), (0, 0, 0)}
    blocks |= {(int(rng.integers(nimg)), int(rng.integers(bh)), int(rng.integers(bw))) for _ in range(300)}
    blocks = sorted(blocks)
    r = np.arange(N)
    px, got, valid = [], [], []
    for (i, by, bx) in blocks:
        ys, xs = np.minimum(N * by + r, h - 1), np.minimum(N * bx + r, w - 1)
        yi = torch.from_numpy(ys).cuda()[:, None]
        xi = torch.from_numpy(xs).cuda()[None, :]
        px.append(src[i][yi, xi].cpu().numpy())
        got.append(dst[i][yi, xi].cpu().numpy())
        valid.append(((N * by + r) < h)[:, None] & ((N * bx + r) < w)[None, :])
    _, u8, nh = oracle.filter_pixels(np.stack(px), W, R)
    got, valid = np.stack(got), np.stack(valid)
    assert np.array_equal(got[valid & ~nh], u8[valid & ~nh])
    assert np.abs(got[valid & nh].astype(int) - u8[valid & nh].astype(int)).max(initial=0) <= 1
