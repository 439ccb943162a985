"""GPU parity of the builder and the single-operator filter against the FP64 oracle.

Tolerances (absolute, per coefficient): FP32 path 2e-3, split-BF16 path 5e-3.
Pixels after the inverse DCT must round to the oracle's uint8 exactly,
except pixels within 1e-3 of a .5 boundary (counted separately).
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_filter(dctf, op, X32, prec):
    X = dev(X32.reshape(-1))
    Y = torch.empty_like(X)
    dctf.dctf_filter_blocks(op, prec, X, Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy().reshape(X32.shape)


def gpu_u8(dctf, N, Y32, expected=None):
    Y = dev(Y32.reshape(-1))
    pix = torch.empty(Y.numel(), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    exp = dev(expected.reshape(-1)) if expected is not None else None
    dctf.dctf_idct_u8_verify(N, Y, pix, exp, cnt)
    torch.cuda.synchronize()
    return pix.cpu().numpy().reshape(Y32.shape), cnt.cpu().numpy()


def image_case(seed, h, w, N):
    px = oracle.tile_u8(syn.image_u8(seed, h, w), N)
    return px, oracle.coeffs_fp32(px)


# ------------------------------------------------------------------ builder

BUILD_CASES = []
for N in (2, 4, 8, 16):
    for kh, kw in [(1, 1), (3, 3), (5, 5), (1, 5), (5, 1), (4, 4), (2, 3), (7, 7),
                   (2 * N + 1, 2 * N + 1)]:
        if kh <= 2 * N + 1 and kw <= 2 * N + 1:
            BUILD_CASES.append((N, kh, kw))


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N,kh,kw", BUILD_CASES)
def test_builder_matches_oracle_probe(dctf, N, kh, kw, border):
    rng = np.random.default_rng(1000 * N + 10 * kh + kw)
    W = rng.uniform(-1, 1, size=(kh, kw))
    op = dctf.dctf_build_operator(W, N, border)
    H = dctf.dctf_operator_fp64(op)
    ref = oracle.operator_probe(N, W, border)
    assert np.abs(H - ref).max() <= 1e-12


def test_builder_identity_and_constant(dctf):
    for N in (2, 4, 8, 16):
        for border in (Z, R):
            H = dctf.dctf_operator_fp64(dctf.dctf_build_operator(syn.delta_mask(5, 5), N, border))
            assert np.abs(H - np.eye(N * N)).max() <= 1e-14
        W = syn.random_mask(np.random.default_rng(N), 5, 5)
        H = dctf.dctf_operator_fp64(dctf.dctf_build_operator(W, N, R))
        e0 = np.zeros(N * N)
        e0[0] = 1
        assert np.abs(H[:, 0] - e0).max() <= 1e-13


def test_build_operators_one_launch_equals_single(dctf):
    rng = np.random.default_rng(7)
    specs = [(rng.uniform(-1, 1, (k, k)), N, b) for k in (3, 5, 7) for N in (8, 16) for b in (Z, R)]
    specs += [(rng.uniform(-1, 1, (3, 3)), 4, Z)] * 12   # more than one launch (16 per launch)
    many = dctf.dctf_build_operators(specs)
    for op, (W, N, b) in zip(many, specs):
        single = dctf.dctf_build_operator(W, N, b)
        assert np.array_equal(dctf.dctf_operator_fp64(op), dctf.dctf_operator_fp64(single))
    dctf.dctf_rebuild_operators(many)
    torch.cuda.synchronize()
    for op, (W, N, b) in zip(many, specs):
        assert np.abs(dctf.dctf_operator_fp64(op) - oracle.operator_probe(N, W, b)).max() <= 1e-12


# ------------------------------------------------------------------- filter

def check_case(dctf, px, X32, W, border, N, prec, check_u8=True):
    op = dctf.dctf_build_operator(W, N, border)
    Y = gpu_filter(dctf, op, X32, prec)
    Yref, u8ref, nh = oracle.filter_pixels(px, W, border)
    err = np.abs(Y.astype(np.float64) - Yref).max()
    assert err <= TOL[prec], (N, border, prec, err)
    if check_u8:
        pix, cnt = gpu_u8(dctf, N, Y, u8ref)
        outside = ~nh
        assert np.array_equal(pix[outside], u8ref[outside])
        assert cnt[0] == 0
    return err


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_small_image_box3_zero(dctf, prec):
    # 64 x 64 image, 3 x 3 box, zero padding, 8 x 8 blocks (64 blocks)
    px, X = image_case(0, 64, 64, 8)
    check_case(dctf, px, X, syn.box_mask(3), Z, 8, prec)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("mask", ["gauss3", "asym5"])
def test_512_image_two_masks_two_borders(dctf, mask, border, prec):
    # 512 x 512 image (4096 blocks), Gaussian 3 x 3 sigma 1 and a 5 x 5
    # asymmetric inseparable sum-1 mask, zero padding and replication
    px, X = image_case(1, 512, 512, 8)
    W = syn.gaussian_mask(3, 1.0) if mask == "gauss3" else syn.asym_mask_5x5()
    check_case(dctf, px, X, W, border, 8, prec)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("border", [Z, R])
def test_n16_asym7(dctf, border, prec):
    # 16 x 16 blocks of a 520 x 344 image (ragged sides padded by replication)
    px, X = image_case(2, 344, 520, 16)
    W = syn.random_mask(np.random.default_rng(4), 7, 7)
    check_case(dctf, px, X, W, border, 16, prec)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [2, 4])
def test_small_block_sizes(dctf, N, prec):
    px, X = image_case(3, 96, 88, N)
    W = syn.random_mask(np.random.default_rng(N), 3, 5)
    check_case(dctf, px, X, W, R, N, prec)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_magic_square_replicate(dctf, prec):
    px, X = image_case(5, 128, 128, 8)
    check_case(dctf, px, X, syn.magic_square_3(True), R, 8, prec)
    # raw magic square (sum 45): coefficients grow 45x, compare relatively
    op = dctf.dctf_build_operator(syn.magic_square_3(False), 8, R)
    Y = gpu_filter(dctf, op, X, prec)
    Yref, _, _ = oracle.filter_pixels(px, syn.magic_square_3(False), R)
    assert np.abs(Y - Yref).max() <= 45 * TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N", [8, 16])
def test_ragged_counts_are_prefix_identical(dctf, N, prec):
    """A block's result does not depend on B, the tile it falls in or the
    variant: every prefix run is bit-identical to the long run."""
    px, X = image_case(6, 16 * N, 17 * N, N)
    X = X[:257]
    W = syn.random_mask(np.random.default_rng(9), 5, 5)
    op = dctf.dctf_build_operator(W, N, Z)
    full = gpu_filter(dctf, op, X, prec)
    Yref, _, _ = oracle.filter_pixels(px[:257], W, Z)
    assert np.abs(full - Yref).max() <= TOL[prec]
    for B in (1, 15, 16, 17, 31, 32, 33, 63, 100, 255):
        assert np.array_equal(gpu_filter(dctf, op, X[:B], prec), full[:B]), B
    for v in range(dctf.dctf_variant_count(N, prec)):
        dctf.dctf_set_variant(N, prec, v)
        try:
            assert np.array_equal(gpu_filter(dctf, op, X, prec), full), dctf.dctf_variant_name(N, prec, v)
            assert np.array_equal(gpu_filter(dctf, op, X[:33], prec), full[:33])
        finally:
            dctf.dctf_set_variant(N, prec, 0)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("N,k", [(8, 5), (8, 7), (16, 7), (16, 9)])
def test_precision_over_random_masks(dctf, N, k, prec):
    """Sum-1 masks with entries U(-1, 1) (largest operator entries near 1),
    both borders: every coefficient within the tolerance of its path."""
    px, X = image_case(10 + N, 16 * N, 16 * N, N)
    rng = np.random.default_rng(100 * N + k)
    worst = 0.0
    for trial in range(6):
        W = syn.random_mask(rng, k, k, symmetric=(trial % 3 == 2))
        for border in (Z, R):
            worst = max(worst, check_case(dctf, px, X, W, border, N, prec, check_u8=False))
    print("N=%d k=%d prec=%d worst=%.3e" % (N, k, prec, worst))


def test_zero_blocks_is_noop(dctf):
    op = dctf.dctf_build_operator(syn.box_mask(3), 8, Z)
    X = torch.empty(0, dtype=torch.float32, device="cuda")
    Y = torch.empty(0, dtype=torch.float32, device="cuda")
    dctf.dctf_filter_blocks(op, SPLIT, X, Y)
    torch.cuda.synchronize()


def test_device_argument_errors(dctf):
    op = dctf.dctf_build_operator(syn.box_mask(3), 8, Z)
    X = torch.zeros(64 * 10 + 4, dtype=torch.float32, device="cuda")
    Y = torch.zeros(64 * 10 + 4, dtype=torch.float32, device="cuda")
    with pytest.raises(dctf.DctfError) as e:          # misaligned by 4 bytes
        dctf.dctf_filter_blocks(op, FP32, X[1:641], Y[:640])
    assert e.value.status == dctf.DCTF_EINVAL
    with pytest.raises(dctf.DctfError):               # in and out overlap
        dctf.dctf_filter_blocks(op, FP32, X[:576], X[64:640])
    with pytest.raises(dctf.DctfError):               # unknown precision
        dctf.dctf_filter_blocks(op, 5, X[:640], Y[:640])


# ------------------------------------------------------- around the path

@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_forward_dct_matches_oracle(dctf, N):
    img = syn.image_u8(8, 100, 75)   # ragged for every N but 2 and 4 (rows)
    X = torch.empty(-(-100 // N) * -(-75 // N) * N * N, dtype=torch.float32, device="cuda")
    dctf.dctf_forward_dct_u8(dev(img), N, X)
    torch.cuda.synchronize()
    ref = oracle.coeffs_fp32(oracle.tile_u8(img, N)).reshape(-1)
    got = X.cpu().numpy()
    diff = np.abs(got.astype(np.float64) - ref)
    # both sides round an FP64 sum once to FP32; only the summation order differs
    assert diff.max() <= 4 * np.spacing(np.float32(255 * N))
    big = np.abs(ref) > 1e-3
    assert np.all(diff[big] <= 2 * np.spacing(np.abs(ref[big]).astype(np.float32)))


def test_forward_dct_rejects_unusable_views(dctf):
    img = dev(syn.image_u8(5, 64, 48))
    X = torch.empty(64 * 48, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        dctf.dctf_forward_dct_u8(img.t(), 8, X)          # columns as rows: not contiguous
    with pytest.raises(ValueError):
        dctf.dctf_forward_dct_u8(img.reshape(-1), 8, X)  # not 2-D
    with pytest.raises(ValueError):
        dctf.dctf_forward_dct_u8(img, 8, X[:64])          # wrong coefficient count


def test_forward_dct_large_image(dctf):
    """An image large enough for the N = 8 forward DCT's long-step launch
    (6144 x 6144: 147,456 units of 2 x 2 blocks), every block against the
    oracle."""
    N, side = 8, 6144
    img = syn.image_u8(31, side, side)
    X = torch.full(((side // N) ** 2 * N * N,), float("nan"), dtype=torch.float32, device="cuda")
    dctf.dctf_forward_dct_u8(dev(img), N, X)
    torch.cuda.synchronize()
    ref = oracle.coeffs_fp32(oracle.tile_u8(img, N)).reshape(-1)
    got = X.cpu().numpy()
    diff = np.abs(got.astype(np.float64) - ref)
    assert diff.max() <= 4 * np.spacing(np.float32(255 * N))
    big = np.abs(ref) > 1e-3
    assert np.all(diff[big] <= 2 * np.spacing(np.abs(ref[big]).astype(np.float32)))


@pytest.mark.parametrize("pad", [37, 40])
@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("h,w", [(1000, 1496), (1016, 1000), (17, 9), (1, 1)])
def test_forward_dct_strided_image(dctf, N, h, w, pad):
    """Images held as a view of a wider buffer (row pitch w + pad: odd, or a
    multiple of 4 where w is, so that units inside the image take the 32-bit
    pixel loads), block counts odd and even in both directions, sides not
    multiples of N, and a single pixel: every block against the oracle."""
    img = syn.image_u8(20 + N, h, w)
    pitch = w + pad
    buf = torch.zeros((h, pitch), dtype=torch.uint8, device="cuda")
    buf[:, :w] = dev(img)
    view = buf[:, :w]
    nb = -(-h // N) * -(-w // N)
    X = torch.full((nb * N * N,), float("nan"), dtype=torch.float32, device="cuda")
    dctf.dctf_forward_dct_u8(view, N, X)
    torch.cuda.synchronize()
    ref = oracle.coeffs_fp32(oracle.tile_u8(img, N)).reshape(-1)
    got = X.cpu().numpy()
    diff = np.abs(got.astype(np.float64) - ref)
    assert diff.max() <= 4 * np.spacing(np.float32(255 * N))
    big = np.abs(ref) > 1e-3
    assert np.all(diff[big] <= 2 * np.spacing(np.abs(ref[big]).astype(np.float32)))


@pytest.mark.parametrize("N,h,w,n,pad", [(8, 130, 204, 5, 40), (8, 64, 64, 700, 0), (16, 100, 75, 9, 13),
                                          (32, 70, 97, 4, 3), (4, 33, 20, 6, 0), (8, 1, 1, 3, 0),
                                          (8, 64, 64, 5, -1)])
def test_forward_dct_many_images_in_one_call(dctf, N, h, w, n, pad):
    """n images in one launch (image stride with padding rows, odd and even
    block counts, ragged sides, many units across image boundaries; pad -1:
    aligned rows but an image stride that is not a multiple of 4):
    bit-identical to one call per image, and every block of the first and
    last images against the oracle."""
    imgs = np.stack([syn.image_u8(600 + i, h, w) for i in range(n)])
    if pad < 0:
        # images h * w + 1 bytes apart: the pixel rows of images 1.. are not 4-byte aligned
        flat = torch.zeros(n * (h * w + 1), dtype=torch.uint8, device="cuda")
        view = torch.as_strided(flat, (n, h, w), (h * w + 1, w, 1))
        view.copy_(dev(imgs))
    else:
        rows = h + (1 if pad else 0)
        buf = torch.zeros((n, rows, w + pad), dtype=torch.uint8, device="cuda")
        buf[:, :h, :w] = dev(imgs)
        view = buf[:, :h, :w]
    nb = -(-h // N) * -(-w // N)
    X = torch.full((n * nb * N * N,), float("nan"), dtype=torch.float32, device="cuda")
    dctf.dctf_forward_dct_u8_images(view, N, X)
    one = torch.empty(nb * N * N, dtype=torch.float32, device="cuda")
    for i in range(n):
        dctf.dctf_forward_dct_u8(view[i], N, one)
        torch.cuda.synchronize()
        assert torch.equal(X[i * nb * N * N:(i + 1) * nb * N * N], one), i
    for i in (0, n - 1):
        ref = oracle.coeffs_fp32(oracle.tile_u8(imgs[i], N)).reshape(-1)
        got = X[i * nb * N * N:(i + 1) * nb * N * N].cpu().numpy()
        assert np.abs(got.astype(np.float64) - ref).max() <= 4 * np.spacing(np.float32(255 * N))


def test_forward_dct_many_images_argument_errors(dctf):
    lib = dctf.raw_library()
    img = torch.zeros(4 * 64 * 64, dtype=torch.uint8, device="cuda")
    X = torch.zeros(4 * 64 * 64, dtype=torch.float32, device="cuda")
    f = lib.dctf_forward_dct_u8_images
    pi, px = img.data_ptr(), X.data_ptr()
    assert f(pi, 64, 64, 64, 4096, 4, 8, px, None) == 0
    assert f(pi, 64, 64, 64, 4000, 4, 8, px, None) == -1       # images overlap
    assert f(pi, 64, 64, 60, 4096, 4, 8, px, None) == -1       # pitch < w
    assert f(pi, 64, 64, 64, 4096, -1, 8, px, None) == -1      # nimg < 0
    assert f(pi, 64, 64, 64, 4096, 0, 8, px, None) == 0        # no-op
    assert f(pi, 64, 64, 64, 4096, 4, 8, px + 4, None) == -1   # alignment
    assert f(pi, 64, 64, 64, 4096, 4, 8, pi, None) == -1       # images overlap the coefficients
    assert f(pi, 64, 64, 64, 4096, 4, 5, px, None) == -2       # block size


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_verify_kernel_all_sizes_strided(dctf, N):
    """Every block size, with enough blocks that each workgroup walks several
    steps and a ragged last one, through byte buffers at odd and at aligned
    addresses (both must give the same pixels)."""
    per_step = 256 // (N * N // min(N, 4))
    B = 3 * 2048 * per_step + per_step // 2 + 1
    rng = np.random.default_rng(100 + N)
    Y = (rng.standard_normal((B, N, N)) * 40).astype(np.float32)
    Y[:, 0, 0] += np.float32(128 * N)          # pixel values around mid-grey, some clipped
    u8ref, nh = oracle.idct_u8(Y)
    Yd = dev(Y.reshape(-1))
    outs = []
    for shift in (1, 0):
        raw = torch.zeros(Y.size + 4, dtype=torch.uint8, device="cuda")
        pix = raw[shift:shift + Y.size]
        eraw = torch.zeros(Y.size + 4, dtype=torch.uint8, device="cuda")
        exp = eraw[shift:shift + Y.size]
        exp.copy_(torch.from_numpy(u8ref.reshape(-1)).cuda())
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        dctf.dctf_idct_u8_verify(N, Yd, pix, exp, cnt)
        torch.cuda.synchronize()
        got = pix.cpu().numpy().reshape(Y.shape)
        assert np.array_equal(got[~nh], u8ref[~nh]), (N, shift)
        assert int(cnt[0]) == 0
        assert abs(int(cnt[1]) - int(nh.sum())) <= max(3, int(nh.sum()) // 50)
        assert int(raw[shift + Y.size:].sum()) == 0 and int(raw[:shift].sum()) == 0   # nothing past the ends
        outs.append(got)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("B", [1, 63, 64, 65, 4097, 98313])
def test_verify_kernel_without_counters_same_pixels(dctf, B):
    """A call without counters (the N = 8 kernel then skips the near-1/2 and
    mismatch tests) writes the same pixels as one with counters, and those
    match the oracle outside the 1/2 band."""
    N = 8
    rng = np.random.default_rng(B)
    Y = (rng.standard_normal((B, N, N)) * 40).astype(np.float32)
    Y[:, 0, 0] += np.float32(128 * N)
    Yd = dev(Y.reshape(-1))
    a = torch.zeros(Y.size, dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    dctf.dctf_idct_u8_verify(N, Yd, a, None, cnt)
    dctf.dctf_idct_u8_verify(N, Yd, b, None, None)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    u8ref, nh = oracle.idct_u8(Y)
    got = b.cpu().numpy().reshape(Y.shape)
    assert np.array_equal(got[~nh], u8ref[~nh])


def test_verify_kernel_counts(dctf):
    N = 8
    px = oracle.tile_u8(syn.image_u8(9, 256, 256), N)
    W = syn.gaussian_mask(3, 1.0)
    Yref, u8ref, nh = oracle.filter_pixels(px, W, R)
    pix, cnt = gpu_u8(dctf, N, Yref.astype(np.float32), u8ref)
    assert cnt[0] == 0
    assert np.array_equal(pix[~nh], u8ref[~nh])
    assert abs(int(cnt[1]) - int(nh.sum())) <= max(3, nh.sum() // 50)
    # a planted difference in the expected pixels is counted (outside the band)
    exp = u8ref.copy()
    flip = np.argwhere(~nh.reshape(-1))[:5, 0]
    exp.reshape(-1)[flip] ^= 1
    _, cnt2 = gpu_u8(dctf, N, Yref.astype(np.float32), exp)
    assert cnt2[0] == 5


@pytest.mark.parametrize("N,prec", [(8, FP32), (8, SPLIT), (16, FP32), (16, SPLIT)])
def test_every_variant_over_many_steps_per_wave(dctf, N, prec):
    """An input long enough that every wave of every variant runs its loop
    for several steps (the prefix tests above stay within a step or two):
    every variant bit-identical to variant 0, and variant 0 against the
    oracle on sampled outputs."""
    B = 1500037 if N == 8 else 400021
    rng = np.random.default_rng(57)
    W = syn.random_mask(rng, 5, 5)
    op = dctf.dctf_build_operator(W, N, R)
    # seeded coefficients whose spread falls with frequency as in natural
    # images (the content the split-BF16 bound is stated for), DC near 128 N
    gen = torch.Generator(device="cuda").manual_seed(57)
    u = torch.arange(N, device="cuda", dtype=torch.float32)
    decay = (40.0 / (1.0 + u.view(N, 1) + u.view(1, N))).reshape(-1)
    X = (torch.randn(B, N * N, device="cuda", generator=gen) * decay).reshape(-1)
    X.view(B, N * N)[:, 0] += 128.0 * N
    v0 = dctf.dctf_get_variant(N, prec)
    try:
        dctf.dctf_set_variant(N, prec, 0)
        ref = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, ref)
        torch.cuda.synchronize()
        bi = rng.integers(0, B, 3000)
        ci = rng.integers(0, N * N, 3000)
        want = oracle.filter_coeffs_sampled(X.view(B, N * N)[torch.from_numpy(bi).cuda()].cpu().numpy(),
                                            W, R, np.arange(3000), ci)
        got = ref.view(B, N * N)[torch.from_numpy(bi).cuda(), torch.from_numpy(ci).cuda()].cpu().numpy()
        assert np.abs(got - want).max() <= TOL[prec]
        for v in range(1, dctf.dctf_variant_count(N, prec)):
            dctf.dctf_set_variant(N, prec, v)
            Y = torch.full_like(X, float("nan"))
            dctf.dctf_filter_blocks(op, prec, X, Y)
            torch.cuda.synchronize()
            assert torch.equal(Y, ref), dctf.dctf_variant_name(N, prec, v)
    finally:
        dctf.dctf_set_variant(N, prec, v0)
