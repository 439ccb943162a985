"""GPU parity of image-level (cross-block) filtering in the DCT domain
against the FP64 oracle.

The builder's FP64 neighbour operators must match the oracle's probes (a
small image whose only non-zero block is e_k) to 1e-12 for every class pair
and offset; the filter must match the oracle's whole-image filter to 2e-3
(FP32) or 5e-3 (split-BF16) per coefficient, on images whose sides exercise
every class (one block, two blocks, many blocks, ragged tile counts).
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


# Bh (or Bw) and the block row of that axis that has the class:
# 0 interior (3 rows, middle), 1 first (2 rows, row 0), 2 last (2 rows, row 1), 3 both (1 row)
CLASS_AXIS = {0: (3, 1), 1: (2, 0), 2: (2, 1), 3: (1, 0)}


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("kh,kw", [(5, 5), (3, 7), (1, 5), (2, 4), (17, 17)])
def test_image_operators_match_oracle_probes(dctf, kh, kw, border):
    N = 8
    W = np.random.default_rng(kh * 31 + kw).uniform(-1, 1, size=(kh, kw))
    op = dctf.dctf_build_image_operator(W, N, border)
    worst = 0.0
    for rc in range(4):
        for cc in range(4):
            Bh, Rr = CLASS_AXIS[rc]
            Bw, Sc = CLASS_AXIS[cc]
            for dr in (-1, 0, 1):
                for ds in (-1, 0, 1):
                    H = dctf.dctf_image_operator_fp64(op, rc, cc, dr, ds)
                    ref = oracle.image_operator_probe(N, W, border, Bh, Bw, Rr, Sc, dr, ds)
                    worst = max(worst, np.abs(H - ref).max())
    assert worst <= 1e-12, worst


def image_blocks(seed, Bh, Bw, nimg=1, N=8):
    out = []
    for i in range(nimg):
        px = oracle.tile_u8(syn.image_u8(seed + i, Bh * N, Bw * N), N)
        out.append(oracle.coeffs_fp32(px))
    return np.concatenate(out)


def gpu_image(dctf, op, X32, Bh, Bw, prec=FP32):
    X = dev(X32.reshape(-1))
    Y = torch.empty_like(X)
    dctf.dctf_filter_image(op, prec, X, Y, Bh, Bw)
    torch.cuda.synchronize()
    return Y.cpu().numpy().reshape(X32.shape)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("Bh,Bw,nimg,mask", [
    (8, 8, 1, "box3"), (64, 64, 1, "asym5"), (1, 1, 3, "asym5"), (1, 37, 2, "rand7"), (37, 1, 2, "rand7"),
    (2, 2, 1, "rand9"), (2, 19, 1, "gauss3"), (33, 18, 2, "asym5"), (5, 40, 1, "rand17"), (3, 3, 4, "h1x5"),
])
def test_image_filter_matches_oracle(dctf, Bh, Bw, nimg, mask, border, prec):
    W = {"box3": syn.box_mask(3), "asym5": syn.asym_mask_5x5(), "gauss3": syn.gaussian_mask(3),
         "rand7": syn.random_mask(np.random.default_rng(4), 7, 7),
         "rand9": syn.random_mask(np.random.default_rng(5), 9, 9),
         "rand17": syn.random_mask(np.random.default_rng(6), 17, 17),
         "h1x5": syn.random_mask(np.random.default_rng(7), 1, 5)}[mask]
    X = image_blocks(40 + Bh + Bw, Bh, Bw, nimg)
    op = dctf.dctf_build_image_operator(W, 8, border)
    Y = gpu_image(dctf, op, X, Bh, Bw, prec)
    Yref = oracle.filter_image_coeffs(X.astype(np.float64), Bh, Bw, W, border)
    err = np.abs(Y.astype(np.float64) - Yref).max()
    assert err <= TOL[prec], err
    # each image's result is the same alone and in the batch
    if nimg > 1:
        per = Bh * Bw
        for i in range(nimg):
            assert np.array_equal(gpu_image(dctf, op, X[i * per:(i + 1) * per], Bh, Bw, prec),
                                  Y[i * per:(i + 1) * per])


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_image_filter_uint8_after_inverse_dct(dctf, prec):
    """Pixels of the image-level result round to the oracle's uint8 (outside
    the 1/2 band), via the library's verify kernel."""
    Bh, Bw, N = 40, 48, 8
    X = image_blocks(90, Bh, Bw)
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_image_operator(W, N, R)
    Y = gpu_image(dctf, op, X, Bh, Bw, prec)
    Yref = oracle.filter_image_coeffs(X.astype(np.float64), Bh, Bw, W, R)
    u8ref, nh = oracle.idct_u8(Yref)
    pix = torch.empty(Y.size, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    dctf.dctf_idct_u8_verify(N, dev(Y.reshape(-1)), pix, dev(u8ref.reshape(-1)), cnt)
    torch.cuda.synchronize()
    got = pix.cpu().numpy().reshape(u8ref.shape)
    assert np.array_equal(got[~nh], u8ref[~nh])


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_full_size_sampled(dctf, prec):
    """64 images of 2048 x 2048 (4,194,304 blocks) in one launch: sampled
    blocks against the oracle's whole-image filter of a window around them
    (a 5 x 5-block window, filtered as its own image, gives the interior
    block's exact result for a mask that reaches at most one block)."""
    N, side, nimg = 8, 2048, 64
    Bh = Bw = side // N
    nb = Bh * Bw
    X = torch.empty(nimg * nb * N * N, dtype=torch.float32, device="cuda")
    for i in range(nimg):
        dctf.dctf_forward_dct_u8(torch.from_numpy(syn.image_u8(1000 + i, side, side)).cuda(), N,
                                 X[i * nb * N * N:(i + 1) * nb * N * N])
    W = syn.asym_mask_5x5()
    op = dctf.dctf_build_image_operator(W, N, R)
    Y = torch.empty_like(X)
    dctf.dctf_filter_image(op, prec, X, Y, Bh, Bw)
    torch.cuda.synchronize()
    Xb = X.view(nimg, Bh, Bw, N, N)
    Yb = Y.view(nimg, Bh, Bw, N, N)
    rng = np.random.default_rng(5)
    worst = 0.0
    picks = [(int(rng.integers(nimg)), int(rng.integers(2, Bh - 2)), int(rng.integers(2, Bw - 2)))
             for _ in range(40)]
    for img, r, c in picks:
        win = Xb[img, r - 2:r + 3, c - 2:c + 3].cpu().numpy().astype(np.float64).reshape(-1, N, N)
        ref = oracle.filter_image_coeffs(win, 5, 5, W, R).reshape(5, 5, N, N)[2, 2]
        worst = max(worst, np.abs(Yb[img, r, c].cpu().numpy() - ref).max())
    # corners and edges of the first and last image against the whole-image oracle
    for img in (0, nimg - 1):
        full = oracle.filter_image_coeffs(Xb[img].cpu().numpy().astype(np.float64).reshape(-1, N, N), Bh, Bw,
                                          W, R).reshape(Bh, Bw, N, N)
        got = Yb[img].cpu().numpy()
        for r, c in ((0, 0), (0, Bw - 1), (Bh - 1, 0), (Bh - 1, Bw - 1), (0, 100), (Bh - 1, 7), (50, 0),
                     (200, Bw - 1)):
            worst = max(worst, np.abs(got[r, c] - full[r, c]).max())
    assert worst <= TOL[prec], worst
    del X, Y
    torch.cuda.empty_cache()


def test_image_filter_argument_errors(dctf):
    op = dctf.dctf_build_image_operator(syn.box_mask(3), 8, Z)
    lib = dctf.raw_library()
    X = torch.zeros(64 * 4, dtype=torch.float32, device="cuda")
    Y = torch.zeros(64 * 4, dtype=torch.float32, device="cuda")
    assert lib.dctf_filter_image(op.handle, 2, X.data_ptr(), Y.data_ptr(), 2, 2, 1, None) == -1
    assert lib.dctf_filter_image(op.handle, FP32, X.data_ptr(), Y.data_ptr(), 0, 2, 1, None) == -1
    assert lib.dctf_filter_image(op.handle, FP32, X.data_ptr(), Y.data_ptr(), 2, 2, -1, None) == -1
    assert lib.dctf_filter_image(op.handle, FP32, X.data_ptr(), X.data_ptr() + 256, 2, 2, 1, None) == -1
    assert lib.dctf_filter_image(op.handle, FP32, X.data_ptr(), Y.data_ptr(), 2, 2, 0, None) == 0
    assert lib.dctf_image_operator_fp64(op.handle, 4, 0, 0, 0, None) == -1


# ---------------------------------------------------------------- N = 16

def _mask16(name):
    rng = np.random.default_rng(sum(map(ord, name)))
    return {"box3": syn.box_mask(3), "asym5": syn.asym_mask_5x5(), "rand7": syn.random_mask(rng, 7, 7),
            "rand3x5": syn.random_mask(rng, 3, 5), "gauss33": syn.gaussian_mask(33, sigma=8.0),
            "rand17": syn.random_mask(rng, 17, 17), "h1x9": syn.random_mask(rng, 1, 9)}[name]


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("mask,pairs", [
    ("rand7", "all"), ("rand3x5", "all"),
    # the largest mask (reaches every row of each neighbour), interior class pair
    ("gauss33", "interior"),
])
def test_image_operators_n16_match_oracle_probes(dctf, mask, pairs, border):
    N = 16
    W = _mask16(mask)
    op = dctf.dctf_build_image_operator(W, N, border)
    cps = [(rc, cc) for rc in range(4) for cc in range(4)] if pairs == "all" else [(0, 0)]
    worst = 0.0
    for rc, cc in cps:
        Bh, Rr = CLASS_AXIS[rc]
        Bw, Sc = CLASS_AXIS[cc]
        for dr in (-1, 0, 1):
            for ds in (-1, 0, 1):
                H = dctf.dctf_image_operator_fp64(op, rc, cc, dr, ds)
                ref = oracle.image_operator_probe(N, W, border, Bh, Bw, Rr, Sc, dr, ds)
                worst = max(worst, np.abs(H - ref).max())
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("prec", [FP32, SPLIT])
@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("Bh,Bw,nimg,mask", [
    (8, 8, 1, "box3"), (20, 33, 1, "rand7"), (1, 1, 3, "asym5"), (1, 37, 2, "rand7"), (37, 1, 2, "rand7"),
    (2, 2, 1, "rand17"), (3, 18, 2, "asym5"), (6, 21, 1, "gauss33"), (4, 35, 1, "h1x9"),
])
def test_image_filter_n16_matches_oracle(dctf, Bh, Bw, nimg, mask, border, prec):
    """Image-level filtering of 16 x 16 blocks against the oracle's whole-image
    filter: every class (one block, two, many), row and column tiles, ragged
    tile counts (33 - 2 interior blocks: a tile of 16 and one of 15), masks up
    to the largest (33 x 33), and each image of a batch equal to it alone."""
    N = 16
    W = _mask16(mask)
    X = image_blocks(140 + Bh + Bw, Bh, Bw, nimg, N=N)
    op = dctf.dctf_build_image_operator(W, N, border)
    Y = gpu_image(dctf, op, X, Bh, Bw, prec)
    Yref = oracle.filter_image_coeffs(X.astype(np.float64), Bh, Bw, W, border)
    err = np.abs(Y.astype(np.float64) - Yref).max()
    assert err <= TOL[prec], err
    if nimg > 1:
        per = Bh * Bw
        for i in range(nimg):
            assert np.array_equal(gpu_image(dctf, op, X[i * per:(i + 1) * per], Bh, Bw, prec),
                                  Y[i * per:(i + 1) * per])


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_image_filter_n16_uint8_after_inverse_dct(dctf, prec):
    Bh, Bw, N = 12, 20, 16
    X = image_blocks(91, Bh, Bw, N=N)
    W = _mask16("rand7")
    op = dctf.dctf_build_image_operator(W, N, R)
    Y = gpu_image(dctf, op, X, Bh, Bw, prec)
    Yref = oracle.filter_image_coeffs(X.astype(np.float64), Bh, Bw, W, R)
    u8ref, nh = oracle.idct_u8(Yref)
    pix = torch.empty(Y.size, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    dctf.dctf_idct_u8_verify(N, dev(Y.reshape(-1)), pix, dev(u8ref.reshape(-1)), cnt)
    torch.cuda.synchronize()
    got = pix.cpu().numpy().reshape(u8ref.shape)
    assert np.array_equal(got[~nh], u8ref[~nh])
    assert int(cnt[0]) == 0


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_full_size_n16_frames_sampled(dctf, prec):
    """32 frames of 3840 x 2160 in 16 x 16 blocks (1,036,800 blocks) in one
    launch, 7 x 7 mask, zero border: sampled interior blocks against the
    oracle's filter of a 3 x 3-block window around them (exact for a mask
    that reaches at most one block), and the corners and edges of the first
    and last frame against the oracle's whole-frame filter."""
    N, frames, h, w = 16, 32, 2160, 3840
    Bh, Bw = h // N, w // N
    nb = Bh * Bw
    X = torch.empty(frames * nb * N * N, dtype=torch.float32, device="cuda")
    for f in range(frames):
        dctf.dctf_forward_dct_u8(torch.from_numpy(syn.image_u8(3000 + f, h, w)).cuda(), N,
                                 X[f * nb * N * N:(f + 1) * nb * N * N])
    W = syn.random_mask(np.random.default_rng(7), 7, 7)
    op = dctf.dctf_build_image_operator(W, N, Z)
    Y = torch.empty_like(X)
    dctf.dctf_filter_image(op, prec, X, Y, Bh, Bw)
    torch.cuda.synchronize()
    Xb = X.view(frames, Bh, Bw, N, N)
    Yb = Y.view(frames, Bh, Bw, N, N)
    rng = np.random.default_rng(15)
    worst = 0.0
    for _ in range(40):
        f, r, c = int(rng.integers(frames)), int(rng.integers(1, Bh - 1)), int(rng.integers(1, Bw - 1))
        win = Xb[f, r - 1:r + 2, c - 1:c + 2].cpu().numpy().astype(np.float64).reshape(-1, N, N)
        ref = oracle.filter_image_coeffs(win, 3, 3, W, Z).reshape(3, 3, N, N)[1, 1]
        worst = max(worst, np.abs(Yb[f, r, c].cpu().numpy() - ref).max())
    for f in (0, frames - 1):
        full = oracle.filter_image_coeffs(Xb[f].cpu().numpy().astype(np.float64).reshape(-1, N, N), Bh, Bw,
                                          W, Z).reshape(Bh, Bw, N, N)
        got = Yb[f].cpu().numpy()
        for r, c in ((0, 0), (0, Bw - 1), (Bh - 1, 0), (Bh - 1, Bw - 1), (0, 100), (Bh - 1, 17), (60, 0),
                     (77, Bw - 1), (1, 1), (Bh - 2, Bw - 2)):
            worst = max(worst, np.abs(got[r, c] - full[r, c]).max())
    assert worst <= TOL[prec], worst
    del X, Y
    torch.cuda.empty_cache()
