"""Pins of the oracle's pixel-output functions (the filtered result taken back
to the spatial domain, Sec. III) and of the JPEG-style dequantisation.

Each check compares the oracle with something other than itself: scipy's
inverse DCT and correlation, the oracle's independent pixel route (filter
the uint8 pixels directly, never touching coefficients), a closed form
(a constant image stays constant), or a bound fixed by the quantiser.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.ndimage

import oracle
import synthetic as syn

Z, R = oracle.BORDER_ZERO, oracle.BORDER_REPLICATE


def _scipy_filter(x, W, border):
    kh, kw = W.shape
    origin = (-1 if kh % 2 == 0 else 0, -1 if kw % 2 == 0 else 0)
    mode = "constant" if border == Z else "nearest"
    return scipy.ndimage.correlate(x, W, mode=mode, cval=0.0, origin=origin)


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N,kh,kw", [(2, 3, 3), (4, 5, 5), (8, 3, 3), (8, 5, 5), (8, 7, 7), (8, 1, 5),
                                     (8, 4, 4), (16, 7, 7)])
def test_pixel_operator_matches_scipy(N, kh, kw, border):
    W = np.random.default_rng(10 * N + kh).uniform(-1, 1, size=(kh, kw))
    G = oracle.pixel_operator_probe(N, W, border)
    ref = np.empty_like(G)
    for k in range(N * N):
        e = np.zeros(N * N)
        e[k] = 1.0
        x = scipy.fft.idctn(e.reshape(N, N), type=2, norm="ortho")
        ref[:, k] = _scipy_filter(x, W, border).reshape(-1)
    assert np.abs(G - ref).max() < 1e-13


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_identity_mask_pixel_operator_is_the_inverse_dct(N):
    for border in (Z, R):
        G = oracle.pixel_operator_probe(N, syn.delta_mask(3, 3), border)
        for k in (0, 1, N, N * N - 1):
            e = np.zeros((N, N))
            e.flat[k] = 1.0
            col = scipy.fft.idctn(e, type=2, norm="ortho").reshape(-1)
            assert np.abs(G[:, k] - col).max() < 1e-14


def test_pixel_operator_box3_n2_closed_form():
    # 2x2 block, 3x3 box, replication: f00 = (4 x00 + 2 x01 + 2 x10 + x11) / 9.
    # Input coefficient 1 (u = 0, v = 1) is x = [[.5, -.5], [.5, -.5]], so
    # f00 = (2 - 1 + 1 - .5) / 9 = 1/6 and, by the sign pattern, f01 = -1/6.
    G = oracle.pixel_operator_probe(2, syn.box_mask(3), R)
    assert abs(G[0, 1] - 1.0 / 6.0) < 1e-15 and abs(G[1, 1] + 1.0 / 6.0) < 1e-15
    assert np.abs(G[:, 0] - 0.5).max() < 1e-15          # the DC basis block stays 1/2


@pytest.mark.parametrize("border", [Z, R])
def test_coeff_route_pixels_equal_pixel_route(border):
    """filter(IDCT(DCT(px))) rounds to the same uint8 as filter(px) computed
    straight from the pixels, except inside the 1e-3 band around .5."""
    px = oracle.tile_u8(syn.image_u8(4, 96, 128), 8)
    X = oracle.dct_pixels(px)
    W = syn.asym_mask_5x5()
    f, u8, nh = oracle.filter_coeffs_to_pixels(X, W, border)
    _, u8_ref, nh_ref = oracle.filter_pixels(px, W, border)
    outside = ~(nh | nh_ref)
    assert np.array_equal(u8[outside], u8_ref[outside])
    ref = np.stack([_scipy_filter(scipy.fft.idctn(b, type=2, norm="ortho"), W, border) for b in X])
    assert np.abs(f - ref).max() < 1e-10


def test_dequantized_constant_image_stays_constant():
    # A constant image of value v: a codec with level shift 128 stores the DC
    # term (v - 128) N; with q0 = 4 and v = 100 that is -224 = -56 q0 exactly.
    N, v = 8, 100.0
    q = syn.quant_table(N)
    assert q[0, 0] == 4.0
    qc = np.zeros((3, N, N), np.int16)
    qc[:, 0, 0] = -56
    X = oracle.dequantize(qc, q, dc_offset=128.0 * N)
    assert np.all(X[:, 0, 0] == N * v)
    W = syn.random_mask(np.random.default_rng(8), 5, 5)   # sum 1
    f, u8, _ = oracle.filter_coeffs_to_pixels(X, W, R)
    assert np.abs(f - v).max() < 1e-11 and np.all(u8 == 100)


def test_quantize_dequantize_error_bound():
    N = 8
    px = oracle.tile_u8(syn.image_u8(5, 64, 64), N)
    X = oracle.dct_pixels(px)
    q = syn.quant_table(N)
    qc = syn.quantize(X, q, dc_offset=128.0 * N)
    Xh = oracle.dequantize(qc, q, dc_offset=128.0 * N)
    assert np.all(np.abs(Xh - X) <= q / 2 + 1e-9)
    assert np.abs(Xh - X).max() > 0.1          # the table does quantise
