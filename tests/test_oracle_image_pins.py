"""Pins of the oracle's image-level (cross-block) filter.

Compared with scipy's correlation over the whole pixel image (its own DCT
and filter code), brute force over an explicitly padded image, the
block-local oracle (a one-block image, and the centre term of an interior
block), exact shifts, constants, and the rank the mask's reach allows.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.ndimage

import oracle
import synthetic as syn

Z, R = oracle.BORDER_ZERO, oracle.BORDER_REPLICATE


def _image_from_blocks(X, Bh, Bw):
    N = X.shape[-1]
    x = scipy.fft.idctn(X, type=2, norm="ortho", axes=(-2, -1))
    return x.reshape(Bh, Bw, N, N).transpose(0, 2, 1, 3).reshape(Bh * N, Bw * N)


def _blocks_from_image(img, N):
    Hh, Ww = img.shape
    b = img.reshape(Hh // N, N, Ww // N, N).transpose(0, 2, 1, 3).reshape(-1, N, N)
    return scipy.fft.dctn(b, type=2, norm="ortho", axes=(-2, -1))


def _scipy_image_filter(X, Bh, Bw, W, border):
    kh, kw = W.shape
    origin = (-1 if kh % 2 == 0 else 0, -1 if kw % 2 == 0 else 0)
    img = _image_from_blocks(X, Bh, Bw)
    f = scipy.ndimage.correlate(img, W, mode="constant" if border == Z else "nearest", cval=0.0,
                                origin=origin)
    return _blocks_from_image(f, X.shape[-1])


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N,Bh,Bw,kh,kw", [(8, 5, 7, 5, 5), (8, 3, 3, 3, 3), (8, 1, 4, 7, 7), (8, 4, 1, 1, 5),
                                           (8, 2, 2, 17, 17), (8, 3, 5, 4, 4), (4, 6, 5, 3, 5),
                                           (2, 4, 4, 5, 5), (16, 2, 3, 7, 7)])
def test_image_filter_matches_scipy(N, Bh, Bw, kh, kw, border):
    rng = np.random.default_rng(100 * N + 10 * kh + kw)
    X = rng.normal(0, 30, size=(Bh * Bw, N, N))
    X[:, 0, 0] += 128 * N
    W = rng.uniform(-1, 1, size=(kh, kw))
    Y = oracle.filter_image_coeffs(X, Bh, Bw, W, border)
    assert np.abs(Y - _scipy_image_filter(X, Bh, Bw, W, border)).max() < 1e-9


@pytest.mark.parametrize("border", [Z, R])
def test_image_filter_brute_force_padded(border):
    N, Bh, Bw = 4, 2, 3
    rng = np.random.default_rng(3)
    X = rng.normal(0, 20, size=(Bh * Bw, N, N))
    W = rng.uniform(-1, 1, size=(3, 5))
    img = _image_from_blocks(X, Bh, Bw)
    pad = np.pad(img, ((1, 1), (2, 2)), mode="constant" if border == Z else "edge")
    f = np.zeros_like(img)
    for y in range(img.shape[0]):
        for x in range(img.shape[1]):
            f[y, x] = sum(W[p, q] * pad[y + p, x + q] for p in range(3) for q in range(5))
    Y = oracle.filter_image_coeffs(X, Bh, Bw, W, border)
    assert np.abs(Y - _blocks_from_image(f, N)).max() < 1e-10


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N", [4, 8])
def test_one_block_image_equals_block_local_filter(N, border):
    rng = np.random.default_rng(N)
    X = rng.normal(0, 30, size=(5, N, N))
    W = syn.random_mask(rng, 5, 5)
    Y = oracle.filter_image_coeffs(X, 1, 1, W, border)       # five 1x1-block images
    assert np.abs(Y - oracle.filter_coeffs(X, W, border)).max() < 1e-10


def test_interior_centre_term_is_block_local_zero_operator():
    N = 8
    W = syn.asym_mask_5x5()
    for border in (Z, R):
        Hc = oracle.image_operator_probe(N, W, border, 3, 3, 1, 1, 0, 0)
        assert np.abs(Hc - oracle.operator_probe(N, W, Z)).max() < 1e-12


def test_neighbour_terms_have_the_rank_of_the_reach():
    # 5x5 mask: two pixel rows / columns reach into a neighbour, so an edge
    # neighbour's operator has rank 2N and a corner neighbour's rank 4.
    N = 8
    W = syn.random_mask(np.random.default_rng(6), 5, 5)
    for (dr, ds), rank in (((0, 1), 2 * N), ((1, 0), 2 * N), ((-1, 0), 2 * N), ((1, 1), 4), ((-1, 1), 4)):
        H = oracle.image_operator_probe(N, W, Z, 3, 3, 1, 1, dr, ds)
        sv = np.linalg.svd(H, compute_uv=False)
        assert int((sv > 1e-10 * sv[0]).sum()) == rank, (dr, ds)
    # a 3x3 mask reaches one pixel: corner rank 1
    H = oracle.image_operator_probe(N, syn.box_mask(3), Z, 3, 3, 1, 1, 1, -1)
    assert int((np.linalg.svd(H, compute_uv=False) > 1e-10).sum()) == 1


def test_shift_mask_shifts_the_image():
    N, Bh, Bw = 8, 3, 4
    rng = np.random.default_rng(9)
    img = rng.uniform(0, 255, size=(Bh * N, Bw * N))
    X = _blocks_from_image(img, N)
    W = syn.delta_mask(7, 7, dy=2, dx=-3)          # selects pixel (y + 2, x - 3)
    f = _image_from_blocks(oracle.filter_image_coeffs(X, Bh, Bw, W, Z), Bh, Bw)
    ref = np.zeros_like(img)
    ref[:-2, 3:] = img[2:, :-3]
    assert np.abs(f - ref).max() < 1e-10


def test_constant_image_stays_constant_under_replication():
    N, Bh, Bw = 8, 3, 2
    X = np.zeros((Bh * Bw, N, N))
    X[:, 0, 0] = 77.0 * N
    W = syn.random_mask(np.random.default_rng(2), 7, 7)
    Y = oracle.filter_image_coeffs(X, Bh, Bw, W, R)
    assert np.abs(Y - X).max() < 1e-10
