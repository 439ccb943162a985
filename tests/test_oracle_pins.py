"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
library routine (scipy's DCT and correlation), a closed form derived by hand
(``tests/golden/closed_forms.txt``), the paper's own printed 3x3 matrices
(``tests/golden/paper_3x3_matrices_n8.txt``, Sec. II.B-C) combined per
eq. 6-20, brute force on tiny blocks, or an invariant of the definition.
"""
import os

import numpy as np
import pytest
import scipy.fft
import scipy.ndimage

import oracle
from oracle import paper_route
import synthetic as syn

Z, R = oracle.BORDER_ZERO, oracle.BORDER_REPLICATE
NS = (2, 4, 8, 16)


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- DCT (eq. 1-3)

@pytest.mark.parametrize("N", NS + (3, 5))
def test_dct_matrix_orthonormal(N):
    C = oracle.dct_matrix(N)
    assert np.abs(C @ C.T - np.eye(N)).max() < 1e-14      # eq. 2: C^-1 = C^t
    assert np.allclose(C[0], np.sqrt(1.0 / N), atol=0, rtol=1e-15)


def test_dct_matrix_n2_closed_form():
    s = 1.0 / np.sqrt(2.0)
    assert np.abs(oracle.dct_matrix(2) - np.array([[s, s], [s, -s]])).max() < 1e-15


@pytest.mark.parametrize("N", NS)
def test_dct2_matches_scipy(N):
    x = _rng(N).uniform(0, 255, size=(7, N, N))
    X = oracle.dct2(x)
    ref = scipy.fft.dctn(x, type=2, norm="ortho", axes=(-2, -1))
    assert np.abs(X - ref).max() < 1e-10
    back = oracle.idct2(X)
    assert np.abs(back - x).max() < 1e-10
    assert np.abs(back - scipy.fft.idctn(X, type=2, norm="ortho", axes=(-2, -1))).max() < 1e-10


def test_dct2_of_constant_block_is_dc_only():
    N = 8
    X = oracle.dct2(np.full((1, N, N), 100.0))[0]
    assert abs(X[0, 0] - N * 100.0) < 1e-11
    X[0, 0] = 0
    assert np.abs(X).max() < 1e-11


def test_dct2_orientation_row_is_first_index():
    # A block that varies along rows only has energy only in column v = 0.
    N = 8
    x = np.repeat(np.arange(N, dtype=float)[:, None], N, axis=1)[None]
    X = oracle.dct2(x)[0]
    assert np.abs(X[:, 1:]).max() < 1e-11 and np.abs(X[1:, 0]).max() > 1.0


# ------------------------------------------------------ spatial filter (eq. 5)

def _scipy_block_filter(x, W, border):
    kh, kw = W.shape
    # scipy centres a kernel at K//2; the oracle's anchor is (K-1)//2.
    origin = (-1 if kh % 2 == 0 else 0, -1 if kw % 2 == 0 else 0)
    mode = "constant" if border == Z else "nearest"
    return scipy.ndimage.correlate(x, W, mode=mode, cval=0.0, origin=origin)


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N,kh,kw", [(8, 3, 3), (8, 5, 5), (8, 7, 7), (8, 1, 5), (8, 5, 1),
                                     (8, 4, 4), (8, 2, 3), (16, 9, 9), (4, 9, 9), (2, 5, 5),
                                     (8, 17, 17)])
def test_filter_matches_scipy_correlate(N, kh, kw, border):
    rng = _rng(kh * 31 + kw)
    W = rng.uniform(-1, 1, size=(kh, kw))
    x = rng.integers(0, 256, size=(3, N, N)).astype(float)
    f = oracle.filter_spatial(x, W, border)
    for b in range(3):
        assert np.abs(f[b] - _scipy_block_filter(x[b], W, border)).max() < 1e-9


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N", [2, 4])
def test_filter_brute_force_padded(N, border):
    """Pad the block explicitly (zeros, or edge copies as in Fig. 1) and take
    every K x K window: a different formulation from the oracle's clamping."""
    rng = _rng(N + 10 * border)
    for kh, kw in [(3, 3), (5, 3), (1, 3)]:
        W = rng.uniform(-1, 1, size=(kh, kw))
        x = rng.integers(0, 256, size=(N, N)).astype(float)
        ah, aw = (kh - 1) // 2, (kw - 1) // 2
        pad = ((ah, kh - 1 - ah), (aw, kw - 1 - aw))
        xp = np.pad(x, pad, mode="constant" if border == Z else "edge")
        ref = np.zeros((N, N))
        for i in range(N):
            for j in range(N):
                acc = 0.0
                for p in range(kh):
                    for q in range(kw):
                        acc += W[p, q] * xp[i + p, j + q]
                ref[i, j] = acc
        assert np.abs(oracle.filter_spatial(x[None], W, border)[0] - ref).max() < 1e-10


def test_filter_is_correlation_not_convolution():
    # w11 multiplies block(i-1, j-1) (the paper's matrices a and b, Sec. II.B).
    N = 8
    W = np.zeros((3, 3))
    W[0, 0] = 1.0
    x = np.arange(N * N, dtype=float).reshape(1, N, N)
    f = oracle.filter_spatial(x, W, Z)[0]
    assert f[3, 4] == x[0, 2, 3]
    assert f[0, 5] == 0.0 and f[5, 0] == 0.0


@pytest.mark.parametrize("border", [Z, R])
def test_shifted_delta_is_exact_shift(border):
    N = 8
    x = _rng(3).integers(0, 256, size=(1, N, N)).astype(float)
    for dy, dx in [(-2, 1), (1, 0), (0, -1), (2, 2)]:
        W = syn.delta_mask(5, 5, dy, dx)
        f = oracle.filter_spatial(x, W, border)[0]
        for i in range(N):
            for j in range(N):
                r, c = i + dy, j + dx
                if border == Z:
                    want = x[0, r, c] if (0 <= r < N and 0 <= c < N) else 0.0
                else:
                    want = x[0, min(max(r, 0), N - 1), min(max(c, 0), N - 1)]
                assert f[i, j] == want


# --------------------------------------------------------- operator (probe)

def _shift_matrix(N, d, border):
    S = np.zeros((N, N))
    for i in range(N):
        m = i + d
        if border == Z:
            if 0 <= m < N:
                S[i, m] = 1.0
        else:
            S[i, min(max(m, 0), N - 1)] = 1.0
    return S


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N", NS)
def test_identity_mask_gives_identity_operator(N, border):
    for W in (np.ones((1, 1)), syn.delta_mask(3, 3), syn.delta_mask(5, 3), syn.delta_mask(4, 2)):
        H = oracle.operator_probe(N, W, border)
        assert np.abs(H - np.eye(N * N)).max() < 1e-13


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N", (4, 8))
def test_shifted_delta_operator_is_kronecker_of_shift_matrices(N, border):
    C = paper_route.dct_matrix(N)
    for dy, dx in [(-1, 2), (1, -1), (0, 1)]:
        H = oracle.operator_probe(N, syn.delta_mask(5, 5, dy, dx), border)
        A = C @ _shift_matrix(N, dy, border) @ C.T
        B = C @ _shift_matrix(N, dx, border) @ C.T
        assert np.abs(H - np.kron(A, B)).max() < 1e-13


@pytest.mark.parametrize("N", NS)
def test_constant_block_stays_constant_under_replicate(N):
    rng = _rng(N)
    for k in (3, 5, 7):
        if k > 2 * N + 1:
            continue
        W = syn.random_mask(rng, k, k)
        H = oracle.operator_probe(N, W, R)
        e0 = np.zeros(N * N)
        e0[0] = 1.0
        assert np.abs(H[:, 0] - e0).max() < 1e-13
        x = np.full((1, N, N), 137.0)
        assert np.abs(oracle.filter_spatial(x, W, R) - 137.0).max() < 1e-11


def _golden_closed_forms(golden_dir):
    rows = {}
    for line in open(os.path.join(golden_dir, "closed_forms.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows[parts[0]] = parts[1:]
    return rows


def test_hand_derived_closed_forms(golden_dir):
    rows = _golden_closed_forms(golden_dir)
    masks = {"box3": syn.box_mask(3), "identity": np.ones((1, 1))}
    checked = 0
    for name, vals in rows.items():
        if name.startswith("gaussian"):
            continue
        N, border = int(vals[0]), int(vals[1])
        diag = np.array([float(v) for v in vals[2:]])
        H = oracle.operator_probe(N, masks[name.split("_")[0]], border)
        assert np.abs(H - np.diag(diag)).max() < 1e-14, name
        checked += 1
    assert checked == 4


def test_gaussian_mask_closed_form(golden_dir):
    vals = _golden_closed_forms(golden_dir)["gaussian3_sigma1"]
    want = dict(zip(vals[0::2], map(float, vals[1::2])))
    g = syn.gaussian_mask(3, 1.0)
    assert abs(g[1, 1] - want["centre"]) < 1e-8
    assert abs(g[0, 1] - want["edge"]) < 1e-7
    assert abs(g[0, 0] - want["corner"]) < 1e-7


@pytest.mark.parametrize("N", NS)
def test_symmetric_separable_3tap_replicate_is_diagonal(N):
    """Clamp at radius 1 is the half-sample symmetric extension whose
    eigenbasis is DCT-II (Martucci, ref. [9] of the paper): for W = g g^T
    with g = [g1, g0, g1], H is diagonal with entries l_u l_v,
    l_k = g0 + 2 g1 cos(pi k / N)."""
    for g0, g1 in [(0.5, 0.25), (0.2041799555 / 0.4518, 0.0), (1.0, -0.4)]:
        g = np.array([g1, g0, g1])
        H = oracle.operator_probe(N, np.outer(g, g), R)
        lam = g0 + 2 * g1 * np.cos(np.pi * np.arange(N) / N)
        assert np.abs(H - np.diag(np.kron(lam, lam))).max() < 1e-13
    H = oracle.operator_probe(N, syn.gaussian_mask(3, 1.0), R)
    assert np.abs(H - np.diag(np.diag(H))).max() < 1e-13


@pytest.mark.parametrize("N", (4, 8))
def test_zero_mode_adjoint_trace_frobenius(N):
    rng = _rng(N + 100)
    for kh, kw in [(3, 3), (5, 5), (3, 5), (7, 7)]:
        W = rng.uniform(-1, 1, size=(kh, kw))
        H = oracle.operator_probe(N, W, Z)
        # rotating an odd mask by 180 degrees gives the adjoint (transpose) operator
        assert np.abs(oracle.operator_probe(N, W[::-1, ::-1].copy(), Z) - H.T).max() < 1e-13
        assert abs(np.trace(H) - N * N * W[(kh - 1) // 2, (kw - 1) // 2]) < 1e-12
        # ||H_dct||_F = ||H_sp||_F (orthogonal similarity); H_sp from explicit shifts
        Hsp = sum(W[p, q] * np.kron(_shift_matrix(N, p - (kh - 1) // 2, Z),
                                    _shift_matrix(N, q - (kw - 1) // 2, Z))
                  for p in range(kh) for q in range(kw))
        assert abs(np.linalg.norm(H) - np.linalg.norm(Hsp)) < 1e-12


@pytest.mark.parametrize("border", [Z, R])
@pytest.mark.parametrize("N", (4, 8, 16))
def test_operator_is_dct_similarity_of_spatial_operator(N, border):
    """H_dct = (C (x) C) H_sp (C (x) C)^T with H_sp assembled from explicit
    0/1 shift (or clamp) matrices, one Kronecker term per mask entry."""
    rng = _rng(N * 3 + border)
    W = rng.uniform(-1, 1, size=(5, 3))
    C = paper_route.dct_matrix(N)
    CC = np.kron(C, C)
    Hsp = sum(W[p, q] * np.kron(_shift_matrix(N, p - 2, border), _shift_matrix(N, q - 1, border))
              for p in range(5) for q in range(3))
    assert np.abs(oracle.operator_probe(N, W, border) - CC @ Hsp @ CC.T).max() < 1e-12


@pytest.mark.parametrize("border", [Z, R])
def test_separable_mask_factorises(border):
    N = 8
    rng = _rng(7 + border)
    g, h = rng.uniform(-1, 1, 5), rng.uniform(-1, 1, 3)
    C = paper_route.dct_matrix(N)
    Mg = sum(g[p] * _shift_matrix(N, p - 2, border) for p in range(5))
    Mh = sum(h[q] * _shift_matrix(N, q - 1, border) for q in range(3))
    H = oracle.operator_probe(N, np.outer(g, h), border)
    assert np.abs(H - np.kron(C @ Mg @ C.T, C @ Mh @ C.T)).max() < 1e-12


@pytest.mark.parametrize("border", [Z, R])
def test_linearity_in_mask(border):
    N = 8
    rng = _rng(11)
    W1, W2 = rng.uniform(-1, 1, (5, 5)), rng.uniform(-1, 1, (5, 5))
    H = oracle.operator_probe(N, 0.3 * W1 - 1.7 * W2, border)
    ref = 0.3 * oracle.operator_probe(N, W1, border) - 1.7 * oracle.operator_probe(N, W2, border)
    assert np.abs(H - ref).max() < 1e-12


# ------------------------------------------ the paper's own route (eq. 6-20)

def _parse_paper_matrices(path):
    mats, name, rows = {}, None, []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("matrix "):
            if name:
                mats[name] = rows
            name, rows = line.split()[1], []
        else:
            rows.append(line.split())
    mats[name] = rows
    return mats


def _eval_symbolic(rows, W):
    sym = {}
    for p in range(3):
        for q in range(3):
            sym[f"w{p + 1}{q + 1}"] = W[p, q]
            sym[f"w{3 * p + q + 1}"] = W[p, q]
    out = np.zeros((len(rows), len(rows[0])))
    for i, r in enumerate(rows):
        for j, tok in enumerate(r):
            out[i, j] = sum(float(t) if t[0].isdigit() else sym[t] for t in tok.split("+"))
    return out


def test_paper_matrices_transcription(golden_dir):
    mats = _parse_paper_matrices(os.path.join(golden_dir, "paper_3x3_matrices_n8.txt"))
    assert len(mats) == 13
    W = _rng(5).uniform(-1, 1, (3, 3))
    built = paper_route.spatial_matrices(W, 8)
    for name, rows in mats.items():
        assert np.array_equal(_eval_symbolic(rows, W), built[name]), name


@pytest.mark.parametrize("N", (4, 8, 16))
def test_paper_route_equals_definition(N):
    rng = _rng(N + 50)
    masks = [rng.uniform(-1, 1, (3, 3)), syn.gaussian_mask(3, 1.0),
             syn.magic_square_3(False), syn.magic_square_3(True)]
    X = oracle.dct2(rng.integers(0, 256, size=(6, N, N)).astype(float))
    for W in masks:
        Yz = oracle.filter_coeffs(X, W, Z)
        Yr = oracle.filter_coeffs(X, W, R)
        for b in range(X.shape[0]):
            assert np.abs(paper_route.filter_zero(X[b], W) - Yz[b]).max() < 1e-9   # eq. 11
            assert np.abs(paper_route.filter_replicate(X[b], W) - Yr[b]).max() < 1e-9  # eq. 20


def test_paper_route_rejects_convolution_reading():
    # The asymmetric magic square distinguishes correlation from convolution:
    # the paper's matrices agree with the former only.
    N = 8
    W = syn.magic_square_3(True)
    X = oracle.dct2(_rng(9).integers(0, 256, size=(1, N, N)).astype(float))
    conv = oracle.filter_coeffs(X, W[::-1, ::-1].copy(), R)[0]
    assert np.abs(paper_route.filter_replicate(X[0], W) - conv).max() > 1.0


def test_paper_symmetric_shortcut_eq12():
    N = 8
    rng = _rng(12)
    r1, r2 = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    W = np.stack([r1, r2, r1])                   # first row equals third row
    X = oracle.dct2(rng.integers(0, 256, size=(1, N, N)).astype(float))[0]
    assert np.abs(paper_route.filter_symmetric_zero(X, W) - oracle.filter_coeffs(X[None], W, Z)[0]).max() < 1e-9


@pytest.mark.parametrize("N", [8, 16])
@pytest.mark.parametrize("border", [Z, R])
def test_doubly_symmetric_mask_decouples_parity_classes(N, border):
    """A mask mirror-symmetric on both axes (odd sides) filters a block's
    mirror images alike, and DCT basis vectors are even or odd under the
    mirror (C J = D C, D = diag((-1)^k)): H_dct vanishes between coefficients
    whose row (or column) indices differ in parity, so it splits into four
    parity-class operators.  Checked on the oracle's probe of the spatial
    filter (not its own H): zero to rounding for symmetric masks, and clearly
    nonzero when either mirror symmetry or the odd side is missing."""
    rng = _rng(44)
    A = rng.uniform(-1, 1, (7, 7))
    B = A + A[::-1]
    sym = (B + B[:, ::-1]) / 4
    u = np.arange(N * N) // N
    v = np.arange(N * N) % N
    odd = ((u[:, None] + u[None, :]) % 2 == 1) | ((v[:, None] + v[None, :]) % 2 == 1)
    for W in (sym, syn.gaussian_mask(5, sigma=1.0), syn.box_mask(3), sym[3:4]):
        H = oracle.operator_probe(N, W, border)
        assert np.abs(H[odd]).max() < 1e-13 * np.abs(H).max()
    for W in ((A + A[:, ::-1]) / 2, (A + A[::-1]) / 2, np.ones((4, 4)) / 16):
        H = oracle.operator_probe(N, W, border)
        assert np.abs(H[odd]).max() > 1e-3


# ------------------------------------------------- pixels, uint8, tiling

def test_u8_rounding_rule():
    # one pixel per case through the identity mask, read back through the rule
    # (Sec. III: the floating filtered value, rounded half up and saturated).
    # 2.5 - 2e-8 is decided in FP64: an FP32 rounding of it would be 2.5 -> 3.
    vals = np.array([2.5, 2.4999, -0.5, -3.0, 255.49, 255.5, 300.0, 0.49, 127.5, 2.5 - 2e-8])
    want = np.array([3, 2, 0, 0, 255, 255, 255, 0, 128, 2], np.uint8)
    N = 2
    Y = np.zeros((len(vals), N, N))
    # a constant block of value v has DC = N * v and no AC
    Y[:, 0, 0] = vals * N
    u8, nh = oracle.idct_u8(Y)
    assert np.array_equal(u8[:, 0, 0], want)
    assert np.array_equal(nh[:, 0, 0], np.abs(vals - np.floor(vals) - 0.5) < 1e-3)


def test_filter_pixels_consistent_with_coeff_route():
    N = 8
    img = syn.image_u8(1, 64, 64)
    px = oracle.tile_u8(img, N)
    W = syn.asym_mask_5x5()
    for border in (Z, R):
        Y, u8, nh = oracle.filter_pixels(px, W, border)
        Yc = oracle.filter_coeffs(oracle.dct_pixels(px), W, border)
        assert np.abs(Y - Yc).max() < 1e-9
        u8b, _ = oracle.idct_u8(Y)
        assert np.array_equal(u8b[~nh], u8[~nh])


def test_box_filter_never_near_half():
    # 3x3 box outputs are k/9 for integer k: never within 1e-3 of a .5 boundary.
    px = oracle.tile_u8(syn.image_u8(0, 64, 64), 8)
    _, _, nh = oracle.filter_pixels(px, syn.box_mask(3), Z)
    assert not nh.any()


def test_tile_u8_raster_order_and_replicate_pad():
    img = np.arange(20 * 12, dtype=np.uint8).reshape(20, 12)
    blocks = oracle.tile_u8(img, 8)
    assert blocks.shape == (3 * 2, 8, 8)
    assert np.array_equal(blocks[1][:, :4], img[0:8, 8:12])
    assert np.array_equal(blocks[1][:, 4:], np.repeat(img[0:8, 11:12], 4, axis=1))
    assert np.array_equal(blocks[4][4:], np.repeat(img[19:20, 0:8], 4, axis=0))


def test_sampled_matches_full():
    N = 8
    X = oracle.coeffs_fp32(oracle.tile_u8(syn.image_u8(4, 64, 64), N))
    W = syn.asym_mask_5x5()
    full = oracle.filter_coeffs(X.astype(np.float64), W, R).reshape(-1, N * N)
    rng = _rng(0)
    bi = rng.integers(0, X.shape[0], 50)
    ci = rng.integers(0, N * N, 50)
    assert np.array_equal(oracle.filter_coeffs_sampled(X, W, R, bi, ci), full[bi, ci])


def test_generators_are_seeded():
    assert np.array_equal(syn.image_u8(7, 32, 48), syn.image_u8(7, 32, 48))
    assert not np.array_equal(syn.image_u8(7, 32, 48), syn.image_u8(8, 32, 48))
    pool = syn.mask_pool_16()
    assert len(pool) == 16 and all(abs(m.mask.sum() - 1) < 1e-12 for m in pool)
    assert all(np.abs(m.mask).max() <= 1.0 for m in pool)
    assert {m.shape[0] for m in pool} <= {3, 5, 7}
    for m in pool:
        if m.symmetric:
            assert np.allclose(m.mask, m.mask[::-1, :]) and np.allclose(m.mask, m.mask[:, ::-1])
    s32 = syn.mask_set_32()
    assert len(s32) == 32
    for m in s32:
        if m.separable:
            assert np.linalg.matrix_rank(m.mask) == 1


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.operator_probe(8, np.ones((18, 3)), Z)      # K > 2N+1
    with pytest.raises(ValueError):
        oracle.operator_probe(8, np.ones((3, 3)), 2)       # unknown border
