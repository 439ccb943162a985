"""Plain FP64 CPU oracle for block-DCT filtering (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
implementation in ``paper_1710_07193_amd`` and never imports it.

The arithmetic lives in ``dctf_oracle.c`` (plain C, FP64, definitions written
out as sums).  This module compiles it with gcc on first use, loads it with
ctypes and wraps it for numpy arrays.  ``paper_route`` holds a second,
independent route that follows the paper's own 3x3 matrix construction
(Sec. II.B-C, eq. 6-20).

Conventions (the paper's notation where it has one):
  * blocks are ``x[i][j]``, i the row, j the column, 0-based;
  * the DCT is orthonormal DCT-II, BLOCK = C.block.C^t (eq. 1, 2);
  * coefficient vectors are row-major, index ``u*N + v``;
  * masks are correlated, anchor ``floor((K-1)/2)`` (eq. 5 read as the
    paper's matrices a..e fix it: w11 weights block(i-1, j-1));
  * border 0 = zero padding (Sec. II.B), 1 = replication (Sec. II.C, Fig. 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

BORDER_ZERO = 0
BORDER_REPLICATE = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dctf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_dctf.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP over blocks)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            i32, i64 = ctypes.c_int, ctypes.c_int64
            sig = {
                "or_num_threads": ([], i32),
                "or_set_num_threads": ([i32], None),
                "or_dct_matrix": ([i32, P], None),
                "or_dct2": ([i32, i64, P, P], i32),
                "or_idct2": ([i32, i64, P, P], i32),
                "or_filter_spatial": ([i32, P, i32, i32, i32, i64, P, P], i32),
                "or_filter_coeffs": ([i32, P, i32, i32, i32, i64, P, P], i32),
                "or_filter_coeffs_sampled": ([i32, P, i32, i32, i32, i64, P, P, P, P], i32),
                "or_filter_pixels": ([i32, P, i32, i32, i32, i64, P, P, P, P], i32),
                "or_idct_u8": ([i32, i64, P, P, P], i32),
                "or_operator_probe": ([i32, P, i32, i32, i32, P], i32),
                "or_filter_coeffs_to_pixels": ([i32, P, i32, i32, i32, i64, P, P, P, P], i32),
                "or_pixel_operator_probe": ([i32, P, i32, i32, i32, P], i32),
                "or_filter_image_coeffs": ([i32, P, i32, i32, i32, i32, i32, i32, P, P], i32),
                "or_tile_u8": ([P, i32, i32, i32, P], i32),
            }
            for name, (args, res) in sig.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = res
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle: invalid arguments to %s" % what)


def _mask(W):
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    if W.ndim == 1:
        W = W.reshape(1, -1)
    if W.ndim != 2:
        raise ValueError("mask must be 2-D")
    return W


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the loops over blocks; n < 1 restores the default."""
    _load().or_set_num_threads(int(n))


def dct_matrix(N: int) -> np.ndarray:
    """Orthonormal DCT-II matrix C (eq. 1-2)."""
    C = np.empty((N, N), np.float64)
    _load().or_dct_matrix(N, _ptr(C))
    return C


def dct2(x) -> np.ndarray:
    """Eq. 1 for a batch ``[..., N, N]`` (FP64)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    N = x.shape[-1]
    out = np.empty_like(x)
    _check(_load().or_dct2(N, x.size // (N * N), _ptr(x), _ptr(out)), "dct2")
    return out


def idct2(X) -> np.ndarray:
    """Eq. 3 for a batch ``[..., N, N]`` (FP64)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    N = X.shape[-1]
    out = np.empty_like(X)
    _check(_load().or_idct2(N, X.size // (N * N), _ptr(X), _ptr(out)), "idct2")
    return out


def filter_spatial(x, W, border: int) -> np.ndarray:
    """Block-local spatial filter (eq. 5 as correlation, Fig. 1) of ``[..., N, N]``."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    W = _mask(W)
    N = x.shape[-1]
    out = np.empty_like(x)
    _check(_load().or_filter_spatial(N, _ptr(W), W.shape[0], W.shape[1], border,
                                     x.size // (N * N), _ptr(x), _ptr(out)), "filter_spatial")
    return out


def filter_coeffs(X, W, border: int) -> np.ndarray:
    """Y = DCT(filter(IDCT(X))) for coefficient blocks ``[..., N, N]`` (FP64)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    W = _mask(W)
    N = X.shape[-1]
    out = np.empty_like(X)
    _check(_load().or_filter_coeffs(N, _ptr(W), W.shape[0], W.shape[1], border,
                                    X.size // (N * N), _ptr(X), _ptr(out)), "filter_coeffs")
    return out


def filter_coeffs_sampled(X32, W, border: int, block_idx, coef_idx) -> np.ndarray:
    """Selected outputs ``Y[block_idx[s]][coef_idx[s]]`` of ``filter_coeffs``.

    ``X32`` is the FP32 coefficient array ``[B, N, N]`` (or ``[B, N*N]``) read as
    exact doubles; each sample is computed from its own block only.
    """
    X32 = np.ascontiguousarray(np.asarray(X32, dtype=np.float32))
    W = _mask(W)
    N = int(round(np.sqrt(X32.shape[-1]))) if X32.ndim == 2 else X32.shape[-1]
    bi = np.ascontiguousarray(np.asarray(block_idx, dtype=np.int64))
    ci = np.ascontiguousarray(np.asarray(coef_idx, dtype=np.int32))
    if bi.shape != ci.shape:
        raise ValueError("index arrays differ in shape")
    nblk = X32.size // (N * N)
    if bi.size and (bi.min() < 0 or bi.max() >= nblk or ci.min() < 0 or ci.max() >= N * N):
        raise ValueError("sample index out of range")
    out = np.empty(bi.shape, np.float64)
    _check(_load().or_filter_coeffs_sampled(N, _ptr(W), W.shape[0], W.shape[1], border,
                                            bi.size, _ptr(bi), _ptr(ci), _ptr(X32), _ptr(out)),
           "filter_coeffs_sampled")
    return out


def filter_pixels(px, W, border: int):
    """From uint8 pixel blocks ``[B, N, N]``: (Y = DCT(filter(px)) FP64,
    uint8 pixels of filter(px), near-1/2 flags)."""
    px = np.ascontiguousarray(np.asarray(px, dtype=np.uint8))
    W = _mask(W)
    N = px.shape[-1]
    Y = np.empty(px.shape, np.float64)
    u8 = np.empty(px.shape, np.uint8)
    nh = np.empty(px.shape, np.uint8)
    _check(_load().or_filter_pixels(N, _ptr(W), W.shape[0], W.shape[1], border,
                                    px.size // (N * N), _ptr(px), _ptr(Y), _ptr(u8), _ptr(nh)),
           "filter_pixels")
    return Y, u8, nh.astype(bool)


def idct_u8(Y):
    """uint8 pixels (and near-1/2 flags) of the inverse DCT of ``[B, N, N]``."""
    Y = np.ascontiguousarray(np.asarray(Y, dtype=np.float64))
    N = Y.shape[-1]
    u8 = np.empty(Y.shape, np.uint8)
    nh = np.empty(Y.shape, np.uint8)
    _check(_load().or_idct_u8(N, Y.size // (N * N), _ptr(Y), _ptr(u8), _ptr(nh)), "idct_u8")
    return u8, nh.astype(bool)


def operator_probe(N: int, W, border: int) -> np.ndarray:
    """H[:, k] = DCT(filter(IDCT(e_k))): the N^2 x N^2 DCT-domain operator,
    row = output coefficient u*N+v, column = input coefficient."""
    W = _mask(W)
    H = np.empty((N * N, N * N), np.float64)
    _check(_load().or_operator_probe(N, _ptr(W), W.shape[0], W.shape[1], border, _ptr(H)),
           "operator_probe")
    return H


def filter_coeffs_to_pixels(X, W, border: int):
    """From coefficient blocks ``[B, N, N]``: (f = filter(IDCT(X)) FP64,
    uint8 pixels of f, near-1/2 flags)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    W = _mask(W)
    N = X.shape[-1]
    f = np.empty(X.shape, np.float64)
    u8 = np.empty(X.shape, np.uint8)
    nh = np.empty(X.shape, np.uint8)
    _check(_load().or_filter_coeffs_to_pixels(N, _ptr(W), W.shape[0], W.shape[1], border,
                                              X.size // (N * N), _ptr(X), _ptr(f), _ptr(u8), _ptr(nh)),
           "filter_coeffs_to_pixels")
    return f, u8, nh.astype(bool)


def pixel_operator_probe(N: int, W, border: int) -> np.ndarray:
    """G[:, k] = filter(IDCT(e_k)): the N^2 x N^2 map from coefficients to
    filtered pixels, row = output pixel i*N+j, column = input coefficient."""
    W = _mask(W)
    G = np.empty((N * N, N * N), np.float64)
    _check(_load().or_pixel_operator_probe(N, _ptr(W), W.shape[0], W.shape[1], border, _ptr(G)),
           "pixel_operator_probe")
    return G


def filter_image_coeffs(X, Bh: int, Bw: int, W, border: int) -> np.ndarray:
    """Image-level filter of block-DCT images: ``X`` holds nimg images of
    Bh x Bw coefficient blocks ``[nimg*Bh*Bw, N, N]`` (raster order); each
    image is inverse transformed, correlated with ``W`` over the whole image
    (zero or replicated pixels outside the image only), and cut into blocks
    and transformed again.  FP64."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    W = _mask(W)
    N = X.shape[-1]
    nb = X.size // (N * N)
    if nb % (Bh * Bw):
        raise ValueError("block count is not a multiple of Bh * Bw")
    Y = np.empty_like(X)
    rc = _load().or_filter_image_coeffs(N, _ptr(W), W.shape[0], W.shape[1], border, Bh, Bw,
                                        nb // (Bh * Bw), _ptr(X), _ptr(Y))
    _check(rc, "filter_image_coeffs")
    return Y


def image_operator_probe(N: int, W, border: int, Bh: int, Bw: int, R: int, S: int, dr: int, ds: int):
    """Column k of the result is the filtered block (R, S) of a Bh x Bw image
    whose only non-zero block is (R + dr, S + ds) = e_k (the operator block
    that carries neighbour (dr, ds) into (R, S)); zero if that neighbour is
    outside the image."""
    nn = N * N
    H = np.zeros((nn, nn))
    if not (0 <= R + dr < Bh and 0 <= S + ds < Bw):
        return H
    X = np.zeros((nn, Bh * Bw, N, N))
    for k in range(nn):
        X[k, (R + dr) * Bw + S + ds].flat[k] = 1.0
    Y = filter_image_coeffs(X.reshape(-1, N, N), Bh, Bw, W, border).reshape(nn, Bh * Bw, nn)
    return Y[:, R * Bw + S, :].T.copy()


def dequantize(qcoef, qtable, dc_offset: float = 0.0) -> np.ndarray:
    """JPEG-style dequantisation of integer coefficient blocks ``[B, N, N]``:
    X[u][v] = qtable[u][v] * qcoef[u][v], plus ``dc_offset`` on X[0][0] (the
    DC term of a level shift: a codec that subtracted 128 from every pixel
    before its orthonormal DCT passes 128 * N here).  FP64."""
    qc = np.asarray(qcoef, dtype=np.float64)
    q = np.asarray(qtable, dtype=np.float64)
    N = qc.shape[-1]
    if q.shape != (N, N):
        raise ValueError("qtable must be N x N")
    X = qc * q
    X[..., 0, 0] += dc_offset
    return X


def tile_u8(img, N: int) -> np.ndarray:
    """Cut a 2-D uint8 image into ``[B, N, N]`` blocks, raster order; ragged
    sides are extended by repeating the last row/column."""
    img = np.ascontiguousarray(np.asarray(img, dtype=np.uint8))
    h, w = img.shape
    bh, bw = -(-h // N), -(-w // N)
    out = np.empty((bh * bw, N, N), np.uint8)
    _check(_load().or_tile_u8(_ptr(img), h, w, N, _ptr(out)), "tile_u8")
    return out


def dct_pixels(px) -> np.ndarray:
    """FP64 forward DCT (eq. 1) of uint8 pixel blocks ``[B, N, N]``."""
    return dct2(np.asarray(px, dtype=np.float64))


def coeffs_fp32(px) -> np.ndarray:
    """The FP32 coefficient input of the DCT-domain filter: RNE of the FP64 DCT."""
    return dct_pixels(px).astype(np.float32)
