"""Python binding of libdctf, the MI355X (gfx950) block-DCT filtering library.

Argument marshalling only: every step of the filtering path runs in the HIP
kernels of ``libdctf.so`` (declared in ``include/dctf.h``).  PyTorch supplies
device memory and streams.  The functions carry the C names; tensors stand in
for device pointers and ``stream`` defaults to torch's current stream.

Importing this module fails loudly when the library has not been built
(``python paper_1710_07193_amd/build.py`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded first: libdctf binds to the HIP runtime torch has loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdctf.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libdctf.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

DCTF_OK, DCTF_EINVAL, DCTF_EUNSUPPORTED, DCTF_ENOMEM, DCTF_EHIP, DCTF_EBUSY = 0, -1, -2, -3, -4, -5
DCTF_BORDER_ZERO, DCTF_BORDER_REPLICATE = 0, 1
DCTF_PREC_FP32, DCTF_PREC_SPLIT_BF16 = 0, 1
DCTF_RUN_REBUILD_OPERATORS = 1

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64


class _MaskDesc(ctypes.Structure):
    _fields_ = [("mask_host", _P), ("kh", _I), ("kw", _I), ("N", _I), ("border", _I)]


class _Job(ctypes.Structure):
    _fields_ = [("op", _P), ("in_", _P), ("out", _P), ("B", _I64)]


class _JobF64(ctypes.Structure):
    _fields_ = [("op", _P), ("in_", _P), ("out", _P), ("B", _I64)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("fronts", _I), ("io", _I), ("nt", _I), ("groups_per_cu", _I)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("arena_bytes", _I64), ("max_inflight", _I), ("max_batch_jobs", _I),
                ("max_cached_ops", _I), ("prec", _I)]


class _Request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("mask_host", _P), ("kh", _I), ("kw", _I), ("N", _I),
                ("border", _I), ("in_dev", _P), ("B", _I64), ("out_dev", _P), ("admit_s", ctypes.c_double),
                ("launch_s", ctypes.c_double), ("done_s", ctypes.c_double), ("status", _I), ("batch", _I)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("batches", _I64), ("cache_hits", _I64), ("cache_misses", _I64), ("cache_evictions", _I64),
                ("peak_arena_bytes", _I64), ("peak_inflight_batches", _I64), ("rejected", _I64),
                ("failed", _I64), ("busy_s", ctypes.c_double)]


_SIGS = {
    "dctf_build_operator": ([_P, _I, _I, _I, _I, _P, ctypes.POINTER(_P)], _I),
    "dctf_build_operators": ([ctypes.POINTER(_MaskDesc), _I, _P, ctypes.POINTER(_P)], _I),
    "dctf_rebuild_operators": ([ctypes.POINTER(_P), _I, _P], _I),
    "dctf_operator_fp64": ([_P, _P], _I),
    "dctf_operator_pixel_fp64": ([_P, _P], _I),
    "dctf_filter_blocks_u8": ([_P, _I, _P, _P, _I64, _P], _I),
    "dctf_filter_blocks_f64": ([_P, _P, _P, _I64, _P], _I),
    "dctf_build_image_operator": ([_P, _I, _I, _I, _I, _P, ctypes.POINTER(_P)], _I),
    "dctf_image_operator_fp64": ([_P, _I, _I, _I, _I, _P], _I),
    "dctf_image_operator_destroy": ([_P], None),
    "dctf_filter_image": ([_P, _I, _P, _P, _I, _I, _I64, _P], _I),
    "dctf_filter_quantized_u8": ([_P, _I, _P, _P, ctypes.c_float, _P, _I64, _P], _I),
    "dctf_filter_blocks_u8_raster": ([_P, _I, _P, _I, _I, _I64, _P, _I64, _I64, _P], _I),
    "dctf_filter_u8_raster": ([_P, _I, _P, _I64, _I64, _I, _I, _I64, _P, _I64, _I64, _P], _I),
    "dctf_operator_pixpix_fp64": ([_P, _P], _I),
    "dctf_filter_quantized_u8_raster": ([_P, _I, _P, _P, ctypes.c_float, _I, _I, _I64, _P, _I64, _I64, _P], _I),
    "dctf_operator_info": ([_P, _P, _P, _P, _P], _I),
    "dctf_operator_destroy": ([_P], None),
    "dctf_filter_blocks": ([_P, _I, _P, _P, _I64, _P], _I),
    "dctf_operator_rank": ([_P, _P], _I),
    "dctf_operator_factors_fp64": ([_P, _P, _P], _I),
    "dctf_filter_blocks_factored": ([_P, _P, _P, _I64, _P], _I),
    "dctf_operator_parity_classes": ([_P, _P], _I),
    "dctf_filter_blocks_parity": ([_P, _I, _P, _P, _I64, _P], _I),
    "dctf_batch_create": ([ctypes.POINTER(_Job), _I, _I, ctypes.POINTER(_P)], _I),
    "dctf_batch_run": ([_P, ctypes.c_uint, _P], _I),
    "dctf_batch_capture": ([_P, ctypes.c_uint, _P], _I),
    "dctf_batch_launch_graph": ([_P, _P], _I),
    "dctf_batch_info": ([_P, _P, _P, _P], _I),
    "dctf_batch_destroy": ([_P], None),
    "dctf_filter_batch": ([ctypes.POINTER(_Job), _I, _I, _P], _I),
    "dctf_filter_batch_noalloc": ([ctypes.POINTER(_Job), _I, _I, _P], _I),
    "dctf_filter_batch_f64": ([ctypes.POINTER(_JobF64), _I, _P], _I),
    "dctf_forward_dct_u8": ([_P, _I, _I, _I64, _I, _P, _P], _I),
    "dctf_forward_dct_u8_images": ([_P, _I, _I, _I64, _I64, _I64, _I, _P, _P], _I),
    "dctf_idct_u8_verify": ([_I, _P, _I64, _P, _P, _P, _P], _I),
    "dctf_stream_copy": ([_P, _P, _I64, _P], _I),
    "dctf_variant_count": ([_I, _I], _I),
    "dctf_variant_name": ([_I, _I, _I], ctypes.c_char_p),
    "dctf_get_variant": ([_I, _I, _P], _I),
    "dctf_set_variant": ([_I, _I, _I], _I),
    "dctf_autotune": ([_P, _I, _P, _P, _I64, _I, _P, _P, _P], _I),
    "dctf_set_batch_fronts": ([_I], _I),
    "dctf_set_batch_config": ([_I, ctypes.POINTER(_BatchConfig)], _I),
    "dctf_get_batch_config": ([_I, ctypes.POINTER(_BatchConfig)], _I),
    "dctf_batch_set_config": ([_P, ctypes.POINTER(_BatchConfig)], _I),
    "dctf_batch_get_config": ([_P, ctypes.POINTER(_BatchConfig), ctypes.POINTER(_BatchConfig)], _I),
    "dctf_batch_autotune": ([_P, ctypes.c_uint, _I, _I, ctypes.POINTER(_BatchConfig), _I, _P,
                             ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_I)], _I),
    "dctf_batch_autotune_candidates": ([ctypes.POINTER(_BatchConfig), _I], _I),
    "dctf_get_batch_fronts": ([], _I),
    "dctf_server_create": ([ctypes.POINTER(_ServerConfig), ctypes.POINTER(_P)], _I),
    "dctf_server_run": ([_P, ctypes.POINTER(_Request), _I], _I),
    "dctf_server_submit": ([_P, ctypes.POINTER(_Request)], _I),
    "dctf_server_poll": ([_P, ctypes.c_double, ctypes.POINTER(ctypes.POINTER(_Request)), _I, ctypes.POINTER(_I)], _I),
    "dctf_server_clock": ([_P], ctypes.c_double),
    "dctf_server_stats_get": ([_P, ctypes.POINTER(_ServerStats)], _I),
    "dctf_server_destroy": ([_P], None),
    "dctf_status_string": ([_I], ctypes.c_char_p),
    "dctf_version": ([], ctypes.c_char_p),
    "dctf_timing_enable": ([_I], _I),
    "dctf_timing_read": ([_P, _P], _I),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


class DctfError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = _lib.dctf_status_string(status).decode()
        super().__init__("%s: %s (status %d)" % (what, msg, status))


def _check(status: int, what: str):
    if status != DCTF_OK:
        raise DctfError(status, what)


def _stream(stream):
    if stream is None:
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return _P(stream.cuda_stream)
    return _P(int(stream))


def _dptr(t, dtype, what):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return _P(t.data_ptr())


class Operator:
    """Owning handle of a device-resident DCT-domain operator."""

    def __init__(self, handle: int, N: int, kh: int, kw: int, border: int):
        self.handle = handle
        self.N, self.kh, self.kw, self.border = N, kh, kw, border

    @property
    def _as_parameter_(self):
        return _P(self.handle)

    def destroy(self):
        if self.handle:
            _lib.dctf_operator_destroy(_P(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _mask_array(mask):
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.float64))
    if m.ndim == 1:
        m = m.reshape(1, -1)
    if m.ndim != 2:
        raise ValueError("mask must be 1-D or 2-D")
    return m


def dctf_build_operator(mask, N: int, border: int, stream=None) -> Operator:
    m = _mask_array(mask)
    h = _P()
    _check(_lib.dctf_build_operator(m.ctypes.data_as(_P), m.shape[0], m.shape[1], N, border,
                                    _stream(stream), ctypes.byref(h)), "dctf_build_operator")
    return Operator(h.value, N, m.shape[0], m.shape[1], border)


def dctf_build_operators(specs, stream=None) -> list:
    """``specs``: iterable of (mask, N, border); one builder launch for all."""
    arrays, descs = [], []
    for mask, N, border in specs:
        m = _mask_array(mask)
        arrays.append(m)
        descs.append(_MaskDesc(m.ctypes.data_as(_P), m.shape[0], m.shape[1], N, border))
    n = len(descs)
    arr = (_MaskDesc * max(n, 1))(*descs)
    out = (_P * max(n, 1))()
    _check(_lib.dctf_build_operators(arr, n, _stream(stream), out), "dctf_build_operators")
    return [Operator(out[i], descs[i].N, descs[i].kh, descs[i].kw, descs[i].border) for i in range(n)]


def dctf_rebuild_operators(ops, stream=None):
    arr = (_P * max(len(ops), 1))(*[o.handle for o in ops])
    _check(_lib.dctf_rebuild_operators(arr, len(ops), _stream(stream)), "dctf_rebuild_operators")


def dctf_operator_fp64(op: Operator) -> np.ndarray:
    nn = op.N * op.N
    H = np.empty((nn, nn), np.float64)
    _check(_lib.dctf_operator_fp64(op, H.ctypes.data_as(_P)), "dctf_operator_fp64")
    return H


def dctf_operator_pixel_fp64(op: Operator) -> np.ndarray:
    nn = op.N * op.N
    G = np.empty((nn, nn), np.float64)
    _check(_lib.dctf_operator_pixel_fp64(op, G.ctypes.data_as(_P)), "dctf_operator_pixel_fp64")
    return G


def dctf_operator_info(op: Operator):
    vals = [ctypes.c_int() for _ in range(4)]
    _check(_lib.dctf_operator_info(op, *[ctypes.byref(v) for v in vals]), "dctf_operator_info")
    return tuple(v.value for v in vals)


def dctf_filter_blocks(op: Operator, prec: int, X: torch.Tensor, Y: torch.Tensor, stream=None):
    """Y[b] = H_dct . X[b]; X, Y: float32 device tensors of B*N*N elements."""
    nn = op.N * op.N
    if X.numel() % nn or Y.numel() != X.numel():
        raise ValueError("X and Y must hold the same whole number of N*N blocks")
    _check(_lib.dctf_filter_blocks(op, prec, _dptr(X, torch.float32, "X"),
                                   _dptr(Y, torch.float32, "Y"), X.numel() // nn, _stream(stream)),
           "dctf_filter_blocks")


def dctf_operator_rank(op: Operator) -> int:
    r = ctypes.c_int()
    _check(_lib.dctf_operator_rank(op, ctypes.byref(r)), "dctf_operator_rank")
    return r.value


def dctf_operator_factors_fp64(op: Operator):
    """(P, Q): two [R, N, N] FP64 arrays with H_dct = sum_r kron(P[r], Q[r])."""
    R = dctf_operator_rank(op)
    P = np.empty((R, op.N, op.N), np.float64)
    Q = np.empty((R, op.N, op.N), np.float64)
    _check(_lib.dctf_operator_factors_fp64(op, P.ctypes.data_as(_P), Q.ctypes.data_as(_P)),
           "dctf_operator_factors_fp64")
    return P, Q


def dctf_filter_blocks_factored(op: Operator, X: torch.Tensor, Y: torch.Tensor, stream=None):
    """Y[b] = sum_r P_r X[b] Q_r^t (factored form, FP32 MFMA, N = 16)."""
    nn = op.N * op.N
    if X.numel() % nn or Y.numel() != X.numel():
        raise ValueError("X and Y must hold the same whole number of N*N blocks")
    _check(_lib.dctf_filter_blocks_factored(op, _dptr(X, torch.float32, "X"), _dptr(Y, torch.float32, "Y"),
                                            X.numel() // nn, _stream(stream)),
           "dctf_filter_blocks_factored")


def dctf_operator_parity_classes(op: Operator) -> int:
    """4 when the operator splits into parity-class operators (N = 16 or 32, mask
    mirror-symmetric on both axes), else 1."""
    c = ctypes.c_int()
    _check(_lib.dctf_operator_parity_classes(op, ctypes.byref(c)), "dctf_operator_parity_classes")
    return c.value


def dctf_filter_blocks_parity(op: Operator, prec: int, X: torch.Tensor, Y: torch.Tensor, stream=None):
    """Y[b] = H_dct . X[b] through the four parity-class operators (N = 16 or 32)."""
    nn = op.N * op.N
    if X.numel() % nn or Y.numel() != X.numel():
        raise ValueError("X and Y must hold the same whole number of N*N blocks")
    _check(_lib.dctf_filter_blocks_parity(op, prec, _dptr(X, torch.float32, "X"), _dptr(Y, torch.float32, "Y"),
                                          X.numel() // nn, _stream(stream)),
           "dctf_filter_blocks_parity")


def dctf_filter_blocks_f64(op: Operator, X: torch.Tensor, Y: torch.Tensor, stream=None):
    """Y[b] = H_dct . X[b] in FP64; X, Y: float64 device tensors of B*N*N elements."""
    nn = op.N * op.N
    if X.numel() % nn or Y.numel() != X.numel():
        raise ValueError("X and Y must hold the same whole number of N*N blocks")
    _check(_lib.dctf_filter_blocks_f64(op, _dptr(X, torch.float64, "X"), _dptr(Y, torch.float64, "Y"),
                                       X.numel() // nn, _stream(stream)),
           "dctf_filter_blocks_f64")


def dctf_filter_blocks_u8(op: Operator, prec: int, X: torch.Tensor, pix: torch.Tensor, stream=None):
    """pix[b] = u8(IDCT(H_dct . X[b])); X float32, pix uint8, B*N*N elements each."""
    nn = op.N * op.N
    if X.numel() % nn or pix.numel() != X.numel():
        raise ValueError("X and pix must hold the same whole number of N*N blocks")
    _check(_lib.dctf_filter_blocks_u8(op, prec, _dptr(X, torch.float32, "X"), _dptr(pix, torch.uint8, "pix"),
                                      X.numel() // nn, _stream(stream)),
           "dctf_filter_blocks_u8")


def dctf_filter_quantized_u8(op: Operator, prec: int, qcoef: torch.Tensor, qtable: torch.Tensor,
                             dc_offset: float, pix: torch.Tensor, stream=None):
    """pix[b] = u8(IDCT(H_dct . (qtable * qcoef[b] + dc_offset e_0))); qcoef int16,
    qtable float32 (N*N), pix uint8."""
    nn = op.N * op.N
    if qcoef.numel() % nn or pix.numel() != qcoef.numel():
        raise ValueError("qcoef and pix must hold the same whole number of N*N blocks")
    if qtable.numel() != nn:
        raise ValueError("qtable must hold N*N factors")
    _check(_lib.dctf_filter_quantized_u8(op, prec, _dptr(qcoef, torch.int16, "qcoef"),
                                         _dptr(qtable, torch.float32, "qtable"), float(dc_offset),
                                         _dptr(pix, torch.uint8, "pix"), qcoef.numel() // nn, _stream(stream)),
           "dctf_filter_quantized_u8")


def _raster_images(img: torch.Tensor, h: int, w: int):
    """(pointer, nimg, pitch, image stride) of uint8 device images: a 2-D
    tensor (one image) or a 3-D one (images along dim 0), rows contiguous,
    any row pitch (e.g. a column slice of wider images), at least h rows of
    w pixels each."""
    if not isinstance(img, torch.Tensor) or not img.is_cuda:
        raise TypeError("img must be a device tensor")
    if img.dtype != torch.uint8 or img.dim() not in (2, 3) or img.stride(-1) != 1:
        raise ValueError("img must be a 2-D or 3-D uint8 tensor with contiguous rows")
    if img.shape[-2] < h or img.shape[-1] < w:
        raise ValueError("img is smaller than h x w")
    nimg = img.shape[0] if img.dim() == 3 else 1
    stride = img.stride(0) if img.dim() == 3 else 0
    return _P(img.data_ptr()), nimg, img.stride(-2), stride


def dctf_filter_blocks_u8_raster(op: Operator, prec: int, X: torch.Tensor, h: int, w: int, img: torch.Tensor,
                                 stream=None):
    """The filtered pixels of coefficient blocks X (each image's ceil(h/N) x
    ceil(w/N) blocks, images one after another) written into the h x w uint8
    image(s) img: 2-D for one image, 3-D for several (row pitch and image
    stride from img's strides)."""
    ptr, nimg, pitch, stride = _raster_images(img, h, w)
    nb = -(-h // op.N) * -(-w // op.N)
    if X.numel() != nimg * nb * op.N * op.N:
        raise ValueError("X must hold the ceil(h/N) x ceil(w/N) blocks of every image")
    _check(_lib.dctf_filter_blocks_u8_raster(op, prec, _dptr(X, torch.float32, "X"), h, w, nimg, ptr, pitch,
                                             stride, _stream(stream)),
           "dctf_filter_blocks_u8_raster")


def dctf_filter_quantized_u8_raster(op: Operator, prec: int, qcoef: torch.Tensor, qtable: torch.Tensor,
                                    dc_offset: float, h: int, w: int, img: torch.Tensor, stream=None):
    """As dctf_filter_blocks_u8_raster from quantised int16 blocks."""
    ptr, nimg, pitch, stride = _raster_images(img, h, w)
    nb = -(-h // op.N) * -(-w // op.N)
    if qcoef.numel() != nimg * nb * op.N * op.N:
        raise ValueError("qcoef must hold the ceil(h/N) x ceil(w/N) blocks of every image")
    if qtable.numel() != op.N * op.N:
        raise ValueError("qtable must hold N*N factors")
    _check(_lib.dctf_filter_quantized_u8_raster(op, prec, _dptr(qcoef, torch.int16, "qcoef"),
                                                _dptr(qtable, torch.float32, "qtable"), float(dc_offset), h, w,
                                                nimg, ptr, pitch, stride, _stream(stream)),
           "dctf_filter_quantized_u8_raster")


def dctf_filter_u8_raster(op: Operator, prec: int, src: torch.Tensor, h: int, w: int, dst: torch.Tensor,
                          stream=None):
    """uint8 image(s) src -> filtered uint8 image(s) dst in one pass (N = 8):
    2-D tensors for one image, 3-D for several (rows contiguous, any row pitch
    and image stride)."""
    sp, sn, spitch, sstride = _raster_images(src, h, w)
    dp, dn, dpitch, dstride = _raster_images(dst, h, w)
    if sn != dn:
        raise ValueError("src and dst must hold the same number of images")
    _check(_lib.dctf_filter_u8_raster(op, prec, sp, spitch, sstride, h, w, sn, dp, dpitch, dstride,
                                      _stream(stream)), "dctf_filter_u8_raster")


def dctf_operator_pixpix_fp64(op: Operator) -> np.ndarray:
    """The FP64 pixel-to-pixel operator (64 x 64) of an N = 8 operator."""
    H = np.empty((64, 64), np.float64)
    _check(_lib.dctf_operator_pixpix_fp64(op, H.ctypes.data_as(_P)), "dctf_operator_pixpix_fp64")
    return H


class ImageOperator:
    """Owning handle of the neighbour operators of image-level filtering."""

    def __init__(self, handle: int, N: int, kh: int, kw: int, border: int):
        self.handle = handle
        self.N, self.kh, self.kw, self.border = N, kh, kw, border

    @property
    def _as_parameter_(self):
        return _P(self.handle)

    def destroy(self):
        if self.handle:
            _lib.dctf_image_operator_destroy(_P(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def dctf_build_image_operator(mask, N: int, border: int, stream=None) -> ImageOperator:
    m = _mask_array(mask)
    h = _P()
    _check(_lib.dctf_build_image_operator(m.ctypes.data_as(_P), m.shape[0], m.shape[1], N, border,
                                          _stream(stream), ctypes.byref(h)), "dctf_build_image_operator")
    return ImageOperator(h.value, N, m.shape[0], m.shape[1], border)


def dctf_image_operator_fp64(op: ImageOperator, row_class: int, col_class: int, dr: int, ds: int) -> np.ndarray:
    nn = op.N * op.N
    H = np.empty((nn, nn), np.float64)
    _check(_lib.dctf_image_operator_fp64(op, row_class, col_class, dr, ds, H.ctypes.data_as(_P)),
           "dctf_image_operator_fp64")
    return H


def dctf_filter_image(op: ImageOperator, prec: int, X: torch.Tensor, Y: torch.Tensor, Bh: int, Bw: int,
                      stream=None):
    """Image-level filter of X.numel() // (Bh*Bw*N*N) images of Bh x Bw blocks."""
    per = Bh * Bw * op.N * op.N
    if X.numel() % per or Y.numel() != X.numel():
        raise ValueError("X and Y must hold the same whole number of Bh x Bw block images")
    _check(_lib.dctf_filter_image(op, prec, _dptr(X, torch.float32, "X"), _dptr(Y, torch.float32, "Y"), Bh, Bw,
                                  X.numel() // per, _stream(stream)),
           "dctf_filter_image")


def filter_blocks(op: Operator, X: torch.Tensor, prec: int = DCTF_PREC_SPLIT_BF16, stream=None):
    Y = torch.empty_like(X)
    dctf_filter_blocks(op, prec, X, Y, stream)
    return Y


def _jobs(jobs):
    descs = []
    keep = []
    for op, X, Y in jobs:
        nn = op.N * op.N
        if X.numel() % nn or Y.numel() != X.numel():
            raise ValueError("job tensors must hold the same whole number of N*N blocks")
        keep.append(op)
        descs.append(_Job(op.handle, _dptr(X, torch.float32, "X"), _dptr(Y, torch.float32, "Y"),
                          X.numel() // nn))
    return (_Job * max(len(descs), 1))(*descs), len(descs), keep


class Batch:
    """Owning handle of a batch plan (work table + optional captured graph)."""

    def __init__(self, handle: int, keep):
        self.handle = handle
        self._keep = keep   # operators and tensors the plan points into

    @property
    def _as_parameter_(self):
        return _P(self.handle)

    def destroy(self):
        if self.handle:
            _lib.dctf_batch_destroy(_P(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def dctf_batch_create(jobs, prec: int) -> Batch:
    """``jobs``: list of (Operator, X, Y)."""
    arr, n, keep = _jobs(jobs)
    h = _P()
    _check(_lib.dctf_batch_create(arr, n, prec, ctypes.byref(h)), "dctf_batch_create")
    return Batch(h.value, (keep, [j[1] for j in jobs], [j[2] for j in jobs]))


def dctf_batch_run(batch: Batch, flags: int = 0, stream=None):
    _check(_lib.dctf_batch_run(batch, flags, _stream(stream)), "dctf_batch_run")


def dctf_batch_capture(batch: Batch, flags: int = 0, stream=None):
    _check(_lib.dctf_batch_capture(batch, flags, _stream(stream)), "dctf_batch_capture")


def dctf_batch_launch_graph(batch: Batch, stream=None):
    _check(_lib.dctf_batch_launch_graph(batch, _stream(stream)), "dctf_batch_launch_graph")


def dctf_batch_info(batch: Batch):
    vals = [ctypes.c_int() for _ in range(3)]
    _check(_lib.dctf_batch_info(batch, *[ctypes.byref(v) for v in vals]), "dctf_batch_info")
    return tuple(v.value for v in vals)


def dctf_filter_batch(jobs, prec: int, stream=None):
    arr, n, _ = _jobs(jobs)
    _check(_lib.dctf_filter_batch(arr, n, prec, _stream(stream)), "dctf_filter_batch")


def dctf_filter_batch_f64(jobs, stream=None):
    """FP64 filter jobs [(op, X, Y)] with float64 device tensors, one launch
    per job on the stream."""
    descs = []
    for op, X, Y in jobs:
        nn = op.N * op.N
        if X.numel() % nn or Y.numel() != X.numel():
            raise ValueError("job tensors must hold the same whole number of N*N blocks")
        descs.append(_JobF64(op.handle, _dptr(X, torch.float64, "X"), _dptr(Y, torch.float64, "Y"),
                             X.numel() // nn))
    arr = (_JobF64 * max(len(descs), 1))(*descs)
    _check(_lib.dctf_filter_batch_f64(arr, len(descs), _stream(stream)), "dctf_filter_batch_f64")


def dctf_filter_batch_noalloc(jobs, prec: int, stream=None):
    """dctf_filter_batch with its work table in the library's fixed device
    array (no device allocation; synchronous)."""
    arr, n, _ = _jobs(jobs)
    _check(_lib.dctf_filter_batch_noalloc(arr, n, prec, _stream(stream)), "dctf_filter_batch_noalloc")


def dctf_forward_dct_u8(img: torch.Tensor, N: int, coeffs: torch.Tensor, stream=None):
    """uint8 image (h, w) on the device -> coefficient blocks (raster order).
    The rows may be a view of a wider buffer: the row pitch is img.stride(0)."""
    if not isinstance(img, torch.Tensor) or not img.is_cuda or img.dtype != torch.uint8:
        raise TypeError("img must be a uint8 device tensor")
    if img.dim() != 2:
        raise ValueError("img must be 2-D")
    h, w = img.shape
    if img.stride(1) != 1 or img.stride(0) < w:
        raise ValueError("img rows must be contiguous, with a row pitch of at least the width")
    nblk = -(-h // N) * -(-w // N)
    if coeffs.numel() != nblk * N * N:
        raise ValueError("coeffs must hold %d blocks" % nblk)
    _check(_lib.dctf_forward_dct_u8(_P(img.data_ptr()), h, w, img.stride(0), N,
                                    _dptr(coeffs, torch.float32, "coeffs"), _stream(stream)),
           "dctf_forward_dct_u8")


def dctf_forward_dct_u8_images(imgs: torch.Tensor, N: int, coeffs: torch.Tensor, stream=None):
    """uint8 images (n, h, w) on the device -> their coefficient blocks, one
    image after another, in one launch.  Rows may be views of wider buffers
    (row pitch imgs.stride(1), image stride imgs.stride(0))."""
    if not isinstance(imgs, torch.Tensor) or not imgs.is_cuda or imgs.dtype != torch.uint8:
        raise TypeError("imgs must be a uint8 device tensor")
    if imgs.dim() != 3:
        raise ValueError("imgs must be 3-D (n, h, w)")
    n, h, w = imgs.shape
    if imgs.stride(2) != 1 or imgs.stride(1) < w:
        raise ValueError("image rows must be contiguous, with a row pitch of at least the width")
    nblk = -(-h // N) * -(-w // N)
    if coeffs.numel() != n * nblk * N * N:
        raise ValueError("coeffs must hold %d blocks" % (n * nblk))
    _check(_lib.dctf_forward_dct_u8_images(_P(imgs.data_ptr()), h, w, imgs.stride(1), imgs.stride(0), n, N,
                                           _dptr(coeffs, torch.float32, "coeffs"), _stream(stream)),
           "dctf_forward_dct_u8_images")


def dctf_idct_u8_verify(N: int, Y: torch.Tensor, pix: torch.Tensor, expected=None, counters=None,
                        stream=None):
    nn = N * N
    if Y.numel() % nn or pix.numel() != Y.numel():
        raise ValueError("Y and pix must hold the same number of N*N blocks")
    if expected is not None and expected.numel() != pix.numel():
        raise ValueError("expected has the wrong size")
    if counters is not None and (counters.numel() != 2 or counters.dtype != torch.int64):
        raise ValueError("counters must be two int64 values")
    _check(_lib.dctf_idct_u8_verify(N, _dptr(Y, torch.float32, "Y"), Y.numel() // nn,
                                    _dptr(pix, torch.uint8, "pix"),
                                    _dptr(expected, torch.uint8, "expected"),
                                    _dptr(counters, torch.int64, "counters"), _stream(stream)),
           "dctf_idct_u8_verify")


def dctf_stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Plain device copy (measurement aid: the achievable-HBM reference)."""
    if src.numel() != dst.numel():
        raise ValueError("sizes differ")
    _check(_lib.dctf_stream_copy(_dptr(src, torch.float32, "src"), _dptr(dst, torch.float32, "dst"),
                                 src.numel(), _stream(stream)), "dctf_stream_copy")


def dctf_variant_count(N: int, prec: int) -> int:
    return int(_lib.dctf_variant_count(N, prec))


def dctf_variant_name(N: int, prec: int, v: int):
    r = _lib.dctf_variant_name(N, prec, v)
    return r.decode() if r else None


def dctf_get_variant(N: int, prec: int) -> int:
    v = ctypes.c_int()
    _check(_lib.dctf_get_variant(N, prec, ctypes.byref(v)), "dctf_get_variant")
    return v.value


def dctf_set_variant(N: int, prec: int, v: int):
    _check(_lib.dctf_set_variant(N, prec, v), "dctf_set_variant")


def dctf_autotune(op: Operator, prec: int, X: torch.Tensor, Y: torch.Tensor, iters: int = 10,
                  stream=None):
    """Time every variant on (X -> Y) and select the fastest; returns (variant, ms)."""
    nn = op.N * op.N
    v, ms = ctypes.c_int(), ctypes.c_float()
    _check(_lib.dctf_autotune(op, prec, _dptr(X, torch.float32, "X"), _dptr(Y, torch.float32, "Y"),
                              X.numel() // nn, iters, _stream(stream), ctypes.byref(v),
                              ctypes.byref(ms)), "dctf_autotune")
    return v.value, ms.value


def dctf_set_batch_fronts(fronts: int):
    _check(_lib.dctf_set_batch_fronts(fronts), "dctf_set_batch_fronts")


def dctf_get_batch_fronts() -> int:
    return int(_lib.dctf_get_batch_fronts())


BATCH_CONFIG_FIELDS = ("fronts", "io", "nt", "groups_per_cu")


def _cfg_struct(cfg) -> _BatchConfig:
    return _BatchConfig(*(int(cfg[k]) for k in BATCH_CONFIG_FIELDS))


def _cfg_dict(c: _BatchConfig) -> dict:
    return {k: int(getattr(c, k)) for k in BATCH_CONFIG_FIELDS}


def dctf_set_batch_config(prec: int, cfg: dict):
    """Process-wide configuration new batch plans of `prec` take (dict with
    fronts, io, nt, groups_per_cu)."""
    c = _cfg_struct(cfg)
    _check(_lib.dctf_set_batch_config(prec, ctypes.byref(c)), "dctf_set_batch_config")


def dctf_get_batch_config(prec: int) -> dict:
    c = _BatchConfig()
    _check(_lib.dctf_get_batch_config(prec, ctypes.byref(c)), "dctf_get_batch_config")
    return _cfg_dict(c)


def dctf_batch_set_config(batch: Batch, cfg: dict):
    c = _cfg_struct(cfg)
    _check(_lib.dctf_batch_set_config(batch, ctypes.byref(c)), "dctf_batch_set_config")


def dctf_batch_get_config(batch: Batch):
    """(configuration the plan was made with, what it resolved to)."""
    c, r = _BatchConfig(), _BatchConfig()
    _check(_lib.dctf_batch_get_config(batch, ctypes.byref(c), ctypes.byref(r)), "dctf_batch_get_config")
    return _cfg_dict(c), _cfg_dict(r)


def dctf_batch_autotune_candidates() -> list:
    n = int(_lib.dctf_batch_autotune_candidates(None, 0))
    arr = (_BatchConfig * n)()
    _lib.dctf_batch_autotune_candidates(arr, n)
    return [_cfg_dict(arr[i]) for i in range(n)]


def dctf_batch_autotune(batch: Batch, flags: int = 0, iters: int = 10, rounds: int = 3, candidates=None,
                        stream=None):
    """Times each candidate configuration on the plan and leaves it with the
    fastest.  Returns (index of the best, list of (candidate, ms per launch or
    -1 when skipped))."""
    cands = list(candidates) if candidates is not None else dctf_batch_autotune_candidates()
    arr = (_BatchConfig * max(len(cands), 1))(*[_cfg_struct(c) for c in cands])
    ms = (ctypes.c_float * max(len(cands), 1))()
    best = _I(-1)
    _check(_lib.dctf_batch_autotune(batch, flags, iters, rounds, arr if candidates is not None else None,
                                    len(cands) if candidates is not None else 0, _stream(stream), ms,
                                    ctypes.byref(best)), "dctf_batch_autotune")
    return best.value, [(c, float(ms[i])) for i, c in enumerate(cands)]


class Server:
    """Owning handle of a continuous-batching server.  Requests submitted
    through the online interface are kept here (their records, masks and
    tensors) until a poll hands them back."""

    def __init__(self, handle: int):
        self.handle = handle
        self.live = {}

    @property
    def _as_parameter_(self):
        return _P(self.handle)

    def destroy(self):
        if self.handle:
            _lib.dctf_server_destroy(_P(self.handle))
            self.handle = 0
            self.live.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class ServerRequest:
    """One request of the online interface (its record is written by the
    server: admit_s, launch_s, done_s on the server clock, status, batch)."""

    def __init__(self, rec, keep):
        self.rec = rec
        self.keep = keep

    def __getattr__(self, name):
        if name in ("admit_s", "launch_s", "done_s", "status", "batch", "arrival_s", "B", "N"):
            return getattr(self.rec, name)
        raise AttributeError(name)


def _request(mask, N, border, X, Y, arrival_s, what):
    m = _mask_array(mask)
    if X.numel() % (N * N) or X.numel() == 0:
        raise ValueError("%s: X must hold a whole, positive number of N*N blocks" % what)
    if Y is not None and Y.numel() != X.numel():
        raise ValueError("%s: Y has the wrong size" % what)
    rec = _Request(arrival_s, m.ctypes.data_as(_P), m.shape[0], m.shape[1], N, border,
                   _dptr(X, torch.float32, "X"), X.numel() // (N * N), _dptr(Y, torch.float32, "Y"),
                   -1.0, -1.0, -1.0, 0, -1)
    return rec, m


def dctf_server_submit(server: Server, mask, N: int, border: int, X: torch.Tensor, Y=None,
                       arrival_s: float = -1.0) -> ServerRequest:
    """Queue one request (online interface).  X (and Y, if given) are device
    float32 tensors of B*N*N elements; they are kept alive with the request."""
    rec, m = _request(mask, N, border, X, Y, arrival_s, "request")
    _check(_lib.dctf_server_submit(server, ctypes.byref(rec)), "dctf_server_submit")
    req = ServerRequest(rec, (m, X, Y))
    server.live[ctypes.addressof(rec)] = req
    return req


def dctf_server_poll(server: Server, wait_s: float = 0.0, max_done: int = 64) -> list:
    """Progress the server; the requests that completed (at most max_done)."""
    arr = (ctypes.POINTER(_Request) * max(max_done, 1))()
    n = _I()
    _check(_lib.dctf_server_poll(server, float(wait_s), arr, int(max_done), ctypes.byref(n)), "dctf_server_poll")
    return [server.live.pop(ctypes.addressof(arr[i].contents)) for i in range(n.value)]


def dctf_server_clock(server: Server) -> float:
    return float(_lib.dctf_server_clock(server))


def dctf_server_create(arena_bytes: int, max_inflight: int = 4, max_batch_jobs: int = 64,
                       max_cached_ops: int = 64, prec: int = DCTF_PREC_SPLIT_BF16) -> Server:
    cfg = _ServerConfig(arena_bytes, max_inflight, max_batch_jobs, max_cached_ops, prec)
    h = _P()
    _check(_lib.dctf_server_create(ctypes.byref(cfg), ctypes.byref(h)), "dctf_server_create")
    return Server(h.value)


def dctf_server_run(server: Server, requests):
    """``requests``: list of dicts with arrival_s, mask, N, border, X (device
    float32 tensor, B*N*N elements) and optionally Y (device tensor receiving
    the output).  Returns a list of dicts with admit_s, launch_s, done_s,
    status and batch for each request."""
    arr = (_Request * max(len(requests), 1))()
    keep = []
    for i, r in enumerate(requests):
        arr[i], m = _request(r["mask"], r["N"], r["border"], r["X"], r.get("Y"), r["arrival_s"], "request %d" % i)
        keep.append(m)
    _check(_lib.dctf_server_run(server, arr, len(requests)), "dctf_server_run")
    return [dict(admit_s=arr[i].admit_s, launch_s=arr[i].launch_s, done_s=arr[i].done_s,
                 status=arr[i].status, batch=arr[i].batch) for i in range(len(requests))]


def dctf_server_stats(server: Server) -> dict:
    st = _ServerStats()
    _check(_lib.dctf_server_stats_get(server, ctypes.byref(st)), "dctf_server_stats_get")
    return {k: getattr(st, k) for k, _ in _ServerStats._fields_}


def dctf_status_string(s: int) -> str:
    return _lib.dctf_status_string(s).decode()


def dctf_version() -> str:
    return _lib.dctf_version().decode()


def dctf_timing_enable(on: bool):
    _check(_lib.dctf_timing_enable(1 if on else 0), "dctf_timing_enable")


def dctf_timing_read():
    avg, n = ctypes.c_double(), ctypes.c_int()
    _check(_lib.dctf_timing_read(ctypes.byref(avg), ctypes.byref(n)), "dctf_timing_read")
    return avg.value, n.value


def raw_library():
    """The ctypes handle of libdctf (for symbol checks)."""
    return _lib
