"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments on the host before any device
work (no compute call is made here)."""
import ctypes
import math
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "dctf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dctf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1710_07193_amd as dctf
    return dctf.raw_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("dctf_build_operator", "dctf_filter_blocks", "dctf_filter_batch",
                     "dctf_batch_create", "dctf_batch_capture", "dctf_idct_u8_verify",
                     "dctf_autotune", "dctf_operator_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_is_in_tree_and_gfx950():
    import paper_1710_07193_amd as dctf
    assert os.path.dirname(dctf.LIB_PATH) == os.path.join(ROOT, "paper_1710_07193_amd")
    assert "gfx950" in dctf.dctf_version()


def test_status_strings(lib):
    import paper_1710_07193_amd as dctf
    for s in (0, -1, -2, -3, -4, -5):
        assert dctf.dctf_status_string(s)
    assert dctf.dctf_status_string(-99) == "unknown status"


def _mask(vals):
    arr = (ctypes.c_double * len(vals))(*vals)
    return ctypes.cast(arr, ctypes.c_void_p), arr


def test_build_operator_validation(lib):
    out = ctypes.c_void_p()
    m, keep = _mask([1.0 / 9] * 9)
    assert lib.dctf_build_operator(m, 3, 3, 3, 0, None, ctypes.byref(out)) == -2   # N = 3
    assert lib.dctf_build_operator(m, 3, 3, 64, 0, None, ctypes.byref(out)) == -2  # N = 64
    assert lib.dctf_build_operator(m, 3, 3, 0, 0, None, ctypes.byref(out)) == -1
    assert lib.dctf_build_operator(None, 3, 3, 8, 0, None, ctypes.byref(out)) == -1
    assert lib.dctf_build_operator(m, 0, 3, 8, 0, None, ctypes.byref(out)) == -1
    assert lib.dctf_build_operator(m, 3, 18, 8, 0, None, ctypes.byref(out)) == -1  # > 2N+1
    assert lib.dctf_build_operator(m, 3, 3, 8, 2, None, ctypes.byref(out)) == -1   # border
    assert lib.dctf_build_operator(m, 3, 3, 8, 0, None, None) == -1
    bad, keep2 = _mask([1.0, math.nan, 0.0])
    assert lib.dctf_build_operator(bad, 1, 3, 8, 0, None, ctypes.byref(out)) == -1
    inf, keep3 = _mask([1.0, math.inf, 0.0])
    assert lib.dctf_build_operator(inf, 1, 3, 8, 0, None, ctypes.byref(out)) == -1


def test_filter_and_batch_validation(lib):
    assert lib.dctf_filter_blocks(None, 0, None, None, 10, None) == -1
    out = ctypes.c_void_p()
    assert lib.dctf_batch_create(None, -1, 0, ctypes.byref(out)) == -1
    assert lib.dctf_batch_create(None, 0, 7, ctypes.byref(out)) == -1
    assert lib.dctf_batch_create(None, 0, 0, None) == -1
    assert lib.dctf_batch_run(None, 0, None) == -1
    assert lib.dctf_batch_capture(None, 0, None) == -1
    assert lib.dctf_batch_launch_graph(None, None) == -1
    assert lib.dctf_rebuild_operators(None, -1, None) == -1
    assert lib.dctf_operator_fp64(None, None) == -1
    assert lib.dctf_autotune(None, 0, None, None, 1, 1, None, None, None) == -1
    assert lib.dctf_operator_rank(None, None) == -1
    assert lib.dctf_operator_factors_fp64(None, None, None) == -1
    assert lib.dctf_filter_blocks_factored(None, None, None, 1, None) == -1
    assert lib.dctf_operator_parity_classes(None, None) == -1
    assert lib.dctf_filter_blocks_parity(None, 1, None, None, 1, None) == -1
    assert lib.dctf_operator_pixel_fp64(None, None) == -1
    assert lib.dctf_filter_blocks_f64(None, None, None, 1, None) == -1
    assert lib.dctf_filter_image(None, 0, None, None, 1, 1, 1, None) == -1
    assert lib.dctf_image_operator_fp64(None, 0, 0, 0, 0, None) == -1
    assert lib.dctf_build_image_operator(None, 3, 3, 8, 0, None, None) == -1
    out = ctypes.c_void_p()
    m, keep = _mask([1.0 / 9] * 9)
    assert lib.dctf_build_image_operator(m, 3, 3, 32, 0, None, ctypes.byref(out)) == -2   # N = 32
    assert lib.dctf_build_image_operator(m, 3, 3, 5, 0, None, ctypes.byref(out)) == -2    # N = 5
    assert lib.dctf_filter_blocks_u8(None, 0, None, None, 1, None) == -1
    assert lib.dctf_filter_quantized_u8(None, 0, None, None, ctypes.c_float(0.0), None, 1, None) == -1


def test_verify_and_forward_dct_validation(lib):
    assert lib.dctf_idct_u8_verify(3, None, 1, None, None, None, None) == -2
    assert lib.dctf_idct_u8_verify(64, None, 1, None, None, None, None) == -2
    assert lib.dctf_idct_u8_verify(32, None, 5, None, None, None, None) == -1   # N = 32 supported: null
    assert lib.dctf_idct_u8_verify(8, None, -1, None, None, None, None) == -1
    assert lib.dctf_idct_u8_verify(8, None, 0, None, None, None, None) == 0     # B = 0: no-op
    assert lib.dctf_idct_u8_verify(8, None, 5, None, None, None, None) == -1
    assert lib.dctf_forward_dct_u8(None, 8, 8, 8, 6, None, None) == -2
    assert lib.dctf_forward_dct_u8(None, 8, 8, 8, 8, None, None) == -1


def test_forward_dct_binding_checks_the_image():
    """The binding passes a row-pitched view's stride as the pitch, and refuses
    host tensors, other dtypes, non-2-D images and rows that are not contiguous
    before any library call."""
    import torch

    import paper_1710_07193_amd as dctf
    X = torch.empty(64)
    with pytest.raises(TypeError):
        dctf.dctf_forward_dct_u8(torch.zeros(8, 8, dtype=torch.uint8), 8, X)   # host tensor
    with pytest.raises(TypeError):
        dctf.dctf_forward_dct_u8(torch.zeros(8, 8), 8, X)                     # float32 image
    with pytest.raises(TypeError):
        dctf.dctf_forward_dct_u8(None, 8, X)


def test_variant_table(lib):
    import paper_1710_07193_amd as dctf
    for N in (2, 4, 8, 16):
        for prec in (0, 1):
            n = dctf.dctf_variant_count(N, prec)
            assert n >= 1
            names = [dctf.dctf_variant_name(N, prec, v) for v in range(n)]
            assert all(names) and len(set(names)) == n
            assert dctf.dctf_variant_name(N, prec, n) is None
    assert dctf.dctf_variant_count(3, 0) == 0
    assert lib.dctf_set_variant(8, 0, 999) == -1
    n8 = dctf.dctf_variant_count(8, 1)
    dctf.dctf_set_variant(8, 1, n8 - 1)
    assert dctf.dctf_get_variant(8, 1) == n8 - 1
    dctf.dctf_set_variant(8, 1, 0)
    assert dctf.dctf_get_variant(8, 1) == 0


def test_batch_fronts_setting(lib):
    f0 = lib.dctf_get_batch_fronts()
    try:
        assert lib.dctf_set_batch_fronts(-2) == -1
        assert lib.dctf_set_batch_fronts(4097) == -1
        assert lib.dctf_set_batch_fronts(3) == 0 and lib.dctf_get_batch_fronts() == 3
        assert lib.dctf_set_batch_fronts(0) == 0 and lib.dctf_get_batch_fronts() == 0
        # -1: each plan takes its precision's default
        assert lib.dctf_set_batch_fronts(-1) == 0 and lib.dctf_get_batch_fronts() == -1
    finally:
        lib.dctf_set_batch_fronts(f0)


def test_server_config_validation(lib):
    import paper_1710_07193_amd as dctf
    out = ctypes.c_void_p()
    for cfg in [(100, 4, 8, 8, 1), (1 << 20, 0, 8, 8, 1), (1 << 20, 17, 8, 8, 1), (1 << 20, 4, 0, 8, 1),
                (1 << 20, 4, 8, 0, 1), (1 << 20, 4, 8, 8, 3)]:
        c = dctf._ServerConfig(*cfg)
        assert lib.dctf_server_create(ctypes.byref(c), ctypes.byref(out)) == -1, cfg
    assert lib.dctf_server_create(None, ctypes.byref(out)) == -1
    assert lib.dctf_server_run(None, None, 0) == -1
    assert lib.dctf_server_stats_get(None, None) == -1


def test_server_online_calls_validate_on_the_host(lib):
    import paper_1710_07193_amd as dctf
    lib.dctf_server_clock.restype = ctypes.c_double
    assert lib.dctf_server_clock(None) == -1.0
    assert lib.dctf_server_submit(None, None) == -1
    n = ctypes.c_int(7)
    assert lib.dctf_server_poll(None, ctypes.c_double(0.0), None, 0, ctypes.byref(n)) == -1
    # a server handle is needed for the request checks; without a GPU none can be made,
    # so the request validation is covered by the GPU tests (NaN mask, bad N, alignment)
    assert dctf.DCTF_EINVAL == -1
