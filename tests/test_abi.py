"""The C-ABI library loads and exports every symbol include/lkc.h declares.

No compute calls: these run on a machine without a GPU.  Calls that must
fail before touching a device (NULL context, missing device) are exercised.
"""
import ctypes
import os
import re

import pytest

from paper_2308_07173_amd import lkc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lkc.LIB_PATH):
        from paper_2308_07173_amd import build_lib
        build_lib.build()
    return lkc.load_library()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lkc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lkc_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(lkc.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_version(lib):
    assert lib.lkc_version() == 100


def test_null_context_is_rejected(lib):
    P = ctypes.c_void_p
    st = lib.lkc_knn_query(None, None, None, 0, 5, 1.0, None, None, None, None)
    assert st == lkc.LKC_ERR_INVALID_ARG
    assert b"ctx" in lib.lkc_last_error(None)
    st = lib.lkc_build_target(None, None, 0, 1.0, ctypes.byref(P()))
    assert st == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_target_free(None, None) == lkc.LKC_OK
    assert lib.lkc_ctx_destroy(None) == lkc.LKC_OK


def test_ctx_create_without_gpu_fails_cleanly(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = lib.lkc_ctx_create(None, ctypes.byref(h))
    assert st == lkc.LKC_ERR_UNSUPPORTED and not h.value


def test_raceline_and_async_calls_reject_null_arguments(lib):
    P = ctypes.c_void_p
    assert lib.lkc_target_rebuild_async(None, None, None, 0) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_raceline_build(None, None, None, 0, 1.0, 1.0, 1.0,
                                  ctypes.byref(P())) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_raceline_get_info(None, None) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_raceline_bins(None, None, None) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_submap_window(None, None, None, 1.0, None, None, 0,
                                 None) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_submap_window_build(None, None, None, 1.0, None, 0, None,
                                       None) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_raceline_free(None, None) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_voxel_filter_async(None, None, 0, None, 0.5, 4, None, None, None, 0, None,
                                      None) == lkc.LKC_ERR_INVALID_ARG
    assert lib.lkc_euclid_cluster_async(None, None, 0, 0.5, None, None, None,
                                        None) == lkc.LKC_ERR_INVALID_ARG


def test_struct_layouts():
    assert ctypes.sizeof(lkc.RaceLineInfo) == 8 * 5 + 4 * 5 + 4 + 8
    assert lkc.RaceLineInfo.device_bytes.offset == 64
    assert ctypes.sizeof(lkc.LaunchCfg) == 24
    assert ctypes.sizeof(lkc.ScanDesc) == 24
    assert ctypes.sizeof(lkc.GicpStats) == 4 + 4 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(lkc.TargetInfo) == 8 * 3 + 4 * 6 + 4 * 3 + 4 + 8
    assert ctypes.sizeof(lkc.AutotuneResult) == 4 + 4 + 24 + 4 + 4 + 8
    assert lkc.AutotuneResult.sample.offset == 40
