"""The C-ABI boundary, checked on the CPU (no GPU compute).

* libcr.so loads and exports every function that include/cr.h declares;
* the product path refuses to fall back: without a GPU, or without the
  library, calls raise instead of computing anything on the CPU;
* the package does not import the oracle.
"""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cr.h")
LIB = os.path.join(ROOT, "paper_2005_12692_amd", "libcr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(cr_[a-z_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


@pytest.fixture(scope="module")
def libcr():
    if not os.path.exists(LIB):
        from paper_2005_12692_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("cr_persistence", "cr_persistence_batched", "cr_persistence_backward",
                     "cr_create", "cr_destroy", "cr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(libcr):
    missing = [n for n in declared_functions() if not hasattr(libcr, n)]
    assert not missing, missing


def test_last_error_is_a_string(libcr):
    libcr.cr_last_error.restype = ctypes.c_char_p
    assert isinstance(libcr.cr_last_error(), bytes)


def test_create_rejects_bad_arguments(libcr):
    libcr.cr_create.restype = ctypes.c_int
    # NULL out pointer: rejected before any device call
    assert libcr.cr_create(None, 0, None, None, None) == 1
    # only one of alloc/free given
    h = ctypes.c_void_p()
    fn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)(lambda *a: None)
    assert libcr.cr_create(ctypes.byref(h), 0, fn, None, None) == 1


def test_null_context_calls_fail_cleanly(libcr):
    libcr.cr_persistence.restype = ctypes.c_int
    assert libcr.cr_persistence(None, None, 2, None, 1, 0, None, None) == 1
    libcr.cr_persistence_backward.restype = ctypes.c_int
    assert libcr.cr_persistence_backward(None, None, None, None, None, 0, None, 0, None) == 1
    libcr.cr_lifetime_image.restype = ctypes.c_int
    assert libcr.cr_lifetime_image(None, None, None, None, None, None, 0, 0, None, 0, None) == 1
    libcr.cr_pixel_coords.restype = ctypes.c_int
    assert libcr.cr_pixel_coords(None, None, 0, 0, 2, None, None, None) == 1
    libcr.cr_batched_workspace_size.restype = ctypes.c_int
    assert libcr.cr_batched_workspace_size(None, 1, None, 2, 1, None) == 1
    libcr.cr_reserve.restype = ctypes.c_int
    assert libcr.cr_reserve(None, ctypes.c_size_t(0)) == 1


def test_package_does_not_import_the_oracle():
    code = ("import sys; sys.path.insert(0, %r); import paper_2005_12692_amd; "
            "assert 'oracle' not in sys.modules; print('ok')" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert out.returncode == 0 and "ok" in out.stdout, out.stderr
    src = open(os.path.join(ROOT, "paper_2005_12692_amd", "__init__.py")).read()
    assert "oracle" not in src


def test_no_gpu_means_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2005_12692_amd as cr
    with pytest.raises(Exception):
        cr.persistence(torch.rand(8, 8))  # CPU tensor: refused


def test_tile_shapes_and_null_handles(libcr):
    """Host-only entry points: tile shapes, and NULL handles rejected."""
    libcr.cr_tile_variants.restype = ctypes.c_int
    libcr.cr_tile_shape.restype = ctypes.c_int
    for ndim in (2, 3):
        n = libcr.cr_tile_variants(ndim)
        assert n >= 1
        for v in range(n):
            e = (ctypes.c_int32 * 3)()
            assert libcr.cr_tile_shape(ndim, v, e) == 0
            assert min(e) >= 1 and (ndim == 3 or e[0] == 1)
        e = (ctypes.c_int32 * 3)()
        assert libcr.cr_tile_shape(ndim, n, e) == 1
    assert libcr.cr_tile_variants(4) == 0
    for f in ("cr_graph_launch", "cr_graph_sync_status"):
        getattr(libcr, f).restype = ctypes.c_int
        assert getattr(libcr, f)(None, None) == 1
    libcr.cr_get_tuning.restype = ctypes.c_int
    assert libcr.cr_get_tuning(None, 3, None) == 1
    libcr.cr_graph_destroy(None)  # a no-op


def test_workspace_size_without_a_context(libcr):
    """cr_batched_workspace_size with ctx = NULL is host-only: it sizes a batch,
    and reports CR_ERR_TOO_LARGE for an image of 2^30 cells or more and for a
    batch whose keys would not fit 64 bits."""
    f = libcr.cr_batched_workspace_size
    f.restype = ctypes.c_int
    out = ctypes.c_size_t(7)
    sh = (ctypes.c_int64 * 2)(64, 64)
    assert f(None, 1, sh, 2, 1, ctypes.byref(out)) == 0
    small = out.value
    assert small > 0
    sh2 = (ctypes.c_int64 * 4)(64, 64, 128, 64)
    assert f(None, 2, sh2, 2, 1, ctypes.byref(out)) == 0 and out.value > small
    # (2 * 600 - 1)^3 = 1.72e9 cells >= 2^30
    big = (ctypes.c_int64 * 3)(600, 600, 600)
    out.value = 7
    assert f(None, 1, big, 3, 2, ctypes.byref(out)) == 3
    assert out.value == 0
    assert b"2^30" in libcr.cr_last_error()
    # one extent beyond 2^29
    huge = (ctypes.c_int64 * 2)(1, (1 << 29) + 1)
    assert f(None, 1, huge, 2, 1, ctypes.byref(out)) == 3
    # 2^16 images of 128 x 64: image field 16 bits + 2 + 32 + 15-bit index > 64
    n = 1 << 16
    many = (ctypes.c_int64 * (2 * n))(*([128, 64] * n))
    assert f(None, n, many, 2, 1, ctypes.byref(out)) == 3
    # bad arguments stay INVALID_ARGUMENT
    assert f(None, 1, sh, 4, 1, ctypes.byref(out)) == 1
    assert f(None, 0, sh, 2, 1, ctypes.byref(out)) == 1
