"""Error paths and the plain call's recovery paths, on the GPU, through the C ABI.

* the column arena of the degree-1 reduction overflows on purpose (a tiny
  first arena through CR_ARENA_ENTRIES): the plain call reruns the whole
  pipeline -- degree 0 on its side stream included -- with a larger arena and
  returns the oracle's diagram;
* an allocator callback that returns NULL for the output block gives
  CR_ERR_OUT_OF_MEMORY with out->n == 0 and nothing allocated;
* NaN anywhere gives CR_ERR_NAN_INPUT.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

import paper_2005_12692_amd as cr
import synth
from test_gpu_parity import check, gpu_diag, oracle_diag, assert_same

pytestmark = pytest.mark.gpu


def test_arena_overflow_reruns_with_a_larger_arena():
    vol = synth.blobs3d(40, 5)
    cr.persistence(torch.from_numpy(vol).cuda())
    used = cr.stats()["arena_used"]
    assert used > 64
    before = cr.stats()["arena_reruns"]
    try:
        # a quarter of the need: the first attempt overflows; 4x growth per rerun
        os.environ["CR_ARENA_ENTRIES"] = str(max(16, used // 4))
        got = gpu_diag(vol)
        reruns = cr.stats()["arena_reruns"] - before
    finally:
        os.environ.pop("CR_ARENA_ENTRIES", None)
    assert reruns >= 1
    assert_same(got, oracle_diag(vol), "40^3 blobs after an arena rerun")
    # a later call without the override runs once
    before = cr.stats()["arena_reruns"]
    check(vol, label="40^3 blobs, default arena")
    assert cr.stats()["arena_reruns"] == before


def test_allocator_returning_null_is_out_of_memory():
    L = cr.lib()
    alloc = cr._ALLOC_FN(lambda n, s, u: None)
    free = cr._FREE_FN(lambda p, s, u: None)
    h = ctypes.c_void_p()
    assert L.cr_create(ctypes.byref(h), torch.cuda.current_device(), alloc, free, None) == cr.CR_OK
    try:
        img = torch.from_numpy(synth.uniform2d((50, 40), 1)).cuda()
        shape = (ctypes.c_int64 * 2)(50, 40)
        out = cr._Diagram()
        out.n = 123
        rc = L.cr_persistence(h, ctypes.c_void_p(img.data_ptr()), 2, shape, 1, 0,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(out))
        assert rc == cr.CR_ERR_OUT_OF_MEMORY, L.cr_last_error()
        assert out.n == 0 and not out.block
        assert b"output allocation" in L.cr_last_error()
    finally:
        L.cr_destroy(h)


@pytest.mark.parametrize("shape", [(17, 23), (9, 10, 11)])
def test_nan_is_an_error(shape):
    img = synth.uniform2d((17, 23), 2) if len(shape) == 2 else synth.grf_seeded(shape, 1.5, 2)
    img = img.copy()
    img.flat[img.size // 3] = np.nan
    with pytest.raises(cr.CRError) as e:
        cr.persistence(torch.from_numpy(img).cuda())
    assert e.value.code == cr.CR_ERR_NAN_INPUT
