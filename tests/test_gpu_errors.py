"""Error paths and the plain call's recovery paths, on the GPU, through the C ABI.

* the column arena of the degree-1 reduction overflows on purpose (a tiny
  first arena through CR_ARENA_ENTRIES): the plain call reruns the whole
  pipeline -- degree 0 on its side stream included -- with a larger arena and
  returns the oracle's diagram;
* an allocator callback that returns NULL for the output block gives
  CR_ERR_OUT_OF_MEMORY with out->n == 0 and nothing allocated;
* NaN anywhere gives CR_ERR_NAN_INPUT;
* the batched call runs a reduction that outlasts its fixed budget of rounds to
  the end (the asynchronous tail), reports an exhausted column arena for
  every image, and marks exactly the images whose rows exceed the capacity.
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


# ---- the batched form runs any batch to the end, or reports each image ----------

def _batch_volumes():
    return [synth.blobs3d(28, 7), synth.grf_seeded((20, 24, 22), 1.2, 8), synth.blobs3d(24, 9),
            synth.grf_seeded((10, 9, 12), 0.8, 10)]


def _per_image(d, offs, i):
    a, b = int(d.pair_offsets[i]), int(d.pair_offsets[i + 1])
    rows = [t[a:b].cpu().numpy() for t in (d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel)]
    rows[3] = rows[3] - offs[i]
    rows[4] = np.where(rows[4] >= 0, rows[4] - offs[i], -1)
    return rows


@pytest.mark.parametrize("budget", ["1", "3"])
def test_batched_runs_past_the_round_budget(budget, monkeypatch):
    """With a budget of one or three rounds, the asynchronous tail runs the
    rest of the reduction: every image equals the oracle's diagram, in the
    eager call and in two graph replays."""
    vols = _batch_volumes()
    ts = [torch.from_numpy(v).cuda() for v in vols]
    packed, shapes, offs = cr.pack(ts)
    want = [oracle_diag(v) for v in vols]
    monkeypatch.setenv("CR_ROUND_BUDGET", budget)
    monkeypatch.setenv("CR_YIELD_ROUNDS", "1")
    monkeypatch.setenv("CR_WAVE_YIELD", "4")  # columns yield in the budget's rounds
    d = cr.persistence_batched(packed, shapes, offs)
    assert (d.status.cpu() == 0).all()
    for i, v in enumerate(vols):
        assert_same(_per_image(d, offs, i), want[i], f"volume {i}, budget {budget}")
    g = cr.BatchedGraph(packed, shapes, offs)
    try:
        for rep in range(2):
            g.launch()
            r = g.result()
            for i in range(len(vols)):
                assert_same(_per_image(r, offs, i), want[i], f"graph replay {rep}, volume {i}, budget {budget}")
    finally:
        g.close()


def test_batched_arena_exhaustion_reports_every_image(monkeypatch):
    """A column arena far too small: the batch stops early and every image's
    status says so (no image's rows are complete); without the override the
    same batch is complete and exact."""
    vols = _batch_volumes()
    ts = [torch.from_numpy(v).cuda() for v in vols]
    packed, shapes, offs = cr.pack(ts)
    monkeypatch.setenv("CR_ARENA_ENTRIES", "64")
    d = cr.persistence_batched(packed, shapes, offs, check=False)
    torch.cuda.synchronize()
    assert (d.status.cpu() == cr.CR_ERR_OUT_OF_MEMORY).all()
    h, _ = cr._context(packed.device)
    assert cr.lib().cr_sync_status(h, cr._stream(packed.device)) == cr.CR_ERR_OUT_OF_MEMORY
    assert b"column-arena" in cr.lib().cr_last_error()
    with pytest.raises(cr.CRError) as e:  # the override pins the arena: the retries cannot help
        cr.persistence_batched(packed, shapes, offs)
    assert e.value.code == cr.CR_ERR_OUT_OF_MEMORY
    monkeypatch.delenv("CR_ARENA_ENTRIES")
    d = cr.persistence_batched(packed, shapes, offs)
    assert (d.status.cpu() == 0).all()
    for i, v in enumerate(vols):
        assert_same(_per_image(d, offs, i), oracle_diag(v), f"volume {i} after the arena failure")


def test_batched_status_marks_images_beyond_capacity():
    """Rows beyond the caller's capacity are dropped: exactly the images whose
    rows do not all fit are marked CR_ERR_CAPACITY, and the total tells the
    capacity needed."""
    imgs = [synth.uniform2d((30, 20), 1), synth.uniform2d((25, 31), 2), synth.uniform2d((12, 40), 3)]
    ts = [torch.from_numpy(i).cuda() for i in imgs]
    packed, shapes, offs = cr.pack(ts)
    full = cr.persistence_batched(packed, shapes, offs)
    po = full.pair_offsets.cpu().numpy()
    cap = int(po[1]) + 3  # image 0 fits, image 1 does not
    out = cr._empty_out(cap, len(imgs), packed.device)
    cr.persistence_batched(packed, shapes, offs, out=out, check=False)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert st[0] == 0 and st[1] == cr.CR_ERR_CAPACITY and st[2] == cr.CR_ERR_CAPACITY
    assert int(out.pair_offsets[-1]) == int(po[-1])
    got0 = [t[:int(po[1])].cpu().numpy() for t in (out.dim, out.birth, out.death, out.birth_pixel, out.death_pixel)]
    want0 = [t[:int(po[1])].cpu().numpy() for t in (full.dim, full.birth, full.death, full.birth_pixel, full.death_pixel)]
    assert_same(got0, want0, "the image that fits")
