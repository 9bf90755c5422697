"""GPU tests of cr_persistence_batched_noalloc, the batched call on the
library's static device scratch, through the C ABI (ctypes).

Its results must be the bytes of cr_persistence_batched on the same batch
(dim, birth, death, both pixel arrays, pair offsets and per-image status), on
two calls in a row of which the second is smaller (the static array keeps the
first call's contents).  A fresh context that only makes allocation-free calls
owns no scratch afterwards, the caller's allocator is never asked for memory,
and a batch larger than the array is refused before any device work.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2005_12692_amd as cr
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("dim", "birth", "death", "birth_pixel", "death_pixel", "pair_offsets", "status")


def fresh_context():
    h = ctypes.c_void_p()
    rc = cr.lib().cr_create(ctypes.byref(h), torch.cuda.current_device(), cr._ALLOC_FN(0), cr._FREE_FN(0), None)
    assert rc == cr.CR_OK, cr.lib().cr_last_error()
    return h


def call_noalloc(h, packed, shapes, offs, maxdim, out):
    """One cr_persistence_batched_noalloc call on context h; returns its status."""
    ndim = len(shapes[0])
    flat = [e for s in shapes for e in s]
    c_shapes = (ctypes.c_int64 * len(flat))(*flat)
    c_offs = (ctypes.c_int64 * len(offs))(*offs)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = cr.lib().cr_persistence_batched_noalloc(h, len(shapes), ctypes.c_void_p(packed.data_ptr()), c_offs,
                                                 c_shapes, ndim, maxdim, 0, stream, *cr._out_args(out))
    torch.cuda.synchronize()
    return rc


def host(d, n=None):
    n = int(d.pair_offsets[-1]) if n is None else n
    rows = [getattr(d, f)[:n].cpu().numpy() for f in FIELDS[:5]]
    return rows + [d.pair_offsets.cpu().numpy(), d.status.cpu().numpy()]


def assert_same_bytes(got, want, label):
    for f, a, b in zip(FIELDS, got, want):
        assert a.shape == b.shape, f"{label}: {f} has {a.shape} rows, expected {b.shape}"
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{label}: {f} differs"


def batches(kind):
    if kind == "3d":
        big = [synth.grf_seeded((12, 13, 11), 1.5, 1), synth.blobs3d(20, 3), synth.grf_seeded((9, 16, 7), 1.0, 2)]
        small = [synth.grf_seeded((8, 9, 10), 1.0, 5), synth.grf_seeded((6, 6, 6), 0.7, 6)]
        return big, small, 2
    rng = np.random.default_rng(11)
    big = [synth.uniform2d((int(rng.integers(3, 90)), int(rng.integers(3, 90))), s) for s in range(7)]
    big += [synth.grf_seeded((64, 57), 2.0, 3), np.zeros((1, 1), np.float32)]
    small = [synth.uniform2d((5, 9), 20), synth.grf_seeded((17, 12), 1.5, 21)]
    return big, small, 1


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_noalloc_matches_batched_on_two_calls(kind):
    big, small, maxdim = batches(kind)
    h = fresh_context()
    try:
        for label, imgs in (("first call", big), ("second, smaller call", small)):
            ts = [torch.from_numpy(i).cuda() for i in imgs]
            packed, shapes, offs = cr.pack(ts)
            want_d = cr.persistence_batched(packed, shapes, offs, maxdim=maxdim)
            want = host(want_d)
            cap = int(offs[-1])
            out = cr._empty_out(cap, len(imgs), packed.device)
            # poison the outputs so stale bytes cannot pass
            for f in FIELDS:
                getattr(out, f).fill_(-7)
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            rc = call_noalloc(h, packed, shapes, offs, maxdim, out)
            assert rc == cr.CR_OK, cr.lib().cr_last_error()
            assert torch.cuda.memory_allocated() == before
            assert cr.lib().cr_sync_status(h, None) == cr.CR_OK, cr.lib().cr_last_error()
            assert_same_bytes(host(out), want, f"{kind} {label}")
        st = cr._Stats()
        assert cr.lib().cr_get_stats(h, ctypes.byref(st)) == cr.CR_OK
        assert st.scratch_bytes == 0, "the allocation-free call made the context allocate scratch"
        assert st.n_pixels == sum(int(np.prod(i.shape)) for i in small)
    finally:
        cr.lib().cr_destroy(h)


def test_noalloc_interleaved_with_batched_contexts():
    """The static array and a context's own scratch do not disturb each other:
    allocation-free calls before and after a plain batched call on the shared
    context give the same bytes."""
    big, small, maxdim = batches("2d")
    ts = [torch.from_numpy(i).cuda() for i in big]
    packed, shapes, offs = cr.pack(ts)
    h = fresh_context()
    try:
        outs = []
        for _ in range(2):
            out = cr._empty_out(int(offs[-1]), len(big), packed.device)
            rc = call_noalloc(h, packed, shapes, offs, maxdim, out)
            assert rc == cr.CR_OK, cr.lib().cr_last_error()
            outs.append(host(out))
            cr.persistence_batched(*cr.pack([torch.from_numpy(i).cuda() for i in small]), maxdim=maxdim)
        assert_same_bytes(outs[1], outs[0], "allocation-free call after a batched call")
    finally:
        cr.lib().cr_destroy(h)


def test_noalloc_refuses_a_batch_beyond_the_array():
    img = synth.uniform2d((2048, 2048), 0)  # about 350 MB of scratch
    t = torch.from_numpy(img).cuda()
    h = fresh_context()
    try:
        out = cr._empty_out(16, 1, t.device)
        out.pair_offsets.fill_(-7)
        torch.cuda.synchronize()
        rc = call_noalloc(h, t, [tuple(img.shape)], [0, img.size], 1, out)
        assert rc == cr.CR_ERR_TOO_LARGE
        assert b"static scratch" in cr.lib().cr_last_error()
        assert (out.pair_offsets.cpu() == -7).all(), "a refused call wrote its outputs"
    finally:
        cr.lib().cr_destroy(h)
