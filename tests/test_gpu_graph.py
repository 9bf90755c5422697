"""GPU tests of the batched form's HIP graph, the launch parameters and the
autotuner, through the C ABI.

Every launch parameter changes speed only, so every setting must give the
same bytes as the default; a graph replay must give the bytes of the eager
batched call, on every replay, with eager work between replays, and after the
input buffer is refilled with other values of the same shapes.  The tuning
cache (CR_TUNE_CACHE) records the autotuner's choice and serves it to a fresh
context's call of the same key only.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2005_12692_amd as cr
import synth
from test_gpu_parity import assert_same

pytestmark = pytest.mark.gpu

FIELDS = ("dim", "birth", "death", "birth_pixel", "death_pixel")


def host(d):
    return [getattr(d, f).cpu().numpy() for f in FIELDS] + [d.pair_offsets.cpu().numpy()]


def same_batch(a, b, label):
    assert np.array_equal(a[5], b[5]), f"{label}: pair offsets differ"
    assert_same(a[:5], b[:5], label)


def images_2d():
    rng = np.random.default_rng(7)
    imgs = [synth.uniform2d((int(rng.integers(3, 70)), int(rng.integers(3, 70))), s) for s in range(6)]
    imgs += [synth.grf_seeded((40, 33), 2.0, 3), np.zeros((1, 1), np.float32)]
    return imgs


def volumes_3d():
    return [synth.grf_seeded((12, 13, 11), 1.5, 1), synth.blobs3d(20, 3), synth.grf_seeded((9, 16, 7), 1.0, 2)]


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_graph_replays_match_eager(kind):
    imgs = images_2d() if kind == "2d" else volumes_3d()
    ts = [torch.from_numpy(i).cuda() for i in imgs]
    packed, shapes, offs = cr.pack(ts)
    want = host(cr.persistence_batched(packed, shapes, offs))
    g = cr.BatchedGraph(packed, shapes, offs)
    try:
        for rep in range(3):
            g.launch()
            got = host(g.result())
            same_batch(got, want, f"{kind} replay {rep}")
            # eager work between replays
            cr.persistence(ts[rep % len(ts)])
            torch.cuda.synchronize()
        # new values, same shapes: refill the captured input buffer in place
        imgs2 = [(i * -1.0 + 0.5).astype(np.float32) for i in imgs]
        packed.copy_(torch.cat([torch.from_numpy(i).cuda().reshape(-1) for i in imgs2]))
        g.launch()
        got = host(g.result())
        want2 = host(cr.persistence_batched(packed, shapes, offs))
        same_batch(got, want2, f"{kind} refilled")
        # and the per-image rows equal the oracle's
        po = want2[5]
        for i, img in enumerate(imgs2[:3]):
            o = oracle.persistence(img)
            rows = [x[po[i]:po[i + 1]] for x in want2[:5]]
            rows[3] = rows[3] - offs[i]
            rows[4] = np.where(rows[4] >= 0, rows[4] - offs[i], -1)
            assert_same(rows, [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel], f"{kind} oracle {i}")
    finally:
        g.close()


@pytest.mark.parametrize("ndim", [2, 3])
def test_every_tuning_gives_the_same_bytes(ndim):
    imgs = images_2d() if ndim == 2 else volumes_3d()
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in imgs])
    default = cr.get_tuning(ndim)
    want = host(cr.persistence_batched(packed, shapes, offs))
    settings = [dict(tile=v) for v in range(len(cr.tile_shapes(ndim)))]
    settings += [dict(grid=64), dict(grid=100), dict(grid=8192)]  # 100: not a multiple of the 8 XCDs
    if ndim == 3:
        settings += [dict(long_len=0, yield_iters=1, front_cap=128), dict(long_len=1000000, yield_iters=1000000),
                     dict(wave_short=0, front_cap=300), dict(wave_yield=0), dict(wave_yield=1, yield_iters=1)]
    try:
        for kw in settings:
            cr.set_tuning(ndim, **{**default, **kw})
            same_batch(host(cr.persistence_batched(packed, shapes, offs)), want, f"ndim {ndim} {kw}")
            # the plain call too
            d = cr.persistence(torch.from_numpy(imgs[0]).cuda())
            o = oracle.persistence(imgs[0])
            assert_same([t.cpu().numpy() for t in d], [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel],
                        f"plain ndim {ndim} {kw}")
    finally:
        cr.set_tuning(ndim, **default)


def test_set_tuning_rejects_out_of_range():
    default = cr.get_tuning(3)
    for kw in (dict(tile=99), dict(grid=1), dict(front_cap=64), dict(front_cap=4096), dict(yield_iters=0)):
        with pytest.raises(cr.CRError) as e:
            cr.set_tuning(3, **kw)
        assert e.value.code == cr.CR_ERR_INVALID_ARGUMENT
    assert cr.get_tuning(3) == default


@pytest.mark.parametrize("ndim", [2, 3])
def test_autotune_keeps_results(ndim):
    imgs = images_2d() if ndim == 2 else volumes_3d()
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in imgs])
    default = cr.get_tuning(ndim)
    want = host(cr.persistence_batched(packed, shapes, offs))
    try:
        chosen = cr.autotune(packed, shapes, offs, repeats=1)
        assert chosen == cr.get_tuning(ndim)
        assert 0 <= chosen["tile"] < len(cr.tile_shapes(ndim))
        same_batch(host(cr.persistence_batched(packed, shapes, offs)), want, f"after autotune {chosen}")
    finally:
        cr.set_tuning(ndim, **default)


def _fresh_context():
    import ctypes
    h = ctypes.c_void_p()
    assert cr.lib().cr_create(ctypes.byref(h), torch.cuda.current_device(), cr._ALLOC_FN(0), cr._FREE_FN(0),
                              None) == cr.CR_OK
    return h


def _batched_on(h, packed, shapes, offs, maxdim):
    import ctypes
    ndim = len(shapes[0])
    flat = [e for s in shapes for e in s]
    out = cr._empty_out(int(offs[-1]), len(shapes), packed.device)
    rc = cr.lib().cr_persistence_batched(h, len(shapes), ctypes.c_void_p(packed.data_ptr()),
                                         (ctypes.c_int64 * len(offs))(*offs), (ctypes.c_int64 * len(flat))(*flat),
                                         ndim, maxdim, 0, cr._stream(packed.device), *cr._out_args(out))
    assert rc == cr.CR_OK, cr.lib().cr_last_error()
    assert cr.lib().cr_sync_status(h, cr._stream(packed.device)) == cr.CR_OK
    st = cr._Stats()
    assert cr.lib().cr_get_stats(h, ctypes.byref(st)) == cr.CR_OK
    n = int(out.pair_offsets[-1])
    return [getattr(out, f)[:n].cpu().numpy() for f in FIELDS] + [out.pair_offsets.cpu().numpy()], st


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    """CR_TUNE_CACHE: the autotuner records its choice under the call's key, a
    fresh context's batched call of the same key runs with it (same bytes), a
    call of another key or after cr_set_tuning does not."""
    import ctypes
    import json
    import math
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CR_TUNE_CACHE", str(path))
    imgs = images_2d()
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in imgs])
    want = host(cr.persistence_batched(packed, shapes, offs))
    h = _fresh_context()
    try:
        out = cr._empty_out(int(offs[-1]), len(imgs), packed.device)
        flat = [e for s in shapes for e in s]
        t = cr._Tuning()
        rc = cr.lib().cr_autotune_batched(h, len(imgs), ctypes.c_void_p(packed.data_ptr()),
                                          (ctypes.c_int64 * len(offs))(*offs), (ctypes.c_int64 * len(flat))(*flat),
                                          2, 1, cr._stream(packed.device), *cr._out_args(out), 1, ctypes.byref(t))
        assert rc == cr.CR_OK, cr.lib().cr_last_error()
    finally:
        cr.lib().cr_destroy(h)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/nd2/md1/img{math.ceil(math.log2(len(imgs)))}/px{math.ceil(math.log2(int(offs[-1])))}"
    entries = json.loads(path.read_text())
    assert entries[key] == [int(getattr(t, f)) for f in cr.TUNING_FIELDS]
    h = _fresh_context()
    try:
        got, st = _batched_on(h, packed, shapes, offs, 1)
        assert st.tuning_from_cache == 1
        same_batch(got, want, "with the cached tuning")
        small = [i[:5, :6].copy() for i in imgs[:2]]
        p2, s2, o2 = cr.pack([torch.from_numpy(i).cuda() for i in small])
        _, st = _batched_on(h, p2, s2, o2, 1)
        assert st.tuning_from_cache == 0, "another key used the entry"
        cur = cr._Tuning()
        assert cr.lib().cr_get_tuning(h, 2, ctypes.byref(cur)) == cr.CR_OK
        assert cr.lib().cr_set_tuning(h, 2, ctypes.byref(cur)) == cr.CR_OK
        got, st = _batched_on(h, packed, shapes, offs, 1)
        assert st.tuning_from_cache == 0, "the cache overrode cr_set_tuning"
        same_batch(got, want, "after cr_set_tuning")
    finally:
        cr.lib().cr_destroy(h)
