"""GPU tests of the batched form and of differentiation, through the C ABI.

* batched: many images of different shapes in one call, every image's rows
  byte-equal to the oracle's diagram of that image (pixel indices shifted by the
  image's offset in the packed buffer) and to the plain call;
* backward: grad_image[p] = sum of dL/dbirth over bars born at p plus sum of
  dL/ddeath over bars dying at p, checked against the oracle's pixel map, and
  against central finite differences on inputs without ties near the probed
  voxels.
"""
import concurrent.futures as cf
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2005_12692_amd as cr
import synth
from test_gpu_parity import assert_same

pytestmark = pytest.mark.gpu


def oracle_rows(img, maxdim=None, offset=0):
    o = oracle.persistence(img, maxdim)
    bp = o.birth_pixel + offset
    dp = np.where(o.death_pixel >= 0, o.death_pixel + offset, -1)
    return [o.dim, o.birth, o.death, bp, dp]


def run_batched(images, maxdim=None):
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in images])
    d = cr.persistence_batched(packed, shapes, offs, maxdim=maxdim)
    po = d.pair_offsets.cpu().numpy()
    host = [t.cpu().numpy() for t in (d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel)]
    return host, po, offs, d


def assert_grad(got, pix, contrib, n, what=""):
    """Gradient bar for fp32 sums: |g - ref| <= 1e-6 * max(|ref|, sum |c|) at
    every pixel, where ref is the float64 sum of the contributions c placed at
    that pixel (births and deaths at one pixel can cancel, so the bar is
    relative to the magnitude of the terms summed, not only to their sum).  A
    pixel with no contribution must be exactly 0."""
    pix = np.asarray(pix, np.int64)
    c = np.asarray(contrib, np.float64)
    ref = np.zeros(n, np.float64)
    mag = np.zeros(n, np.float64)
    np.add.at(ref, pix, c)
    np.add.at(mag, pix, np.abs(c))
    g = np.asarray(got, np.float64).ravel()
    bound = 1e-6 * np.maximum(np.abs(ref), mag)
    bad = np.nonzero(np.abs(g - ref) > bound)[0]
    assert bad.size == 0, (what, int(bad[0]), g[bad[0]], ref[bad[0]], mag[bad[0]])


def check_batched(images, maxdim=None, workers=8):
    host, po, offs, d = run_batched(images, maxdim)
    assert int((d.status != 0).sum()) == 0
    with cf.ThreadPoolExecutor(workers) as ex:
        wants = list(ex.map(lambda a: oracle_rows(a[1], maxdim, offs[a[0]]), enumerate(images)))
    for i, want in enumerate(wants):
        got = [x[po[i]:po[i + 1]] for x in host]
        assert_same(got, want, f"image {i} shape {images[i].shape}")
    return host, po, offs


def test_batched_2d_mixed():
    imgs = synth.config("C4", small=True)
    imgs += [np.full((5, 7), 2.0, np.float32), np.zeros((1, 1), np.float32),
             synth.uniform2d((3, 40), 9)]
    host, po, offs = check_batched(imgs)
    # the batched rows equal the plain call's rows, shifted by the image offset
    for i, img in enumerate(imgs[:6]):
        d = cr.persistence(torch.from_numpy(img).cuda())
        plain = [t.cpu().numpy() for t in d]
        plain[3] = plain[3] + offs[i]
        plain[4] = np.where(plain[4] >= 0, plain[4] + offs[i], -1)
        assert_same([x[po[i]:po[i + 1]] for x in host], plain, f"plain vs batched {i}")


def test_batched_3d_mixed():
    vols = synth.config("C5", small=True) + [synth.blobs3d(20, 8), synth.grf_seeded((7, 9, 5), 1.0, 2)]
    check_batched(vols)
    check_batched(vols, maxdim=1)


def test_batched_nan_status_and_capacity():
    imgs = [synth.uniform2d((10, 12), 1), synth.uniform2d((9, 9), 2)]
    imgs[1][4, 4] = np.nan
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in imgs])
    with pytest.raises(cr.CRError) as e:
        cr.persistence_batched(packed, shapes, offs)
    assert e.value.code == cr.CR_ERR_NAN_INPUT
    # a too-small capacity is reported through pair_offsets and retried by the binding
    imgs = [synth.uniform2d((30, 30), 3), synth.uniform2d((20, 25), 4)]
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in imgs])
    d = cr.persistence_batched(packed, shapes, offs, capacity=5)
    want = sum(len(oracle.persistence(i)) for i in imgs)
    assert d.dim.shape[0] == want


def test_backward_pixel_map():
    img = synth.uniform2d((40, 37), 5)
    x = torch.from_numpy(img).cuda().requires_grad_(True)
    dim, birth, death, bp, dp = cr.PersistenceFn.apply(x)
    fin = torch.isfinite(death)
    w = torch.arange(birth.shape[0], device="cuda", dtype=torch.float32) * 0.25 + 1.0
    loss = (w[fin] * (death[fin] - birth[fin]) ** 2).sum() + birth[~fin].sum()
    loss.backward()
    o = oracle.persistence(img)
    wn = np.arange(len(o), dtype=np.float64) * 0.25 + 1.0
    f = o.death_pixel >= 0
    life = o.death.astype(np.float64) - o.birth.astype(np.float64)
    pix = np.concatenate([o.death_pixel[f], o.birth_pixel[f], o.birth_pixel[~f]])
    c = np.concatenate([(2 * wn * life)[f], (-2 * wn * life)[f], np.ones(int((~f).sum()))])
    assert_grad(x.grad.cpu().numpy(), pix, c, img.size, "pixel map")


def _loss_terms(vol, thr=0.1):
    """Terms of L = sum over finite degree-1/2 bars with lifetime > thr of lifetime^2,
    from the oracle.  Activity is decided in float32 (as the GPU loss does); the
    terms use the exact float64 difference of the two float32 end points."""
    o = oracle.persistence(vol)
    life32 = (o.death - o.birth).astype(np.float32)
    act = (o.dim >= 1) & (o.death_pixel >= 0) & (life32 > np.float32(thr))
    life64 = o.death.astype(np.float64) - o.birth.astype(np.float64)
    return [float(l) * float(l) for l in life64[act]], o, act


def test_backward_finite_differences():
    """dL/dvoxel against central differences on voxels whose neighbourhood of
    values and whose active lifetimes are free of ties within the step."""
    vol = synth.grf_seeded((14, 15, 13), 1.5, 11)
    x = torch.from_numpy(vol).cuda().requires_grad_(True)
    dim, birth, death, bp, dp = cr.PersistenceFn.apply(x)
    life = death - birth
    act = (dim >= 1) & torch.isfinite(death) & (life > 0.1)
    loss = (life[act] ** 2).sum()
    loss.backward()
    g = x.grad.cpu().numpy().ravel()
    terms0, o, act0 = _loss_terms(vol)
    rng = np.random.default_rng(104)
    cand = np.unique(np.concatenate([o.birth_pixel[act0], o.death_pixel[act0]]))
    picks = list(rng.choice(cand, min(12, len(cand)), replace=False)) + list(rng.integers(0, vol.size, 4))
    flat = vol.ravel()
    checked = 0
    for p in picks:
        v = np.float32(flat[p])
        h = np.float32(2) * np.spacing(v) if v != 0 else np.float32(1e-6)
        others = np.delete(flat, p)
        if np.min(np.abs(others - v)) <= 3 * h:
            continue
        lifes = (o.death - o.birth).astype(np.float32)[act0]
        if np.any(np.abs(lifes - np.float32(0.1)) <= 3 * h):
            continue
        plus = vol.copy().ravel()
        minus = vol.copy().ravel()
        plus[p] = v + h
        minus[p] = v - h
        tp, _, _ = _loss_terms(plus.reshape(vol.shape))
        tm, _, _ = _loss_terms(minus.reshape(vol.shape))
        fd = math.fsum(tp + [-t for t in tm]) / (float(plus[p]) - float(minus[p]))
        # the bar relative to the magnitude of the fp32 sum's terms at p
        life64 = (o.death.astype(np.float64) - o.birth.astype(np.float64))
        contrib = np.sum(np.abs(2 * life64[act0 & ((o.birth_pixel == p) | (o.death_pixel == p))]))
        if fd == 0.0 and contrib == 0.0:
            assert g[p] == 0.0, (p, g[p])
        else:
            assert abs(g[p] - fd) <= 1e-6 * max(abs(fd), contrib), (p, g[p], fd, contrib)
        checked += 1
    assert checked >= 8


def test_batched_backward_matches_plain():
    vols = [synth.grf_seeded((12, 12, 12), 1.5, s) for s in range(3)]
    ts = [torch.from_numpy(v).cuda() for v in vols]
    packed, shapes, offs = cr.pack(ts)
    packed = packed.clone().requires_grad_(True)
    dim, birth, death, bp, dp, po = cr.PersistenceBatchedFn.apply(packed, shapes)
    life = death - birth
    act = torch.isfinite(death)
    (life[act] ** 2).sum().backward()
    gb = packed.grad.cpu().numpy()
    for i, v in enumerate(ts):
        x = v.clone().requires_grad_(True)
        d, b, e, _, _ = cr.PersistenceFn.apply(x)
        l = e - b
        a = torch.isfinite(e)
        (l[a] ** 2).sum().backward()
        # both against the float64 sums of the oracle's rows
        o = oracle.persistence(vols[i])
        f = o.death_pixel >= 0
        life = o.death[f].astype(np.float64) - o.birth[f].astype(np.float64)
        pix = np.concatenate([o.death_pixel[f], o.birth_pixel[f]])
        c = np.concatenate([2 * life, -2 * life])
        assert_grad(gb[offs[i]:offs[i + 1]], pix, c, vols[i].size, f"batched volume {i}")
        assert_grad(x.grad.cpu().numpy(), pix, c, vols[i].size, f"plain volume {i}")


def test_batched_yield_within_the_round_budget():
    """Wave columns stored and resumed after every addition: the batched call
    (a fixed budget of rounds, no host checks) still finishes and matches the
    oracle, because columns yield only in the first part of the budget."""
    import os
    vols = [synth.grf_seeded((20, 22, 18), 1.5, 30 + i) for i in range(5)] + [synth.blobs3d(24, 9)]
    packed, shapes, offs = cr.pack([torch.from_numpy(v).cuda() for v in vols])
    try:
        for y in ("1", "4"):
            os.environ["CR_WAVE_YIELD"] = y
            os.environ["CR_LONG_LEN"] = "0"
            os.environ["CR_YIELD_ITERS"] = "1"
            d = cr.persistence_batched(packed, shapes, offs)
            po = d.pair_offsets.cpu()
            for i, v in enumerate(vols):
                got = [t.cpu().numpy() for t in d.image(i, po)]
                got[3] = got[3] - offs[i]
                got[4] = np.where(got[4] >= 0, got[4] - offs[i], -1)
                o = oracle.persistence(v)
                assert_same(got, [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel], f"yield {y} volume {i}")
    finally:
        for k in ("CR_WAVE_YIELD", "CR_LONG_LEN", "CR_YIELD_ITERS"):
            os.environ.pop(k, None)


def test_reserve_then_batched_call_allocates_nothing():
    """cr_batched_workspace_size / cr_reserve: after reserving the reported
    scratch, a batched call into preallocated outputs takes no device memory."""
    imgs = [synth.uniform2d((40 + 3 * i, 50 - 2 * i), i) for i in range(8)]
    packed, shapes, offs = cr.pack([torch.from_numpy(a).cuda() for a in imgs])
    need = cr.workspace_size(shapes)
    assert need > 0
    assert cr.workspace_size(shapes + shapes) > need  # more images, more scratch
    cr.reserve(need)
    out = cr._empty_out(int(offs[-1]), len(imgs), packed.device)
    cr.persistence_batched(packed, shapes, offs, out=out, check=False)  # first call: host staging
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    d = cr.persistence_batched(packed, shapes, offs, out=out, check=False)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    po = d.pair_offsets.cpu()
    for i in (0, 5):
        got = [t.cpu().numpy() for t in d.image(i, po)]
        got[3] = got[3] - offs[i]
        got[4] = np.where(got[4] >= 0, got[4] - offs[i], -1)
        o = oracle.persistence(imgs[i])
        assert_same(got, [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel], f"reserved image {i}")
