"""The full-size workloads on the GPU against the oracle.

The oracle's diagrams of these inputs take minutes to compute, so their sha256
digests are stored in tests/golden/oracle_digests.json (written by
tests/golden/make_oracle_digests.py, which calls only the oracle and the input
generators).  Each stored entry also holds the digest of its input: if the
generated input ever differs (another BLAS, another NumPy), the test computes
the oracle live instead of trusting the stored digest.
"""
import concurrent.futures as cf
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2005_12692_amd as cr
import synth
from test_gpu_parity import assert_same
from test_gpu_forms import assert_grad

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "oracle_digests.json")


def _digests():
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_oracle_digests.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m, json.load(open(DIGESTS))


def local_rows(rows, offset):
    dim, birth, death, bp, dp = rows
    return [dim, birth, death, bp - offset, np.where(dp >= 0, dp - offset, -1)]


def check_against_oracle(img, rows, stored, m, label):
    """rows: GPU rows with pixel indices local to img."""
    if stored is not None and m.input_digest(img) == stored["input"]:
        got = m.diagram_digest(*rows)
        if got == stored["diagram"]:
            return
        assert np.bincount(rows[0], minlength=3).tolist() == stored["rows_per_dim"], label
        raise AssertionError(f"{label}: diagram digest differs from the oracle's")
    o = oracle.persistence(img)
    assert_same(rows, [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel], label)


def _invariants(img, rows):
    dim, birth, death, bp, dp = rows
    flat = img.ravel()
    ess = dp < 0
    assert ess.sum() == 1 and dim[ess][0] == 0 and birth[ess][0] == flat.min()
    assert np.all(birth[~ess] < death[~ess])
    assert np.array_equal(birth.view(np.uint32), flat[bp].view(np.uint32))
    assert np.array_equal(death[~ess].view(np.uint32), flat[dp[~ess]].view(np.uint32))


def test_volume_256():
    m, dg = _digests()
    vol = synth.config("C3")
    rows = [t.cpu().numpy() for t in cr.persistence(torch.from_numpy(vol).cuda())]
    _invariants(vol, rows)
    check_against_oracle(vol, rows, dg.get("C3"), m, "256^3 blobs")


def test_image_1024():
    m, dg = _digests()
    img = synth.config("C2")
    rows = [t.cpu().numpy() for t in cr.persistence(torch.from_numpy(img).cuda())]
    check_against_oracle(img, rows, dg.get("C2"), m, "1024^2 GRF")


def _check_batch(images, stored, m, label):
    packed, shapes, offs = cr.pack([torch.from_numpy(i).cuda() for i in images])
    d = cr.persistence_batched(packed, shapes, offs)
    po = d.pair_offsets.cpu().numpy()
    host = [t.cpu().numpy() for t in (d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel)]
    todo = []
    for i, img in enumerate(images):
        rows = local_rows([x[po[i]:po[i + 1]] for x in host], offs[i])
        todo.append((i, img, rows))

    def one(a):
        i, img, rows = a
        check_against_oracle(img, rows, stored[i] if stored else None, m, f"{label} image {i}")
    with cf.ThreadPoolExecutor(8) as ex:
        list(ex.map(one, todo))
    return d, offs


def test_batch_512_images():
    m, dg = _digests()
    _check_batch(synth.config("C4"), dg.get("C4"), m, "512 images")


def test_batch_32_volumes_forward_backward():
    m, dg = _digests()
    vols = synth.config("C5")
    _check_batch(vols, dg.get("C5"), m, "32 volumes")
    # forward + backward of L = sum over degree-1/2 bars with lifetime > 0.1 of lifetime^2
    packed, shapes, offs = cr.pack([torch.from_numpy(v).cuda() for v in vols])
    packed = packed.clone().requires_grad_(True)
    dim, birth, death, bp, dp, po = cr.PersistenceBatchedFn.apply(packed, shapes)
    life = death - birth
    act = (dim >= 1) & torch.isfinite(death) & (life > 0.1)
    assert int(act.sum()) > 0
    (life[act] ** 2).sum().backward()
    g = packed.grad
    # dL/dpixel from the rows (byte-equal to the oracle's above): 2*life at death
    # pixels, -2*life at birth pixels, summed in float64
    a_h = act.cpu().numpy()
    life64 = death.detach().double().cpu().numpy() - birth.detach().double().cpu().numpy()
    pix = np.concatenate([dp.cpu().numpy()[a_h], bp.cpu().numpy()[a_h]])
    c = np.concatenate([2 * life64[a_h], -2 * life64[a_h]])
    assert_grad(g.cpu().numpy(), pix, c, int(offs[-1]), "32 volumes")
    # central differences of the GPU forward on voxels of the first volume
    v0 = vols[0]
    x0 = torch.from_numpy(v0).cuda()

    def loss_terms(x):
        """Terms lifetime^2 of the active bars (activity decided in float32 as in
        the loss above; lifetimes as exact float64 differences)."""
        d = cr.persistence(x)
        l = (d.death - d.birth)
        a = (d.dim >= 1) & torch.isfinite(d.death) & (l > 0.1)
        l64 = (d.death[a].double() - d.birth[a].double()).cpu().numpy()
        return [float(t) * float(t) for t in l64]
    g0 = g[offs[0]:offs[1]].cpu().numpy()
    rng = np.random.default_rng(104)
    n0 = int(po[1])
    a0 = act[:n0].cpu().numpy()
    bp0, dp0 = bp[:n0].cpu().numpy(), dp[:n0].cpu().numpy()
    life0 = (death[:n0].double() - birth[:n0].double()).detach().cpu().numpy()
    hi0 = (dim[:n0] >= 1).cpu().numpy() & (dp0 >= 0)
    cand = np.unique(np.concatenate([bp0[a0], dp0[a0]]))
    flat = v0.ravel()
    srt = np.sort(flat)
    checked = 0
    for p in list(rng.choice(cand, 12, replace=False)) + list(rng.integers(0, v0.size, 4)):
        v = np.float32(flat[p])
        h = np.float32(2) * np.spacing(v)
        j = np.searchsorted(srt, v)
        near = srt[max(0, j - 2): j + 3]
        if np.sum(np.abs(near - v) <= 3 * h) > 1:
            continue
        touch = hi0 & ((bp0 == p) | (dp0 == p))
        if np.any(np.abs(life0[touch] - 0.1) <= 3 * h):
            continue
        xp = x0.clone().view(-1)
        xm = x0.clone().view(-1)
        xp[p] = float(v + h)
        xm[p] = float(v - h)
        tp, tm = loss_terms(xp.view(v0.shape)), loss_terms(xm.view(v0.shape))
        fd = math.fsum(tp + [-t for t in tm]) / (float(v + h) - float(v - h))
        contrib = np.sum(np.abs(2 * life0[a0 & ((bp0 == p) | (dp0 == p))]))
        assert abs(g0[p] - fd) <= 1e-6 * max(abs(fd), contrib), (p, g0[p], fd, contrib)
        checked += 1
    assert checked >= 8


def test_masked_volume_256():
    m, dg = _digests()
    vol = m.masked_c3()
    rows = [t.cpu().numpy() for t in cr.persistence(torch.from_numpy(vol).cuda())]
    _invariants(vol, rows)
    check_against_oracle(vol, rows, dg.get("C3_masked"), m, "256^3 blobs, +inf outside the ball")


def test_batch_of_two_256_volumes():
    """Two 256^3 volumes in one batched call (the blobs volume and the same
    volume masked to the ball): each image's rows against the oracle's stored
    digest of that volume."""
    m, dg = _digests()
    vols = [synth.config("C3"), m.masked_c3()]
    packed, shapes, offs = cr.pack([torch.from_numpy(v).cuda() for v in vols])
    d = cr.persistence_batched(packed, shapes, offs)
    assert (d.status.cpu() == 0).all()
    po = d.pair_offsets.cpu().numpy()
    for i, (v, key) in enumerate(zip(vols, ("C3", "C3_masked"))):
        rows = [t[po[i]:po[i + 1]].cpu().numpy() for t in (d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel)]
        rows = local_rows(rows, offs[i])
        _invariants(v, rows)
        check_against_oracle(v, rows, dg.get(key), m, f"batched 256^3 volume {i}")


def test_signal_2_24():
    m, dg = _digests()
    sig = m.walk_2_24()
    rows = [t.cpu().numpy() for t in cr.persistence(torch.from_numpy(sig).cuda())]
    _invariants(sig, rows)
    check_against_oracle(sig, rows, dg.get("walk_2_24"), m, "random walk of 2^24 steps")


def test_lifetime_image_256():
    # the 256^3 diagram is pinned to the oracle above; here the lifetime image
    # must be the per-pixel maximum of death - birth over the rows located there
    vol = synth.config("C3")
    d = cr.persistence(torch.from_numpy(vol).cuda())
    dim, birth, death, bp, dp = [t.cpu().numpy() for t in d]
    life = (death - birth).astype(np.float32)
    for location, pix in (("birth", bp), ("death", dp)):
        got = cr.lifetime_image(d, vol.size, location).cpu().numpy()
        want = np.zeros((3, vol.size), np.float32)
        keep = pix >= 0
        np.maximum.at(want, (dim[keep], pix[keep]), life[keep])
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), location
