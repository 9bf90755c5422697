"""GPU parity of the widened inputs and outputs, through the C ABI, against the
CPU oracle: 1D signals and masked (non-rectangular, +inf outside) domains
(Sec. 2), the pixel locations of the output rows (Sec. 3) and the
lifetime-enhanced image (Sec. 4).  Every comparison is byte-for-byte."""
import numpy as np
import pytest
import torch

import oracle
import paper_2005_12692_amd as cr
import synth
from test_gpu_parity import assert_same, check, oracle_diag

pytestmark = pytest.mark.gpu


def masked(img, mask):
    return np.where(mask, img, np.float32(np.inf)).astype(np.float32)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 1000, 100003])
def test_signals_1d(n):
    rng = np.random.default_rng(n)
    check(rng.random(n, dtype=np.float32), label=f"1D uniform {n}")
    check(rng.integers(0, 5, size=n).astype(np.float32), label=f"1D ties {n}")
    # maxdim above 0 is clamped for a signal
    check(rng.random(n, dtype=np.float32), maxdim=2, label=f"1D maxdim {n}")


def test_signal_worked_and_time_series():
    check(np.array([0, 3, 1, 4, 2], np.float32), label="worked 1D")
    x = np.linspace(0, 4 * np.pi, 100)
    check((np.sin(x) + 0.1 * x).astype(np.float32), label="sin + 0.1 x")


def test_signals_batched():
    rng = np.random.default_rng(3)
    sigs = [rng.random(int(n), dtype=np.float32) for n in rng.integers(1, 3000, size=40)]
    packed, shapes, offs = cr.pack([torch.from_numpy(s).cuda() for s in sigs])
    d = cr.persistence_batched(packed, shapes, offs)
    po = d.pair_offsets.cpu()
    for i, s in enumerate(sigs):
        got = [t.cpu().numpy() for t in d.image(i, po)]
        got[3] = got[3] - offs[i]
        got[4] = np.where(got[4] >= 0, got[4] - offs[i], -1)
        assert_same(got, oracle_diag(s), f"batched signal {i}")


@pytest.mark.parametrize("shape,hole", [((33, 40), 0.0), ((41, 41), 0.45), ((64, 50), 0.3)])
def test_masked_2d(shape, hole):
    m = synth.ball_mask(shape, hole)
    check(masked(synth.uniform2d(shape, shape[0]), m), label=f"masked uniform {shape}")
    check(masked(synth.grf_seeded(shape, 2.0, shape[1]), m), label=f"masked grf {shape}")
    rng = np.random.default_rng(shape[1])
    check(masked(rng.integers(0, 3, size=shape).astype(np.float32), m), label=f"masked ties {shape}")


@pytest.mark.parametrize("shape,hole", [((17, 19, 21), 0.0), ((21, 21, 21), 0.5)])
def test_masked_3d(shape, hole):
    m = synth.ball_mask(shape, hole)
    check(masked(synth.grf_seeded(shape, 1.5, shape[0]), m), label=f"masked volume {shape}")
    rng = np.random.default_rng(shape[2])
    check(masked(rng.random(shape, dtype=np.float32), m), label=f"masked noise {shape}")


def test_masked_batched():
    imgs = []
    for i, shape in enumerate([(30, 31), (45, 28), (12, 60), (50, 50)]):
        imgs.append(masked(synth.uniform2d(shape, i), synth.ball_mask(shape, 0.2 * i)))
    packed, shapes, offs = cr.pack([torch.from_numpy(a).cuda() for a in imgs])
    d = cr.persistence_batched(packed, shapes, offs)
    po = d.pair_offsets.cpu()
    for i, a in enumerate(imgs):
        got = [t.cpu().numpy() for t in d.image(i, po)]
        got[3] = got[3] - offs[i]
        got[4] = np.where(got[4] >= 0, got[4] - offs[i], -1)
        assert_same(got, oracle_diag(a), f"batched masked {i}")


LIFE_CASES = [
    ("signal", lambda: np.random.default_rng(1).random(5000, dtype=np.float32)),
    ("uniform 2D", lambda: synth.uniform2d((70, 90), 5)),
    ("grf 2D", lambda: synth.grf_seeded((256, 256), 3.0, 2)),
    ("masked 2D", lambda: masked(synth.uniform2d((41, 41), 4), synth.ball_mask((41, 41), 0.4))),
    ("grf 3D", lambda: synth.grf_seeded((20, 22, 24), 1.5, 6)),
    ("ties 3D", lambda: np.random.default_rng(2).integers(0, 3, size=(9, 10, 11)).astype(np.float32)),
]


@pytest.mark.parametrize("name,make", LIFE_CASES, ids=[c[0] for c in LIFE_CASES])
@pytest.mark.parametrize("location", ["birth", "death"])
def test_lifetime_image(name, make, location):
    img = make()
    d = cr.persistence(torch.from_numpy(img).cuda())
    got = cr.lifetime_image(d, img.size, location).view((3,) + img.shape).cpu().numpy()
    want = oracle.lifetime_image(oracle.persistence(img), img.shape, location)
    assert got.shape == want.shape
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), f"{name} {location}"


def test_lifetime_image_batched():
    imgs = [synth.uniform2d((20 + 7 * i, 31 + 3 * i), i) for i in range(6)]
    packed, shapes, offs = cr.pack([torch.from_numpy(a).cuda() for a in imgs])
    d = cr.persistence_batched(packed, shapes, offs)
    for location in ("birth", "death"):
        got = cr.lifetime_image(d, offs[-1], location).cpu().numpy()
        for i, a in enumerate(imgs):
            want = oracle.lifetime_image(oracle.persistence(a), a.shape, location).reshape(3, -1)
            assert np.array_equal(got[:, offs[i]:offs[i + 1]].view(np.uint32), want.view(np.uint32)), (i, location)


def test_pixel_coords():
    for img in [synth.uniform2d((23, 37), 1), synth.grf_seeded((9, 11, 13), 1.0, 2),
                np.random.default_rng(0).random(300, dtype=np.float32)]:
        d = cr.persistence(torch.from_numpy(img).cuda())
        for pix in (d.birth_pixel, d.death_pixel):
            got = cr.pixel_coords(pix, img.shape).cpu().numpy()
            assert np.array_equal(got, oracle.pixel_coords(pix.cpu().numpy(), img.shape).astype(np.int32))
    # a batched image: indices relative to its offset
    imgs = [synth.uniform2d((10, 12), 0), synth.uniform2d((7, 30), 1)]
    packed, shapes, offs = cr.pack([torch.from_numpy(a).cuda() for a in imgs])
    d = cr.persistence_batched(packed, shapes, offs)
    di = d.image(1)
    got = cr.pixel_coords(di.birth_pixel, shapes[1], base=offs[1]).cpu().numpy()
    assert np.array_equal(got, oracle.pixel_coords(di.birth_pixel.cpu().numpy() - offs[1], shapes[1]).astype(np.int32))


def test_bad_rows_are_errors():
    img = synth.uniform2d((8, 8), 0)
    d = cr.persistence(torch.from_numpy(img).cuda())
    with pytest.raises(cr.CRError):
        cr.lifetime_image(d, 10)  # n_pixels smaller than the image
    with pytest.raises(ValueError):
        cr.lifetime_image(d, 64, "middle")
    with pytest.raises(cr.CRError):
        cr.pixel_coords(d.birth_pixel, (4, 4))
    # the context still works afterwards
    check(img, label="after errors")


def test_signals_graph_and_autotune():
    # the graph and autotuner entry points take ndim 1 too (the 2D setting)
    rng = np.random.default_rng(9)
    sigs = [synth.random_walk(int(n), int(n)) for n in rng.integers(2, 20000, size=24)]
    packed, shapes, offs = cr.pack([torch.from_numpy(s).cuda() for s in sigs])
    eager = cr.persistence_batched(packed, shapes, offs)
    cap = int(eager.pair_offsets[-1].item())
    before = cr.get_tuning(2)
    try:
        tuned = cr.autotune(packed, shapes, offs, capacity=cap, repeats=1)
        assert cr.get_tuning(1) == cr.get_tuning(2) == tuned
        g = cr.BatchedGraph(packed, shapes, offs, capacity=cap)
        try:
            for _ in range(2):
                g.launch()
                got = g.result()
                po = got.pair_offsets.cpu()
                for i in (0, 7, 23):
                    rows = [t.cpu().numpy() for t in got.image(i, po)]
                    rows[3] = rows[3] - offs[i]
                    rows[4] = np.where(rows[4] >= 0, rows[4] - offs[i], -1)
                    assert_same(rows, oracle_diag(sigs[i]), f"graph signal {i}")
        finally:
            g.close()
    finally:
        cr.set_tuning(2, **before)
