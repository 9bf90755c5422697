"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Every comparison is byte-for-byte on the five output arrays (dim, birth, death,
birth_pixel, death_pixel) in canonical order: the bar end points are copies of
input values and the pixel map is fixed by the written convention, so exact
equality is the bar.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2005_12692_amd as cr
import synth

pytestmark = pytest.mark.gpu
FIELDS = ("dim", "birth", "death", "birth_pixel", "death_pixel")


def gpu_diag(img, maxdim=None):
    d = cr.persistence(torch.from_numpy(np.ascontiguousarray(img)).cuda(), maxdim)
    return [t.cpu().numpy() for t in d]


def oracle_diag(img, maxdim=None):
    o = oracle.persistence(img, maxdim)
    return [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel]


def assert_same(got, want, label=""):
    for name, g, w in zip(FIELDS, got, want):
        if g.shape != w.shape or not np.array_equal(g.view(np.uint8), w.view(np.uint8)):
            msg = [f"{label}: field {name} differs: gpu {g.shape} oracle {w.shape}",
                   f"rows per dim gpu {np.bincount(got[0], minlength=3)} oracle {np.bincount(want[0], minlength=3)}"]
            n = min(len(g), len(w))
            bad = np.flatnonzero(g[:n].view(np.uint8).reshape(n, -1).any(1) !=
                                 w[:n].view(np.uint8).reshape(n, -1).any(1)) if n else []
            first = next((i for i in range(n) if g[i].tobytes() != w[i].tobytes()), None)
            if first is not None:
                msg.append(f"first differing row {first}: gpu {[x[first] for x in got]} "
                           f"oracle {[x[first] for x in want]}")
            raise AssertionError("\n".join(msg))


def check(img, maxdim=None, label=""):
    assert_same(gpu_diag(img, maxdim), oracle_diag(img, maxdim), label or str(img.shape))


TINY_2D = [(1, 1), (1, 2), (2, 1), (2, 2), (1, 9), (9, 1), (3, 3), (2, 5), (4, 5), (7, 3)]


@pytest.mark.parametrize("shape", TINY_2D)
def test_tiny_2d(shape):
    rng = np.random.default_rng(sum(shape))
    for levels in (2, 3, 1000):
        for _ in range(4):
            img = rng.integers(0, levels, size=shape).astype(np.float32)
            check(img, label=f"{shape} levels={levels}")


@pytest.mark.parametrize("name", ["ttk", "fig2", "void"])
def test_worked_examples(name):
    if name == "ttk":
        img = np.array([[0, 0, 0], [0, 9, 0], [0, 0, 0]], np.float32)
    elif name == "fig2":
        img = np.array([[-1, 1, -2], [3, 3, 2], [3, 3, -1]], np.float32)
    else:
        img = np.zeros((3, 3, 3), np.float32)
        img[1, 1, 1] = 9
    check(img, label=name)


def test_uniform_64x64_seeds():
    """64x64 i.i.d. uniform images, seeds 0..199."""
    for seed in range(200):
        check(synth.uniform2d((64, 64), seed), label=f"seed {seed}")


@pytest.mark.parametrize("shape", [(33, 17), (100, 37), (5, 200), (257, 129), (31, 1000)])
def test_ragged_2d(shape):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    check(synth.uniform2d(shape, shape[0]), label=f"uniform {shape}")
    check(synth.grf_seeded(shape, 2.0, shape[1]), label=f"grf {shape}")
    check(rng.integers(0, 4, size=shape).astype(np.float32), label=f"ties {shape}")


def test_special_values_2d():
    check(np.full((17, 23), 1.5, np.float32), label="constant")
    check((np.indices((20, 21)).sum(0) % 2).astype(np.float32), label="checkerboard")
    img = synth.uniform2d((40, 40), 3)
    img[10:20, 5:30] = np.inf
    img[0, :] = -np.inf
    check(img, label="infinities")
    img = np.zeros((12, 12), np.float32)
    img[::3, ::2] = -0.0
    img[5, 5] = 1.0
    check(img, label="negative zero")


def test_grf_1024():
    """The 2D workload: 1024x1024 Gaussian random field, sigma 4."""
    check(synth.config("C2"), label="C2")


TINY_3D = [(2, 2, 2), (1, 4, 5), (3, 1, 4), (2, 3, 1), (3, 4, 5), (5, 3, 2)]


@pytest.mark.parametrize("shape", TINY_3D)
def test_tiny_3d(shape):
    rng = np.random.default_rng(sum(shape) + 100)
    for levels in (2, 3, 1000):
        for _ in range(4):
            img = rng.integers(0, levels, size=shape).astype(np.float32)
            check(img, label=f"{shape} levels={levels}")


@pytest.mark.parametrize("shape", [(9, 8, 10), (17, 16, 15), (6, 33, 5), (20, 20, 20)])
def test_ragged_3d(shape):
    rng = np.random.default_rng(sum(shape))
    check(synth.grf_seeded(shape, 1.5, 1), label=f"grf {shape}")
    check(rng.random(shape, dtype=np.float32), label=f"uniform {shape}")
    check(rng.integers(0, 3, size=shape).astype(np.float32), label=f"ties {shape}")


@pytest.mark.parametrize("n", [24, 48, 64])
def test_blobs_3d(n):
    """The 3D workload's recipe at sizes the oracle finishes in seconds."""
    check(synth.blobs3d(n, 2), label=f"blobs {n}")


def test_maxdim():
    vol = synth.grf_seeded((14, 13, 12), 1.5, 5)
    for md in (0, 1, 2, 7):
        check(vol, maxdim=md, label=f"maxdim {md}")
    img = synth.uniform2d((30, 30), 4)
    for md in (0, 1, 3):
        check(img, maxdim=md, label=f"2d maxdim {md}")


def test_nan_and_bad_arguments():
    img = synth.uniform2d((16, 16), 1)
    img[3, 4] = np.nan
    with pytest.raises(cr.CRError) as e:
        cr.persistence(torch.from_numpy(img).cuda())
    assert e.value.code == cr.CR_ERR_NAN_INPUT
    with pytest.raises(cr.CRError) as e:
        cr.persistence(torch.rand(8, 8, device="cuda"), maxdim=-1)
    assert e.value.code == cr.CR_ERR_INVALID_ARGUMENT
    with pytest.raises((TypeError, ValueError)):
        cr.persistence(torch.rand(2, 3, 4, 5, device="cuda"))  # four axes (1D signals are valid)
    # the context is still usable after errors
    check(synth.uniform2d((16, 16), 2), label="after errors")


def test_deterministic_repeat():
    vol = synth.blobs3d(40, 7)
    x = torch.from_numpy(vol).cuda()
    a = [t.cpu().numpy() for t in cr.persistence(x)]
    for _ in range(5):
        b = [t.cpu().numpy() for t in cr.persistence(x)]
        assert_same(b, a, "repeat")


WAVE_ENV = ("CR_LONG_LEN", "CR_YIELD_ITERS", "CR_WAVE_SHORT", "CR_FRONT_CAP", "CR_MID_CAP", "CR_NARROW_MIN",
            "CR_NARROW_CAP", "CR_GROUP_MAX", "CR_GROUP_CAP", "CR_WAVE_YIELD", "CR_ASYNC_MAX")


@pytest.mark.parametrize("setting", [
    # every column to wave mode after two additions; narrow configuration with a
    # tiny front list; wave columns stored and resumed every 3 additions
    ("0", "2", "0", "4032", "8192", "0", "128", "0", "4096", "3", "0"),
    ("8", "8", "0", "4032", "8192", "1000000000", "256", "0", "4096", "0", "0"),  # wide configuration only
    # whole rounds in wave mode, tiny front and middle lists
    ("0", "1", "1000000", "128", "300", "1000000000", "320", "0", "4096", "1", "0"),
    ("0", "1", "1000000", "128", "300", "0", "320", "0", "4096", "5", "0"),
    # the middle list folded into the tail at every push; all three configurations
    ("4", "4", "64", "200", "0", "64", "200", "16", "128", "2", "0"),
    # a workgroup per column in every wave-mode round: small lists, then the defaults
    ("0", "1", "1000000", "128", "300", "1000000000", "256", "1000000000", "128", "1", "0"),
    ("0", "2", "0", "1024", "0", "1000000000", "256", "1000000000", "200", "0", "0"),
    ("16", "1024", "4096", "1024", "8192", "8192", "256", "1000000000", "4096", "16", "0"),
    # the asynchronous tail: after the first round (small lists, so that every
    # merge runs in it), and after rounds of wave mode once at most 8 or 64
    # columns are left
    ("0", "1", "1000000", "128", "300", "1000000000", "256", "1000000000", "128", "1", "1000000000"),
    ("0", "2", "0", "4032", "8192", "0", "128", "0", "4096", "3", "64"),
    ("4", "4", "64", "200", "0", "64", "200", "16", "128", "2", "8"),
])
def test_wave_mode_forced(setting):
    """Volumes whose columns are handed to the wavefront-per-column mode after a
    few additions, with small front and middle lists so that the merges into the
    arena lists run (the thresholds are lowered through the environment, which
    the library reads at every call)."""
    import os
    rng = np.random.default_rng(5)
    cases = [(synth.blobs3d(16, 1), "blobs 16"), (synth.blobs3d(24, 2), "blobs 24"),
             (synth.blobs3d(40, 3), "blobs 40"),
             (rng.integers(0, 3, size=(9, 10, 11)).astype(np.float32), "ties"),
             (synth.grf_seeded((20, 18, 22), 1.5, 4), "grf")]
    try:
        for k, v in zip(WAVE_ENV, setting):
            os.environ[k] = v
        for img, label in cases:
            check(img, label=f"{label} {setting}")
    finally:
        for k in WAVE_ENV:
            os.environ.pop(k, None)


def test_against_cohomology_oracle():
    """The GPU reduces boundary columns (homology); the oracle's cohomology mode
    reduces the coboundary matrix as the paper does (Sec. 2).  Different
    algorithms, the same diagram: volumes, a 2D image and a 1D signal."""
    rng = np.random.default_rng(31)
    cases = [(synth.blobs3d(20, 5), "blobs 20"), (synth.grf_seeded((14, 13, 12), 1.5, 2), "grf"),
             (rng.integers(0, 3, size=(9, 8, 10)).astype(np.float32), "ties 3D"),
             (synth.uniform2d((40, 37), 6), "uniform 2D"), (synth.random_walk(300, 3), "signal")]
    for img, label in cases:
        o = oracle.persistence(img, mode="cohomology")
        assert_same(gpu_diag(img), [o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel], f"{label} (cohomology)")


def test_first_round_in_rank_order(monkeypatch):
    """The first round of the degree-1 reduction takes its columns in spatial
    order by default; with CR_SPATIAL=0 it takes them in rank order (the
    commit of the first round too): both give the oracle's diagram, with the
    asynchronous tail off and on."""
    cases = [(synth.blobs3d(40, 3), "blobs 40"), (synth.grf_seeded((30, 26, 34), 1.5, 6), "grf"),
             (np.random.default_rng(9).integers(0, 4, size=(12, 13, 11)).astype(np.float32), "ties")]
    for spatial in ("0", "1"):
        for tail in ("0", "4096"):
            monkeypatch.setenv("CR_SPATIAL", spatial)
            monkeypatch.setenv("CR_ASYNC_MAX", tail)
            for img, label in cases:
                check(img, label=f"{label} spatial {spatial} tail {tail}")


_MODE_VOLUMES = {}


def _mode_volumes():
    """Larger volumes for the reduction modes, with their oracle diagrams
    (computed once): smooth blobs, a rough field and i.i.d. noise."""
    if not _MODE_VOLUMES:
        rng = np.random.default_rng(11)
        vols = [(synth.blobs3d(96, 7, n_blobs=80), "blobs 96"),
                (synth.grf_seeded((64, 56, 60), 2.0, 8), "grf 64x56x60"),
                (rng.random((44, 40, 48), dtype=np.float32), "uniform 44x40x48")]
        for img, label in vols:
            _MODE_VOLUMES[label] = (img, oracle_diag(img))
    return _MODE_VOLUMES


@pytest.mark.parametrize("setting", [
    # (long_len, yield_iters, wave_short, front_cap, mid_cap, narrow_min, narrow_cap, group_max, group_cap,
    #  wave_yield, async_max)
    None,                                                                                      # the defaults
    ("0", "4", "1000000", "128", "256", "1000000000", "256", "1000000000", "128", "1", "0"),   # group mode, small lists
    ("0", "4", "1000000", "128", "0", "0", "128", "0", "4096", "7", "0"),                      # narrow mode, small lists
    ("8", "64", "1000000", "128", "512", "1000000000", "256", "0", "4096", "3", "0"),          # wide mode, small lists
    ("32", "16", "0", "4032", "100000", "1000000000", "256", "1000000000", "4096", "0", "0"),  # large lists, group mode
    # the asynchronous tail after the first round, small lists; after wide-mode
    # rounds with at most 32 columns left
    ("0", "4", "1000000", "128", "256", "1000000000", "256", "1000000000", "128", "1", "1000000000"),
    ("8", "64", "1000000", "128", "512", "1000000000", "256", "0", "4096", "3", "32"),
])
def test_reduction_modes_larger(setting):
    """Volumes of 10^5 to 10^6 pixels with many long columns, each reduction mode forced
    with lists small enough that owner columns go to every level (P, F, the
    middle list directly, the middle list by merge) and the lists fold often."""
    import os
    try:
        if setting is not None:
            for k, v in zip(WAVE_ENV, setting):
                os.environ[k] = v
        for label, (img, want) in _mode_volumes().items():
            assert_same(gpu_diag(img), want, f"{label} {setting}")
    finally:
        for k in WAVE_ENV:
            os.environ.pop(k, None)
