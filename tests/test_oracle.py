"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

The oracle (``oracle/cr_oracle.c``) is checked against:
* the paper's worked examples (golden fixtures, each citing its source);
* brute force on tiny grids: per-threshold Betti numbers by flood fill and the
  Euler characteristic, and the exact diagram recovered from persistent Betti
  numbers (GF(2) ranks) -- exhaustively on all 3x3 images and 2x2x2 volumes with
  values in {0,1,2};
* closed forms (constant, binary and checkerboard images, a hollow shell);
* invariants (one essential bar at the global minimum, pixel map, cell count,
  Euler characteristic at every threshold);
* metamorphic relations (flips, transposes, monotone maps of the values);
* its two reduction modes against each other and against a textbook Kruskal.
"""
import itertools
import os

import numpy as np
import pytest

import brute
import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLDEN, name))]
    lines = [l for l in lines if l]
    shape = tuple(int(x) for x in lines[1].split()[1:])
    i = lines.index("image") + 1
    j = lines.index("bars")
    vals = [float(x) for l in lines[i:j] for x in l.split()]
    img = np.array(vals, np.float32).reshape(shape)
    bars = brute.Counter()
    rows = []
    for l in lines[j + 1:]:
        f = l.split()
        bars[(int(f[0]), float(f[1]), float(f[2]))] += 1
        if len(f) == 5:
            rows.append((int(f[0]), float(f[1]), float(f[2]), int(f[3]), int(f[4])))
    return img, bars, rows


def diag_counter(d):
    return brute.diagram_counter(d.dim, d.birth, d.death)


@pytest.mark.parametrize("name", sorted(os.listdir(GOLDEN)))
def test_golden(name):
    if not name.endswith(".txt"):
        pytest.skip("not a fixture")
    img, bars, rows = load_golden(name)
    for mode in ("twist", "plain"):
        d = oracle.persistence(img, mode=mode)
        assert diag_counter(d) == bars
        if rows:  # hand-derived pixel map, in canonical row order
            got = list(zip(d.dim.tolist(), d.birth.tolist(), d.death.tolist(),
                           d.birth_pixel.tolist(), d.death_pixel.tolist()))
            assert got == rows
    assert brute.diagram_from_ranks(img) == bars


def _betti_check(img, d, thresholds=None):
    vals = np.unique(img) if thresholds is None else thresholds
    for t in vals:
        b = brute.betti(img, t)
        for k in range(3):
            assert brute.bars_alive(d.dim, d.birth, d.death, k, t) == b[k], (k, t)


def test_exhaustive_3x3_betti():
    """All 3^9 images with values in {0,1,2}: bars alive at each threshold equal
    the Betti numbers of the sublevel set."""
    vals = np.array([0, 1, 2], np.float32)
    rng = np.random.default_rng(0)
    sample = set(rng.choice(3 ** 9, 400, replace=False).tolist())
    for n, combo in enumerate(itertools.product(range(3), repeat=9)):
        img = vals[list(combo)].reshape(3, 3)
        d = oracle.persistence(img)
        # per-threshold Betti numbers (fast: b0 by counting, chi by counting)
        for t in (0.0, 1.0, 2.0):
            b = brute.betti(img, t)
            for k in range(2):
                assert brute.bars_alive(d.dim, d.birth, d.death, k, t) == b[k], (combo, k, t)
        if n in sample:
            assert diag_counter(d) == brute.diagram_from_ranks(img), combo
            assert diag_counter(oracle.persistence(img, mode="plain")) == diag_counter(d)


def test_exhaustive_2x2x2():
    vals = np.array([0, 1, 2], np.float32)
    rng = np.random.default_rng(1)
    sample = set(rng.choice(3 ** 8, 300, replace=False).tolist())
    for n, combo in enumerate(itertools.product(range(3), repeat=8)):
        img = vals[list(combo)].reshape(2, 2, 2)
        d = oracle.persistence(img)
        for t in (0.0, 1.0, 2.0):
            b = brute.betti(img, t)
            for k in range(3):
                assert brute.bars_alive(d.dim, d.birth, d.death, k, t) == b[k], (combo, k, t)
        if n in sample:
            assert diag_counter(d) == brute.diagram_from_ranks(img), combo


@pytest.mark.parametrize("shape,levels,count", [
    ((4, 4), 3, 60), ((5, 5), 4, 40), ((6, 6), 5, 15), ((4, 7), 3, 20),
    ((3, 3, 3), 3, 25), ((2, 3, 4), 4, 25), ((4, 4, 3), 3, 6)])
def test_random_ties_persistent_betti(shape, levels, count):
    """Tie-heavy random grids: the exact diagram from GF(2) ranks."""
    rng = np.random.default_rng(hash(shape) % 2 ** 32)
    for _ in range(count):
        img = rng.integers(0, levels, size=shape).astype(np.float32) - 1.0
        d = oracle.persistence(img)
        assert diag_counter(d) == brute.diagram_from_ranks(img), img.tolist()


@pytest.mark.parametrize("seed", range(6))
def test_uniform_invariants(seed):
    img = synth.uniform2d((24, 31), seed)
    d = oracle.persistence(img, cell_pairs=True)
    _invariants(img, d)
    _betti_check(img, d)
    assert diag_counter(d) == diag_counter(oracle.persistence(img, mode="plain"))
    h0 = d.dim == 0
    k = oracle.persistence_h0(img)
    for f in ("dim", "birth", "death", "birth_pixel", "death_pixel"):
        assert np.array_equal(getattr(k, f), getattr(d, f)[h0])
    assert brute.h0_kruskal(img) == brute.diagram_counter(d.dim[h0], d.birth[h0], d.death[h0])


def _invariants(img, d):
    flat = img.ravel()
    ess = d.death_pixel < 0
    # exactly one essential bar, in degree 0, born at the global minimum
    assert ess.sum() == 1 and d.dim[ess][0] == 0 and d.birth[ess][0] == flat.min()
    assert np.all(np.isinf(d.death[ess]))
    fin = ~ess
    assert np.all(d.birth[fin] < d.death[fin])
    # pixel map: birth == image[birth_pixel], death == image[death_pixel], bit for bit
    assert np.array_equal(d.birth.view(np.uint32), flat[d.birth_pixel].view(np.uint32))
    assert np.array_equal(d.death[fin].view(np.uint32), flat[d.death_pixel[fin]].view(np.uint32))
    # canonical order: (dim, birth_pixel, death_pixel as unsigned)
    key = list(zip(d.dim.tolist(), d.birth_pixel.tolist(),
                   (d.death_pixel.astype(np.uint64)).tolist()))
    assert key == sorted(key)
    if d.cell_birth is not None:
        n_cells = int(np.prod([2 * s - 1 for s in img.shape]))
        n_ess = int((d.cell_death < 0).sum())
        assert 2 * (len(d.cell_birth) - n_ess) + n_ess == n_cells
        assert len(np.unique(np.concatenate([d.cell_birth, d.cell_death[d.cell_death >= 0]]))) \
            == n_cells


@pytest.mark.parametrize("shape,seed", [((9, 8, 10), 0), ((12, 12, 12), 1), ((5, 16, 7), 2)])
def test_3d_invariants(shape, seed):
    img = synth.grf_seeded(shape, 1.5, seed)
    d = oracle.persistence(img, cell_pairs=True)
    _invariants(img, d)
    _betti_check(img, d)
    assert diag_counter(d) == diag_counter(oracle.persistence(img, mode="plain"))


def test_blob_volume_betti_sampled():
    img = synth.blobs3d(32, 5)
    d = oracle.persistence(img)
    _invariants(img, d)
    ts = np.quantile(img, np.linspace(0.02, 0.98, 9)).astype(np.float32)
    _betti_check(img, d, ts)
    h0 = d.dim == 0
    assert diag_counter(oracle.persistence_h0(img)) == brute.diagram_counter(
        d.dim[h0], d.birth[h0], d.death[h0])


def test_tie_free_pixel_map():
    """Without ties the birth pixel is the unique pixel holding the birth value."""
    rng = np.random.default_rng(7)
    img = rng.permutation(20 * 17).astype(np.float32).reshape(20, 17)
    d = oracle.persistence(img)
    flat = img.ravel()
    for b, p in zip(d.birth, d.birth_pixel):
        assert np.flatnonzero(flat == b).tolist() == [p]
    # and the number of degree-0 bars equals the number of strict local minima
    pad = np.pad(img, 1, constant_values=np.inf)
    c = pad[1:-1, 1:-1]
    minima = (c < pad[:-2, 1:-1]) & (c < pad[2:, 1:-1]) & (c < pad[1:-1, :-2]) & (c < pad[1:-1, 2:])
    assert int((d.dim == 0).sum()) == int(minima.sum())


def test_closed_forms():
    # constant image: only [c, inf)
    for shape in [(5, 7), (3, 4, 5)]:
        d = oracle.persistence(np.full(shape, 2.5, np.float32))
        assert diag_counter(d) == {(0, 2.5, float("inf")): 1}
    # binary image: (k0 - 1) x [0,1) in degree 0, b1(0-set) x [0,1) in degree 1
    rng = np.random.default_rng(3)
    for _ in range(20):
        img = (rng.random((9, 11)) < 0.5).astype(np.float32)
        if img.min() > 0:
            continue
        d = oracle.persistence(img)
        k0 = brute.betti(img, 0.0)[0]
        b1 = brute.betti(img, 0.0)[1]
        want = brute.Counter({(0, 0.0, float("inf")): 1})
        if k0 > 1:
            want[(0, 0.0, 1.0)] = k0 - 1
        if b1:
            want[(1, 0.0, 1.0)] = b1
        assert diag_counter(d) == want
    # checkerboard: every 0 pixel is its own component (diagonals do not connect)
    cb = (np.indices((6, 7)).sum(0) % 2).astype(np.float32)
    d = oracle.persistence(cb)
    assert diag_counter(d) == {(0, 0.0, float("inf")): 1, (0, 0.0, 1.0): int((cb == 0).sum()) - 1}
    # hollow shell of 0s inside 1s: one void [0,1)
    v = np.ones((7, 7, 7), np.float32)
    v[1:6, 1:6, 1:6] = 0
    v[2:5, 2:5, 2:5] = 1
    d = oracle.persistence(v)
    assert diag_counter(d) == {(0, 0.0, float("inf")): 1, (2, 0.0, 1.0): 1}


def test_metamorphic():
    img = synth.uniform2d((13, 13), 11)
    base = diag_counter(oracle.persistence(img))
    for t in [img[::-1], img[:, ::-1], img.T, img[::-1, ::-1].T]:
        assert diag_counter(oracle.persistence(np.ascontiguousarray(t))) == base
    # phi -> 2 phi (exact in float32) doubles every value
    d2 = diag_counter(oracle.persistence(img * np.float32(2)))
    assert d2 == brute.Counter({(k, 2 * b, 2 * e): n for (k, b, e), n in base.items()})
    # an order isomorphism (dense rank) maps the diagram through the same map
    u, inv = np.unique(img, return_inverse=True)
    r = inv.reshape(img.shape).astype(np.float32)
    m = {float(x): float(i) for i, x in enumerate(u)}
    m[float("inf")] = float("inf")
    dr = diag_counter(oracle.persistence(r))
    assert dr == brute.Counter({(k, m[b], m[e]): n for (k, b, e), n in base.items()})
    vol = synth.grf_seeded((6, 7, 8), 1.0, 3)
    vb = diag_counter(oracle.persistence(vol))
    for t in [vol[::-1], vol[:, :, ::-1], np.transpose(vol, (2, 1, 0))]:
        assert diag_counter(oracle.persistence(np.ascontiguousarray(t))) == vb


def test_negative_zero_and_errors():
    img = np.zeros((4, 4), np.float32)
    img[1, 2] = -0.0
    img[3, 1] = -0.0
    img[2, 2] = 1.0
    a = oracle.persistence(img)
    b = oracle.persistence(np.abs(img))
    for f in ("dim", "birth", "death", "birth_pixel", "death_pixel"):
        assert np.array_equal(getattr(a, f).view(np.uint8), getattr(b, f).view(np.uint8))
    bad = img.copy()
    bad[0, 0] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.persistence(bad)
    assert e.value.code == oracle.ERR_NAN
    with pytest.raises(oracle.OracleError):
        oracle.persistence(img, maxdim=-1)
    # +inf is an ordinary value (pixels outside a domain, Sec. 2)
    inf_img = synth.uniform2d((6, 6), 2)
    inf_img[2:4, 2:4] = np.inf
    d = oracle.persistence(inf_img)
    assert np.isinf(d.birth).sum() == 0
    assert diag_counter(d) == brute.diagram_from_ranks(inf_img)


def test_maxdim_filter():
    vol = synth.grf_seeded((7, 6, 5), 1.0, 9)
    full = oracle.persistence(vol)
    for md in (0, 1):
        part = oracle.persistence(vol, maxdim=md)
        keep = full.dim <= md
        for f in ("dim", "birth", "death", "birth_pixel", "death_pixel"):
            assert np.array_equal(getattr(part, f), getattr(full, f)[keep])
    # maxdim above the data is clamped
    assert len(oracle.persistence(vol, maxdim=5)) == len(full)


def test_one_dimensional():
    # a 1D image is a 2D image on one line (Sec. 2).  Worked by hand: minima 0,
    # 1, 2 at pixels 0, 2, 4; the edges (0,1), (1,2) enter at 3 and (2,3),
    # (3,4) at 4; the edge at 3 joining {0,1} to {2} kills the younger
    # component (born 1) at the edge's larger vertex, pixel 1, and the edge at
    # 4 joining pixel 4 kills it at pixel 3.
    d = oracle.persistence(np.array([0, 3, 1, 4, 2], np.float32))
    rows = list(zip(d.dim.tolist(), d.birth.tolist(), d.death.tolist(), d.birth_pixel.tolist(),
                    d.death_pixel.tolist()))
    assert rows == [(0, 0.0, float("inf"), 0, -1), (0, 1.0, 3.0, 2, 1), (0, 2.0, 4.0, 4, 3)]
    rng = np.random.default_rng(5)
    for n in [1, 2, 3, 7, 16, 40]:
        for levels in [3, 1000]:
            s = rng.integers(0, levels, size=n).astype(np.float32)
            d = oracle.persistence(s)
            assert diag_counter(d) == brute.diagram_from_ranks(s)
            # the same signal as a 1 x n and an n x 1 image: same diagram, same pixels
            for t in (s[None, :], s[:, None]):
                e = oracle.persistence(np.ascontiguousarray(t))
                for f in ("dim", "birth", "death", "birth_pixel", "death_pixel"):
                    assert np.array_equal(getattr(d, f), getattr(e, f))
    # the paper's time-series example: sin(x) + 0.1 x on 100 samples of [0, 4 pi]
    x = np.linspace(0, 4 * np.pi, 100)
    s = (np.sin(x) + 0.1 * x).astype(np.float32)
    d = oracle.persistence(s)
    assert diag_counter(d) == brute.diagram_from_ranks(s)
    assert len(d) == 3 and int((d.death_pixel < 0).sum()) == 1  # three valleys, one essential


def test_masked_domains():
    # pixels outside a non-rectangular domain take +inf (Sec. 2).  An annulus of
    # constant value c: one component [c, inf) and one loop born at c that dies
    # only when the +inf hole enters -- a finite pair whose death is +inf, told
    # apart from an essential bar by its death pixel.
    yy, xx = np.mgrid[:13, :13]
    r2 = (yy - 6) ** 2 + (xx - 6) ** 2
    ring = (r2 >= 4) & (r2 <= 25)
    img = np.where(ring, np.float32(1.5), np.float32(np.inf)).astype(np.float32)
    d = oracle.persistence(img)
    rows = sorted(zip(d.dim.tolist(), d.birth.tolist(), d.death.tolist(), (d.death_pixel >= 0).tolist()))
    assert rows == [(0, 1.5, float("inf"), False), (1, 1.5, float("inf"), True)]
    assert np.isinf(img.reshape(-1)[d.death_pixel[d.dim == 1][0]])
    # varying values on the annulus: the exact diagram from persistent Betti numbers
    rng = np.random.default_rng(8)
    small = ((yy[:9, :9] - 4) ** 2 + (xx[:9, :9] - 4) ** 2)
    mask = (small >= 2) & (small <= 12)
    for _ in range(3):
        v = np.where(mask, rng.integers(0, 4, size=mask.shape).astype(np.float32), np.float32(np.inf))
        d = oracle.persistence(v.astype(np.float32))
        assert diag_counter(d) == brute.diagram_from_ranks(v)
        assert int((d.death_pixel < 0).sum()) == 1  # one essential bar: the full grid is contractible
    # a spherical shell of value 0 in a +inf volume: one void [0, inf), finite
    z, y, x = np.mgrid[:9, :9, :9]
    r = (z - 4) ** 2 + (y - 4) ** 2 + (x - 4) ** 2
    vol = np.where((r >= 4) & (r <= 12), np.float32(0), np.float32(np.inf)).astype(np.float32)
    d = oracle.persistence(vol)
    rows = sorted(zip(d.dim.tolist(), d.birth.tolist(), d.death.tolist(), (d.death_pixel >= 0).tolist()))
    assert rows == [(0, 0.0, float("inf"), False), (2, 0.0, float("inf"), True)]


def test_lifetime_image_and_locations():
    # the worked 1D example above: bars (0,[0,inf)) at pixel 0, (0,[1,3)) born at
    # pixel 2 killed at pixel 1, (0,[2,4)) born at 4 killed at 3 (Sec. 4: each
    # pixel holds the largest lifetime of the bars located there)
    d = oracle.persistence(np.array([0, 3, 1, 4, 2], np.float32))
    lb = oracle.lifetime_image(d, (5,))
    assert lb.shape == (3, 5)
    assert lb[0].tolist() == [float("inf"), 0.0, 2.0, 0.0, 2.0] and not lb[1:].any()
    ld = oracle.lifetime_image(d, (5,), "death")
    assert ld[0].tolist() == [0.0, 2.0, 0.0, 2.0, 0.0] and not ld[1:].any()
    # two bars at one pixel keep the larger lifetime
    two = oracle.Diagram(np.array([1, 1], np.int32), np.array([0, 1], np.float32),
                         np.array([5, 2], np.float32), np.array([3, 3]), np.array([0, 1]))
    assert oracle.lifetime_image(two, (2, 2))[1].tolist() == [[0, 0], [0, 5]]
    # a binary image: every component is born at its own pixel, lifetime 1
    # (or inf for the one essential bar)
    rng = np.random.default_rng(4)
    img = (rng.random((10, 12)) < 0.5).astype(np.float32)
    d = oracle.persistence(img)
    c0 = oracle.lifetime_image(d, img.shape)[0]
    k0 = brute.betti(img, 0.0)[0]
    assert int((c0 == 1).sum()) == k0 - 1 and int(np.isinf(c0).sum()) == 1 and int((c0 != 0).sum()) == k0
    # locations: (x, y, z) with x the last axis
    assert oracle.pixel_coords(np.array([0, 7, 11, -1]), (3, 4)).tolist() == [
        [0, 0, 0], [3, 1, 0], [3, 2, 0], [-1, -1, -1]]
    assert oracle.pixel_coords(np.array([1 * 20 + 2 * 5 + 3]), (2, 4, 5)).tolist() == [[3, 2, 1]]


def _cell_pair_set(d):
    return sorted(zip(d.cell_birth.tolist(), d.cell_death.tolist()))


@pytest.mark.parametrize("shape,levels,count", [
    ((5, 5), 3, 40), ((7, 6), 1000, 20), ((1, 9), 3, 20), ((9,), 4, 20),
    ((3, 3, 3), 3, 25), ((4, 3, 5), 1000, 15), ((2, 5, 4), 2, 20), ((5, 5, 5), 4, 6)])
def test_cohomology_mode_same_pairs(shape, levels, count):
    """The coboundary reduction (the paper's formulation, Sec. 2) and the
    boundary reductions are different algorithms over the same total order of
    cells; by the duality of persistent homology and cohomology they pair the
    same cells, zero-length pairs and essential cells included, so the
    diagrams are identical byte for byte.  On the smaller grids the cohomology
    diagram is also the exact one from GF(2) ranks."""
    rng = np.random.default_rng(7 * len(shape) + levels)
    for _ in range(count):
        img = rng.integers(0, levels, size=shape).astype(np.float32) - 1.0
        if levels > 100:
            img = rng.random(shape, dtype=np.float32)
        for maxdim in sorted({0, len(shape) - 1}):
            co = oracle.persistence(img, maxdim=maxdim, mode="cohomology", cell_pairs=True)
            for mode in ("plain", "twist"):
                ho = oracle.persistence(img, maxdim=maxdim, mode=mode, cell_pairs=True)
                assert _cell_pair_set(co) == _cell_pair_set(ho), (mode, maxdim, img.tolist())
                for f in ("dim", "birth", "death", "birth_pixel", "death_pixel"):
                    a, b = getattr(co, f), getattr(ho, f)
                    assert a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8)), (f, mode)
        if img.size <= 36:
            assert diag_counter(oracle.persistence(img, mode="cohomology")) == brute.diagram_from_ranks(img)


def test_cohomology_mode_volumes_and_masks():
    """Larger cases of the same identity: a smooth volume, a tie-heavy one and
    a volume with +inf outside a ball (the masked domains)."""
    rng = np.random.default_rng(21)
    ball = synth.ball_mask((9, 10, 11))
    cases = [synth.grf_seeded((10, 9, 12), 1.5, 3), rng.integers(0, 3, size=(8, 9, 7)).astype(np.float32),
             np.where(ball, synth.grf_seeded((9, 10, 11), 1.0, 4), np.float32(np.inf)).astype(np.float32)]
    for img in cases:
        co = oracle.persistence(img, mode="cohomology", cell_pairs=True)
        ho = oracle.persistence(img, mode="twist", cell_pairs=True)
        assert _cell_pair_set(co) == _cell_pair_set(ho)
        for f in ("dim", "birth", "death", "birth_pixel", "death_pixel"):
            a, b = getattr(co, f), getattr(ho, f)
            assert a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8)), f
