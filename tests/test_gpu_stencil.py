"""The stencil pass (filtration values, apparent pairs, survivor compaction)
on its own: the number of surviving cells of each dimension that the GPU
reports after a call equals the count left by the apparent pairs found on the
CPU from their definition (tests/apparent.py, itself pinned to the oracle's
cell pairing by tests/test_apparent.py).  The inputs span several stencil
tiles in every axis with ragged edges, and include ties, +inf (masked) pixels
and a 1D signal.
"""
import numpy as np
import pytest
import torch

import paper_2005_12692_amd as cr
import synth
from apparent import survivors_per_dim

pytestmark = pytest.mark.gpu


def cases():
    rng = np.random.default_rng(41)
    ball = synth.ball_mask((47, 40, 71))
    masked = np.where(ball, synth.grf_seeded((47, 40, 71), 2.0, 3), np.float32(np.inf)).astype(np.float32)
    return [("field 3D", synth.grf_seeded((70, 40, 45), 1.5, 1)),
            ("blobs 3D", synth.blobs3d(50, 6)),
            ("ties 3D", rng.integers(0, 5, (35, 30, 129)).astype(np.float32)),
            ("masked 3D", masked),
            ("uniform 2D", synth.uniform2d((300, 130), 2)),
            ("ties 2D", rng.integers(0, 3, (77, 190)).astype(np.float32)),
            ("signal", synth.random_walk(5000))]


@pytest.mark.parametrize("label,img", cases(), ids=[c[0] for c in cases()])
def test_survivors_per_dimension(label, img):
    cr.persistence(torch.from_numpy(np.ascontiguousarray(img)).cuda())
    got = cr.stats()["survivors"]
    want = survivors_per_dim(img if img.ndim > 1 else img[None])
    assert got == want, f"{label}: GPU survivors per dimension {got}, apparent pairs leave {want}"


@pytest.mark.parametrize("stage", ["0", "100", "700"])
def test_survivor_staging(monkeypatch, stage):
    """In a volume the stencil stages each plane's survivor keys in LDS and
    writes them out one plane later; a plane with more survivors than the
    staging holds is written straight out.  With the capacity lowered
    (CR_STAGE_KEYS: 0 writes every plane straight out, 100 and 700 mix the two
    ways from plane to plane) the survivor counts and the whole diagram still
    equal the apparent-pair count and the oracle's diagram."""
    import oracle
    monkeypatch.setenv("CR_STAGE_KEYS", stage)
    rng = np.random.default_rng(43)
    for label, img in [("blobs 3D", synth.blobs3d(50, 6)),
                       ("ties 3D", rng.integers(0, 5, (35, 30, 129)).astype(np.float32)),
                       ("uniform 3D", rng.random((33, 40, 70), dtype=np.float32))]:
        d = cr.persistence(torch.from_numpy(np.ascontiguousarray(img)).cuda())
        assert cr.stats()["survivors"] == survivors_per_dim(img), f"{label} stage {stage}: survivor counts"
        o = oracle.persistence(img)
        for name, g, w in zip(("dim", "birth", "death", "birth_pixel", "death_pixel"), d,
                              (o.dim, o.birth, o.death, o.birth_pixel, o.death_pixel)):
            g = g.cpu().numpy()
            assert g.shape == w.shape and np.array_equal(g.view(np.uint8), w.view(np.uint8)), \
                f"{label} stage {stage}: field {name} differs from the oracle"
