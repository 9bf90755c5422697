"""Apparent pairs (CPU): the pairs found from their definition (tests/apparent.py)
are pairs of the oracle's full cell pairing, each of length zero.

This pins the rule the GPU stencil implements against the oracle's reduction:
an apparent pair is a persistence pair (the Ripser lineage the paper builds on),
and in this max filtration it has zero length, so removing both cells before
the reduction changes no bar.  The GPU stencil's survivor counts are compared
with the same rule in tests/test_gpu_stencil.py.
"""
import numpy as np
import pytest

import oracle
import synth
from apparent import apparent_pairs, survivors_per_dim


def cases():
    rng = np.random.default_rng(31)
    out = [("uniform 2D", synth.uniform2d((23, 19), 4)),
           ("ties 2D", rng.integers(0, 4, (17, 21)).astype(np.float32)),
           ("field 3D", synth.grf_seeded((9, 8, 10), 1.2, 5)),
           ("ties 3D", rng.integers(0, 3, (7, 8, 6)).astype(np.float32)),
           ("constant 3D", np.full((4, 5, 3), 2.5, np.float32)),
           ("signal", rng.random((1, 40), dtype=np.float32))]
    return out


@pytest.mark.parametrize("label,img", cases(), ids=[c[0] for c in cases()])
def test_apparent_pairs_are_zero_length_pairs_of_the_oracle(label, img):
    s, t, dim, val = apparent_pairs(img)
    assert len(s) > 0
    assert np.all(dim[t] == dim[s] + 1)
    assert np.array_equal(val[s], val[t]), "an apparent pair of positive length"
    o = oracle.persistence(img, cell_pairs=True)
    pairing = set(zip(o.cell_birth.tolist(), o.cell_death.tolist()))
    missing = [(a, b) for a, b in zip(s.tolist(), t.tolist()) if (a, b) not in pairing]
    assert not missing, f"{label}: {len(missing)} apparent pairs are not pairs of the oracle, e.g. {missing[:3]}"


def test_survivor_counts_add_up():
    img = synth.grf_seeded((6, 7, 5), 1.0, 2)
    surv = survivors_per_dim(img)
    s, t, dim, _ = apparent_pairs(img)
    assert sum(surv) + 2 * len(s) == dim.size
