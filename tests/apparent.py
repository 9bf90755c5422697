"""Apparent pairs of a V-construction cubical complex, written out in NumPy
from the definitions (test infrastructure; shares nothing with the oracle or
the GPU path).

Cells are addressed by Khalimsky coordinates (0 <= c_a <= 2 n_a - 2, an odd
coordinate meaning the cell extends along that axis); a cell's value is the
maximum of its vertex pixels (the V-construction, Sec. 2 of the paper); cells
are ordered by (value, dimension, flat Khalimsky index).  The earliest
cofacet of a cell is its cofacet smallest in that order, its latest facet the
facet largest in it; a cell s and a cell t form an apparent pair when t is the
earliest cofacet of s and s the latest facet of t.  Such pairs are pairs of
the persistence pairing with zero length, so a correct pairing contains them.
"""
import numpy as np


def khalimsky_values(img: np.ndarray) -> np.ndarray:
    """Values of all cells, shape (2n-1) per axis of the image as a volume
    (a 2D image gets a leading axis of extent 1)."""
    a = np.asarray(img, np.float32)
    a = np.where(a == 0, np.float32(0), a)  # -0.0 reads as +0.0
    while a.ndim < 3:
        a = a[None]
    K = tuple(2 * n - 1 for n in a.shape)
    v = np.full(K, -np.inf, np.float32)
    v[::2, ::2, ::2] = a
    for ax in range(3):  # an odd coordinate: the max of the two cells beside it
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        mid = [slice(None)] * 3
        lo[ax], hi[ax], mid[ax] = slice(0, -1, 2), slice(2, None, 2), slice(1, None, 2)
        v[tuple(mid)] = np.maximum(v[tuple(lo)], v[tuple(hi)])
    return v


def apparent_pairs(img: np.ndarray):
    """(lower kidx, upper kidx) arrays of the apparent pairs, and the cell dims."""
    v = khalimsky_values(img)
    K = v.shape
    kidx = np.arange(v.size, dtype=np.int64).reshape(K)
    par = [np.indices(K)[a] & 1 for a in range(3)]
    dim = par[0] + par[1] + par[2]
    big = np.iinfo(np.int64).max
    # earliest cofacet: neighbours along an axis where the cell is even
    ecf_v = np.full(K, np.inf, np.float32)
    ecf_k = np.full(K, big, np.int64)
    # latest facet: neighbours along an axis where the cell is odd
    lf_v = np.full(K, -np.inf, np.float32)
    lf_k = np.full(K, -1, np.int64)
    for ax in range(3):
        for step in (-1, 1):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if step < 0:
                dst[ax], src[ax] = slice(1, None), slice(0, -1)
            else:
                dst[ax], src[ax] = slice(0, -1), slice(1, None)
            dst, src = tuple(dst), tuple(src)
            nv, nk = v[src], kidx[src]
            even = par[ax][dst] == 0
            better = even & ((nv < ecf_v[dst]) | ((nv == ecf_v[dst]) & (nk < ecf_k[dst])))
            ecf_v[dst] = np.where(better, nv, ecf_v[dst])
            ecf_k[dst] = np.where(better, nk, ecf_k[dst])
            odd = ~even
            later = odd & ((nv > lf_v[dst]) | ((nv == lf_v[dst]) & (nk > lf_k[dst])))
            lf_v[dst] = np.where(later, nv, lf_v[dst])
            lf_k[dst] = np.where(later, nk, lf_k[dst])
    flat_ecf = ecf_k.ravel()
    flat_lf = lf_k.ravel()
    s = np.flatnonzero(flat_ecf != big)
    t = flat_ecf[s]
    keep = flat_lf[t] == s
    return s[keep], t[keep], dim.ravel(), v.ravel()


def survivors_per_dim(img: np.ndarray) -> list:
    """Cells of each dimension 0..3 left after removing the apparent pairs."""
    s, t, dim, _ = apparent_pairs(img)
    total = np.bincount(dim, minlength=4)
    gone = np.bincount(dim[s], minlength=4) + np.bincount(dim[t], minlength=4)
    return (total - gone).tolist()
