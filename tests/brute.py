"""Brute-force topology for tiny and mid-sized images, independent of the oracle.

Nothing here reduces a filtration.  It builds the sublevel complex K_t of the
V-construction straight from its definition (a cell is in K_t iff every vertex
of it has value <= t, Sec. 2 of the paper) and measures it with textbook tools:

* ``betti(img, t)``: Betti numbers of K_t.  b0 by flood fill of {phi <= t} with
  4-/6-neighbour connectivity (the paper's connectivity, Sec. 2); the Euler
  characteristic by counting cells of each dimension; in 3D, b2 from the
  bounded 26-connected components of the complement (Alexander duality for
  the (6,26) pair); the remaining Betti number from Euler-Poincare.
* ``persistent_betti(img, k, s, t)``: rank of H_k(K_s) -> H_k(K_t), from GF(2)
  ranks of boundary matrices: dim(Z_k(K_s) + B_k(K_t)) - dim B_k(K_t).
* ``diagram_from_ranks(img)``: the whole (dim, birth, death) multiset recovered
  from persistent Betti numbers by inclusion-exclusion (the "fundamental lemma"
  of persistent homology).  Exact, for grids of a few dozen pixels.
* ``h0_kruskal(img)``: a textbook Kruskal / elder-rule 0-th diagram in Python.
"""
from __future__ import annotations

import itertools
from collections import Counter

import numpy as np
from scipy import ndimage


def _as3d(img):
    a = np.asarray(img, dtype=np.float32)
    a = np.where(a == 0, np.float32(0), a)  # -0.0 -> +0.0
    while a.ndim < 3:
        a = a[None]
    return a


# --------------------------------------------------------------------------- #
# cell enumeration straight from the definition of the cubical complex
# --------------------------------------------------------------------------- #
def cells(img):
    """All cells as (dim, kz, ky, kx, value) with value = max over vertices."""
    a = _as3d(img)
    nz, ny, nx = a.shape
    out = []
    for kz in range(2 * nz - 1):
        for ky in range(2 * ny - 1):
            for kx in range(2 * nx - 1):
                zs = [kz // 2] if kz % 2 == 0 else [kz // 2, kz // 2 + 1]
                ys = [ky // 2] if ky % 2 == 0 else [ky // 2, ky // 2 + 1]
                xs = [kx // 2] if kx % 2 == 0 else [kx // 2, kx // 2 + 1]
                v = max(a[z, y, x] for z in zs for y in ys for x in xs)
                out.append((kz % 2 + ky % 2 + kx % 2, kz, ky, kx, float(v)))
    return out


def _facets(c):
    _, kz, ky, kx, _ = c
    k = [kz, ky, kx]
    res = []
    for ax in range(3):
        if k[ax] % 2 == 1:
            for s in (-1, 1):
                f = list(k)
                f[ax] += s
                res.append(tuple(f))
    return res


# --------------------------------------------------------------------------- #
# Betti numbers of a sublevel set
# --------------------------------------------------------------------------- #
def euler_char(img, t):
    a = _as3d(img) <= t
    chi = 0
    for mask in itertools.product((0, 1), repeat=3):  # which axes the cell spans
        m = a
        for ax, span in enumerate(mask):
            if span:
                sl0 = [slice(None)] * 3
                sl1 = [slice(None)] * 3
                sl0[ax] = slice(0, -1)
                sl1[ax] = slice(1, None)
                m = m[tuple(sl0)] & m[tuple(sl1)]
        chi += (-1) ** sum(mask) * int(m.sum())
    return chi


def betti(img, t):
    """(b0, b1, b2) of the sublevel complex K_t."""
    a = _as3d(img)
    fg = a <= t
    if not fg.any():
        return (0, 0, 0)
    b0 = ndimage.label(fg, structure=ndimage.generate_binary_structure(3, 1))[1]
    # complement, padded by a background layer so the exterior is one component
    bg = np.pad(~fg, 1, constant_values=True)
    if a.shape[0] == 1:  # a 2D image: background 8-connectivity in its plane
        bg2 = np.pad(~fg[0], 1, constant_values=True)
        ncomp = ndimage.label(bg2, structure=np.ones((3, 3), bool))[1]
        b2 = 0
        b1_dual = ncomp - 1
    else:
        ncomp = ndimage.label(bg, structure=np.ones((3, 3, 3), bool))[1]
        b2 = ncomp - 1
        b1_dual = None
    chi = euler_char(img, t)
    b1 = b0 + b2 - chi
    if b1_dual is not None:
        assert b1 == b1_dual, (b1, b1_dual)
    return (b0, b1, b2)


def bars_alive(dims, births, deaths, k, t):
    m = (dims == k) & (births <= t) & (t < deaths)
    return int(m.sum())


# --------------------------------------------------------------------------- #
# GF(2) linear algebra with Python ints as bit vectors
# --------------------------------------------------------------------------- #
def _rank_and_basis(vectors):
    """Row-echelon basis of the span of int bit vectors."""
    basis = {}  # leading bit -> vector
    for v in vectors:
        while v:
            h = v.bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                break
    return basis


def _nullspace(columns, nrows):
    """Basis (as int bit vectors over the column index) of the kernel of the
    GF(2) matrix whose j-th column is the int bit vector columns[j]."""
    n = len(columns)
    # augment each column with an identity tag in bits >= nrows
    rows = [columns[j] | (1 << (nrows + j)) for j in range(n)]
    low_mask = (1 << nrows) - 1
    basis = {}
    kernel = []
    for v in rows:
        while v & low_mask:
            h = (v & low_mask).bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                break
        else:
            kernel.append(v >> nrows)
    return kernel


def persistent_betti_table(img):
    """For k = 0,1,2 and distinct values s <= t: rank H_k(K_s) -> H_k(K_t)."""
    cs = cells(img)
    index = {}
    by_dim = {d: [] for d in range(4)}
    for c in cs:
        index[(c[1], c[2], c[3])] = c
        by_dim[c[0]].append(c)
    pos = {d: {(c[1], c[2], c[3]): i for i, c in enumerate(by_dim[d])} for d in range(4)}
    vals = sorted(set(c[4] for c in cs))

    def bnd(c):
        d = c[0]
        v = 0
        for f in _facets(c):
            v |= 1 << pos[d - 1][f]
        return v

    boundary = {d: [bnd(c) if d > 0 else 0 for c in by_dim[d]] for d in range(4)}
    table = {}
    for k in range(3):
        for si, s in enumerate(vals):
            # cycles of K_s in degree k, as vectors over k-cells
            kcells = [i for i, c in enumerate(by_dim[k]) if c[4] <= s]
            if k == 0:
                Z = [1 << i for i in kcells]
            else:
                cols = [boundary[k][i] for i in kcells]
                ker = _nullspace(cols, max(1, len(by_dim[k - 1])))
                Z = []
                for kv in ker:
                    z = 0
                    j = 0
                    while kv:
                        if kv & 1:
                            z |= 1 << kcells[j]
                        kv >>= 1
                        j += 1
                    Z.append(z)
            for t in vals[si:]:
                B = [boundary[k + 1][i] for i, c in enumerate(by_dim[k + 1]) if c[4] <= t] \
                    if k + 1 <= 3 else []
                rb = len(_rank_and_basis(B))
                rzb = len(_rank_and_basis(B + Z))
                table[(k, s, t)] = rzb - rb
    return vals, table


def diagram_from_ranks(img):
    """Multiset of (dim, birth, death) bars with death > birth (death = inf for
    essential bars), by inclusion-exclusion of persistent Betti numbers."""
    vals, table = persistent_betti_table(img)
    m = len(vals)

    def beta(k, i, j):  # i, j are indices into vals; i = -1 means "before the first value"
        if i < 0:
            return 0
        return table[(k, vals[i], vals[j])]

    bars = Counter()
    for k in range(3):
        for i in range(m):
            for j in range(i + 1, m):
                mu = beta(k, i, j - 1) - beta(k, i - 1, j - 1) - beta(k, i, j) + beta(k, i - 1, j)
                if mu:
                    bars[(k, vals[i], vals[j])] += mu
            mu_inf = beta(k, i, m - 1) - beta(k, i - 1, m - 1)
            if mu_inf:
                bars[(k, vals[i], float("inf"))] += mu_inf
    assert all(v > 0 for v in bars.values())
    return bars


def diagram_counter(dims, births, deaths):
    return Counter((int(d), float(b), float(e)) for d, b, e in zip(dims, births, deaths))


# --------------------------------------------------------------------------- #
# textbook 0-th persistence (Kruskal with the elder rule)
# --------------------------------------------------------------------------- #
def h0_kruskal(img):
    """Multiset of (0, birth, death) bars; ties between equal values are broken
    arbitrarily, which cannot change bars of positive length."""
    a = _as3d(img)
    nz, ny, nx = a.shape
    flat = a.ravel()
    edges = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                p = (z * ny + y) * nx + x
                for dz, dy, dx in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    if z + dz < nz and y + dy < ny and x + dx < nx:
                        q = ((z + dz) * ny + y + dy) * nx + x + dx
                        edges.append((max(flat[p], flat[q]), p, q))
    edges.sort()
    parent = list(range(flat.size))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    bars = Counter()
    for w, p, q in edges:
        rp, rq = find(p), find(q)
        if rp == rq:
            continue
        if (flat[rp], rp) < (flat[rq], rq):
            rp, rq = rq, rp  # rp is younger
        if w > flat[rp]:
            bars[(0, float(flat[rp]), float(w))] += 1
        parent[rp] = rq
    root = find(0)
    bars[(0, float(flat[root]), float("inf"))] += 1
    return bars
