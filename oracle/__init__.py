"""Reference oracle for persistence diagrams of V-construction cubical complexes.

TEST INFRASTRUCTURE ONLY.  The test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers; the GPU product path never
imports, links or executes anything under ``oracle/``.

``cr_oracle.c`` is a plain boundary-matrix reduction over Z/2 in homology (the
standard reduction behind the paper's pivot pairing, Sec. 2 of Kaji-Sudo-Ahara,
"Cubical Ripser"), written from the definitions:

* cell values by the V-construction (maximum over the cell's vertices, Sec. 2);
* a total order key = (value, dim, Khalimsky index) refining the filtration;
* ``mode="plain"``: all columns reduced left to right;
  ``mode="twist"``: dimension by dimension from the top, with clearing (Sec. 2,
  "reduced to zero without computation");
  ``mode="cohomology"``: the paper's own formulation (Sec. 2), the coboundary
  matrix in reverse order, each cell paired with the earliest cofacet its
  reduced column ends on; a second reduction algorithm that must give the same
  pairs (duality of persistent homology and cohomology);
* output: pairs with death > birth and essential bars (death = +inf,
  death_pixel = -1), each with the flat index of the pixel whose value the birth
  (death) cell takes, in canonical order (dim, birth_pixel, death_pixel), an
  essential bar counting as after every finite one.

``lifetime_image`` is the paper's lifetime-enhanced image (Sec. 4, the example
on localised features): for each degree d = 0, 1, 2 an image whose pixel holds
the largest lifetime (death minus birth) among the bars of degree d located at
that pixel (the birth pixel, or the death pixel), zero elsewhere.

``persistence_h0`` is the paper's own description of degree 0 written out:
union-find over the 1-cells in increasing order with the elder rule (Sec. 2,
Fig. 2).  It needs memory linear in the image, so it serves full-size checks of
the 0-th diagram where the full reduction is out of reach.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cr_oracle.c")
_LIB = os.path.join(_HERE, "libcr_oracle.so")
_lib = None

ERR_ARG, ERR_NAN, ERR_TOO_LARGE, ERR_NOMEM = 1, 2, 3, 5


class OracleError(RuntimeError):
    def __init__(self, code: int):
        names = {ERR_ARG: "invalid argument", ERR_NAN: "NaN in input",
                 ERR_TOO_LARGE: "complex too large", ERR_NOMEM: "out of memory"}
        super().__init__(f"oracle error {code}: {names.get(code, '?')}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libcr_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_run.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_void_p)]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_n_pairs.argtypes = [ctypes.c_void_p]
        lib.oracle_n_pairs.restype = ctypes.c_int64
        lib.oracle_n_cell_pairs.argtypes = [ctypes.c_void_p]
        lib.oracle_n_cell_pairs.restype = ctypes.c_int64
        lib.oracle_get_pairs.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
        lib.oracle_get_pairs.restype = None
        lib.oracle_get_cell_pairs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_get_cell_pairs.restype = None
        lib.oracle_h0_run.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_void_p)]
        lib.oracle_h0_run.restype = ctypes.c_int
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Diagram:
    dim: np.ndarray          # int32
    birth: np.ndarray        # float32
    death: np.ndarray        # float32, +inf for essential bars
    birth_pixel: np.ndarray  # int64 flat C-order pixel index
    death_pixel: np.ndarray  # int64, -1 for essential bars
    cell_birth: np.ndarray | None = None  # full cell pairing (zero-length pairs included)
    cell_death: np.ndarray | None = None

    def __len__(self):
        return int(self.dim.shape[0])


def _fetch(lib, handle, cell_pairs=False) -> Diagram:
    n = lib.oracle_n_pairs(handle)
    d = Diagram(np.empty(n, np.int32), np.empty(n, np.float32), np.empty(n, np.float32),
                np.empty(n, np.int64), np.empty(n, np.int64))
    lib.oracle_get_pairs(handle, d.dim.ctypes.data, d.birth.ctypes.data, d.death.ctypes.data,
                         d.birth_pixel.ctypes.data, d.death_pixel.ctypes.data)
    if cell_pairs:
        m = lib.oracle_n_cell_pairs(handle)
        d.cell_birth = np.empty(m, np.int64)
        d.cell_death = np.empty(m, np.int64)
        lib.oracle_get_cell_pairs(handle, d.cell_birth.ctypes.data, d.cell_death.ctypes.data)
    return d


def persistence_h0(img) -> Diagram:
    """Degree-0 diagram of ``img`` by union-find with the elder rule."""
    a = np.ascontiguousarray(np.asarray(img, dtype=np.float32))
    if a.ndim not in (1, 2, 3):
        raise OracleError(ERR_ARG)
    lib = _load()
    shape = (ctypes.c_int64 * a.ndim)(*a.shape)
    handle = ctypes.c_void_p()
    code = lib.oracle_h0_run(a.ctypes.data, a.ndim, shape, ctypes.byref(handle))
    if code != 0:
        raise OracleError(code)
    try:
        return _fetch(lib, handle)
    finally:
        lib.oracle_free(handle)


def persistence(img, maxdim: int | None = None, mode: str = "twist",
                cell_pairs: bool = False) -> Diagram:
    """Diagram of ``img`` (2D or 3D float array, C order) up to ``maxdim``."""
    a = np.ascontiguousarray(np.asarray(img, dtype=np.float32))
    if a.ndim not in (1, 2, 3):
        raise OracleError(ERR_ARG)
    if maxdim is None:
        maxdim = a.ndim - 1
    lib = _load()
    shape = (ctypes.c_int64 * a.ndim)(*a.shape)
    handle = ctypes.c_void_p()
    code = lib.oracle_run(a.ctypes.data, a.ndim, shape, int(maxdim),
                          {"plain": 0, "twist": 1, "cohomology": 2}[mode], ctypes.byref(handle))
    if code != 0:
        raise OracleError(code)
    try:
        return _fetch(lib, handle, cell_pairs)
    finally:
        lib.oracle_free(handle)


def lifetime_image(d: Diagram, shape, location: str = "birth") -> np.ndarray:
    """Channels d = 0, 1, 2 of the lifetime-enhanced image, shape (3, *shape).

    Pixel p of channel k holds the maximum of death - birth (float32
    arithmetic) over the bars of degree k whose location is p, and 0 where there
    is none.  The location is the birth pixel, or with ``location="death"`` the
    death pixel; an essential bar has no death pixel and is then skipped, and
    with birth locations its lifetime is +inf.
    """
    if location not in ("birth", "death"):
        raise OracleError(ERR_ARG)
    n_pix = int(np.prod(shape))
    out = np.zeros((3, n_pix), np.float32)
    pix = d.birth_pixel if location == "birth" else d.death_pixel
    for k, b, e, p in zip(d.dim, d.birth, d.death, pix):
        if p < 0:
            continue
        life = np.float32(e) - np.float32(b)
        if life > out[int(k), int(p)]:
            out[int(k), int(p)] = life
    return out.reshape((3,) + tuple(shape))


def pixel_coords(pixel: np.ndarray, shape) -> np.ndarray:
    """(x, y, z) of each flat pixel index (x the last axis; y, z = 0 beyond the
    image's own axes), -1 for an index of -1: the location columns of the
    paper's output rows (Sec. 3)."""
    pixel = np.asarray(pixel, np.int64)
    out = np.full((len(pixel), 3), -1, np.int64)
    for i, p in enumerate(pixel):
        if p < 0:
            continue
        idx = np.unravel_index(int(p), tuple(shape))
        rev = list(reversed(idx)) + [0] * (3 - len(shape))
        out[i] = rev
    return out
