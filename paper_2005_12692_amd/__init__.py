"""Python binding of libcr: persistent homology of images and volumes on an MI355X.

Thin ctypes layer over the C ABI declared in ``include/cr.h``; it only marshals
arguments.  Every stage of the computation runs in the HIP kernels of
``libcr.so``; PyTorch provides device memory and streams.  There is no CPU
fallback: if the library is missing, every call raises.

    import torch, paper_2005_12692_amd as cr
    d = cr.persistence(torch.rand(512, 512, device="cuda"))
    d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel   # device tensors

Bars follow Kaji-Sudo-Ahara, "Cubical Ripser" (Sec. 1-2): [birth, death) of
dimension 0..ndim-1 for the V-construction cubical complex (a cell takes the
maximum of its vertices), Z/2 coefficients, 4-/6-neighbour connectivity.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcr.so")

CR_OK, CR_ERR_INVALID_ARGUMENT, CR_ERR_NAN_INPUT, CR_ERR_TOO_LARGE = 0, 1, 2, 3
CR_ERR_CAPACITY, CR_ERR_OUT_OF_MEMORY, CR_ERR_HIP, CR_ERR_INTERNAL = 4, 5, 6, 7


class CRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libcr error {code}: {msg}")
        self.code = code


class _Diagram(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_void_p), ("birth", ctypes.c_void_p),
                ("death", ctypes.c_void_p), ("birth_pixel", ctypes.c_void_p),
                ("death_pixel", ctypes.c_void_p), ("block", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_pixels", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("survivors", ctypes.c_int64 * 4), ("n_rows", ctypes.c_int64),
                ("arena_used", ctypes.c_int64), ("red_adds", ctypes.c_int64),
                ("red_merged", ctypes.c_int64),
                ("red_rounds", ctypes.c_int64), ("arena_reruns", ctypes.c_int64),
                ("scratch_bytes", ctypes.c_int64), ("tuning_from_cache", ctypes.c_int64)]


class _Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("grid", ctypes.c_int32), ("long_len", ctypes.c_int32),
                ("yield_iters", ctypes.c_int32), ("wave_short", ctypes.c_int32), ("front_cap", ctypes.c_int32),
                ("wave_yield", ctypes.c_int32), ("group_max", ctypes.c_int32), ("narrow_min", ctypes.c_int32)]


TUNING_FIELDS = tuple(f for f, _ in _Tuning._fields_)

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_ctx = {}        # device index -> cr_context*
_live = {}       # data_ptr -> tensor handed to the library by the allocator callback
_alloc_dev = [0]


def _py_alloc(nbytes, stream, user):
    try:
        t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{_alloc_dev[0]}")
    except Exception:  # the library reports CR_ERR_OUT_OF_MEMORY
        return None
    _live[t.data_ptr()] = t
    return t.data_ptr()


def _py_free(ptr, stream, user):
    _live.pop(ptr, None)


_alloc_cb = _ALLOC_FN(_py_alloc)
_free_cb = _FREE_FN(_py_free)


def lib():
    """The loaded libcr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CRError(CR_ERR_HIP, f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2005_12692_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.cr_create.argtypes = [ctypes.POINTER(vp), i32, _ALLOC_FN, _FREE_FN, vp]
        L.cr_destroy.argtypes = [vp]
        L.cr_destroy.restype = None
        L.cr_last_error.restype = ctypes.c_char_p
        L.cr_persistence.argtypes = [vp, vp, i32, ctypes.POINTER(i64), i32, ctypes.c_uint32, vp,
                                     ctypes.POINTER(_Diagram)]
        L.cr_diagram_free.argtypes = [vp, ctypes.POINTER(_Diagram)]
        L.cr_diagram_free.restype = None
        L.cr_persistence_batched.argtypes = [vp, i32, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i32, i32,
                                             ctypes.c_uint32, vp, vp, vp, vp, vp, vp, i64, vp, vp]
        L.cr_persistence_batched_noalloc.argtypes = L.cr_persistence_batched.argtypes
        L.cr_sync_status.argtypes = [vp, vp]
        L.cr_persistence_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, i64, vp]
        L.cr_lifetime_image.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, vp, i64, vp]
        L.cr_pixel_coords.argtypes = [vp, vp, i64, i64, i32, ctypes.POINTER(i64), vp, vp]
        L.cr_batched_workspace_size.argtypes = [vp, i32, ctypes.POINTER(i64), i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.cr_reserve.argtypes = [vp, ctypes.c_size_t]
        L.cr_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.cr_get_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)]
        batch = [vp, i32, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i32, i32]
        outs = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.cr_get_tuning.argtypes = [vp, i32, ctypes.POINTER(_Tuning)]
        L.cr_set_tuning.argtypes = [vp, i32, ctypes.POINTER(_Tuning)]
        L.cr_tile_variants.argtypes = [i32]
        L.cr_tile_shape.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_int32)]
        L.cr_autotune_batched.argtypes = batch + [vp] + outs + [i32, ctypes.POINTER(_Tuning)]
        L.cr_batched_graph_create.argtypes = batch + [ctypes.c_uint32, vp] + outs + [ctypes.POINTER(vp)]
        L.cr_graph_launch.argtypes = [vp, vp]
        L.cr_graph_sync_status.argtypes = [vp, vp]
        L.cr_graph_destroy.argtypes = [vp]
        L.cr_graph_destroy.restype = None
        for f in ("cr_create", "cr_persistence", "cr_persistence_batched", "cr_persistence_batched_noalloc",
                  "cr_sync_status",
                  "cr_persistence_backward", "cr_lifetime_image", "cr_pixel_coords", "cr_batched_workspace_size",
                  "cr_reserve", "cr_get_stats", "cr_get_stage_times", "cr_get_tuning",
                  "cr_set_tuning", "cr_tile_variants", "cr_tile_shape", "cr_autotune_batched",
                  "cr_batched_graph_create", "cr_graph_launch", "cr_graph_sync_status"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != CR_OK:
        raise CRError(code, lib().cr_last_error().decode(errors="replace"))


def _context(device: torch.device):
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _ctx:
        h = ctypes.c_void_p()
        _check(lib().cr_create(ctypes.byref(h), idx, _alloc_cb, _free_cb, None))
        _ctx[idx] = h
    return _ctx[idx], idx


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Diagram(NamedTuple):
    dim: torch.Tensor          # int32
    birth: torch.Tensor        # float32
    death: torch.Tensor        # float32, +inf for essential bars
    birth_pixel: torch.Tensor  # int64 flat index into the input
    death_pixel: torch.Tensor  # int64, -1 for essential bars


def _check_image(image: torch.Tensor, ndims=(1, 2, 3)) -> torch.Tensor:
    if not isinstance(image, torch.Tensor) or image.device.type != "cuda":
        raise TypeError("image must be a CUDA (HIP) tensor")
    if image.dtype != torch.float32:
        raise TypeError("image must be float32")
    if image.dim() not in ndims:
        raise ValueError(f"image must have {ndims} dimensions")
    return image.contiguous()


def _view(block: torch.Tensor, base: int, ptr: int, n: int, dtype, itemsize: int) -> torch.Tensor:
    off = ptr - base
    return block[off:off + n * itemsize].view(dtype)


CR_FLAG_STAGE_TIMES = 1
STAGES = ("stencil", "sort_cells", "degree0", "degree1", "degree2", "sort_rows")


def persistence(image: torch.Tensor, maxdim: int | None = None, stage_times: bool = False) -> Diagram:
    """Persistence diagram of a 1D signal, 2D image or 3D volume (float32, on the GPU).

    With ``stage_times`` the library records HIP events between its stages;
    read them with ``stage_times()``."""
    image = _check_image(image)
    h, dev = _context(image.device)
    if maxdim is None:
        maxdim = image.dim() - 1
    shape = (ctypes.c_int64 * image.dim())(*image.shape)
    out = _Diagram()
    _alloc_dev[0] = dev
    _check(lib().cr_persistence(h, ctypes.c_void_p(image.data_ptr()), image.dim(), shape, int(maxdim),
                                CR_FLAG_STAGE_TIMES if stage_times else 0,
                                _stream(image.device), ctypes.byref(out)))
    n = int(out.n)
    if n == 0:
        z = lambda dt: torch.empty(0, dtype=dt, device=image.device)
        return Diagram(z(torch.int32), z(torch.float32), z(torch.float32), z(torch.int64), z(torch.int64))
    block = _live.pop(out.block)
    base = out.block
    return Diagram(_view(block, base, out.dim, n, torch.int32, 4),
                   _view(block, base, out.birth, n, torch.float32, 4),
                   _view(block, base, out.death, n, torch.float32, 4),
                   _view(block, base, out.birth_pixel, n, torch.int64, 8),
                   _view(block, base, out.death_pixel, n, torch.int64, 8))


class BatchedDiagram(NamedTuple):
    dim: torch.Tensor
    birth: torch.Tensor
    death: torch.Tensor
    birth_pixel: torch.Tensor   # index into the packed buffer
    death_pixel: torch.Tensor
    pair_offsets: torch.Tensor  # int64 [n_images + 1] (device)
    status: torch.Tensor        # int32 [n_images] (device)

    def image(self, i: int, offsets=None) -> Diagram:
        o = self.pair_offsets.cpu() if offsets is None else offsets
        a, b = int(o[i]), int(o[i + 1])
        return Diagram(self.dim[a:b], self.birth[a:b], self.death[a:b], self.birth_pixel[a:b],
                       self.death_pixel[a:b])


def pack(images: Sequence[torch.Tensor]):
    """Packs images of one ndim into one buffer; returns (packed, shapes, pixel_offsets)."""
    shapes = [tuple(int(s) for s in t.shape) for t in images]
    packed = torch.cat([t.reshape(-1) for t in images])
    offs = [0]
    for s in shapes:
        n = 1
        for e in s:
            n *= e
        offs.append(offs[-1] + n)
    return packed, shapes, offs


def persistence_batched(packed: torch.Tensor, shapes, pixel_offsets=None, maxdim: int | None = None,
                        capacity: int | None = None, out: BatchedDiagram | None = None,
                        check: bool = True, _arena_retries: int = 3) -> BatchedDiagram:
    """Diagrams of many images (one ndim) packed in one buffer, in one pass.

    ``capacity`` rows are allocated (default: one per pixel).  With ``check``
    the call synchronises, raises on device-side errors and retries once with
    the exact capacity if the rows did not fit, and again (at most three times)
    if the reduction's column arena ran out (the context's arena has grown by
    then).  With ``check=False`` and a preallocated ``out`` the call neither
    allocates nor synchronises (it can be captured in a HIP graph once the same
    shapes have been run before); ``out.status`` then holds each image's
    status once the stream has completed.
    """
    if packed.device.type != "cuda" or packed.dtype != torch.float32 or not packed.is_contiguous():
        raise TypeError("packed must be a contiguous float32 CUDA tensor")
    shapes = [tuple(int(e) for e in s) for s in shapes]
    ndim = len(shapes[0])
    if any(len(s) != ndim for s in shapes):
        raise ValueError("all images must have the same ndim")
    if pixel_offsets is None:
        pixel_offsets = [0]
        for s in shapes:
            n = 1
            for e in s:
                n *= e
            pixel_offsets.append(pixel_offsets[-1] + n)
    if maxdim is None:
        maxdim = ndim - 1
    nimg = len(shapes)
    h, dev = _context(packed.device)
    flat = [e for s in shapes for e in s]
    c_shapes = (ctypes.c_int64 * len(flat))(*flat)
    c_offs = (ctypes.c_int64 * (nimg + 1))(*pixel_offsets)
    if out is None:
        cap = int(pixel_offsets[-1]) if capacity is None else int(capacity)
        dv = packed.device
        out = BatchedDiagram(torch.empty(cap, dtype=torch.int32, device=dv),
                             torch.empty(cap, dtype=torch.float32, device=dv),
                             torch.empty(cap, dtype=torch.float32, device=dv),
                             torch.empty(cap, dtype=torch.int64, device=dv),
                             torch.empty(cap, dtype=torch.int64, device=dv),
                             torch.empty(nimg + 1, dtype=torch.int64, device=dv),
                             torch.empty(nimg, dtype=torch.int32, device=dv))
    cap = out.dim.shape[0]
    stream = _stream(packed.device)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    _check(lib().cr_persistence_batched(h, nimg, p(packed), c_offs, c_shapes, ndim, int(maxdim), 0, stream,
                                        p(out.dim), p(out.birth), p(out.death), p(out.birth_pixel),
                                        p(out.death_pixel), cap, p(out.pair_offsets), p(out.status)))
    if not check:
        return out
    code = lib().cr_sync_status(h, stream)
    if code == CR_ERR_OUT_OF_MEMORY and b"column-arena" in lib().cr_last_error() and _arena_retries > 0:
        return persistence_batched(packed, shapes, pixel_offsets, maxdim, capacity=capacity, check=True,
                                   _arena_retries=_arena_retries - 1)
    total = int(out.pair_offsets[-1])
    if total > cap:
        return persistence_batched(packed, shapes, pixel_offsets, maxdim, capacity=total, check=True,
                                   _arena_retries=_arena_retries)
    _check(code)
    return BatchedDiagram(out.dim[:total], out.birth[:total], out.death[:total], out.birth_pixel[:total],
                          out.death_pixel[:total], out.pair_offsets, out.status)


def persistence_batched_noalloc(packed: torch.Tensor, shapes, out: BatchedDiagram, pixel_offsets=None,
                                maxdim: int | None = None) -> BatchedDiagram:
    """cr_persistence_batched_noalloc: the batched call on the library's static
    device scratch, into the caller's preallocated ``out`` (see ``_empty_out``).
    Neither allocates nor synchronises; read ``out.pair_offsets`` and
    ``out.status`` (or call ``sync_status``) after the stream completes."""
    args, ndim, nimg, _, _, _ = _batch_prefix(packed, shapes, pixel_offsets, maxdim)
    if out.pair_offsets.shape[0] != nimg + 1 or out.status.shape[0] != nimg:
        raise ValueError("out does not match the number of images")
    _check(lib().cr_persistence_batched_noalloc(*args, 0, _stream(packed.device), *_out_args(out)))
    return out


def sync_status(device=None) -> None:
    """cr_sync_status: waits for the current stream and raises on a device-side
    error of the last batched call on the device's context."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    _check(lib().cr_sync_status(h, _stream(dev)))


def _batch_prefix(packed, shapes, pixel_offsets, maxdim):
    if packed.device.type != "cuda" or packed.dtype != torch.float32 or not packed.is_contiguous():
        raise TypeError("packed must be a contiguous float32 CUDA tensor")
    shapes = [tuple(int(e) for e in s) for s in shapes]
    ndim = len(shapes[0])
    if any(len(s) != ndim for s in shapes):
        raise ValueError("all images must have the same ndim")
    if pixel_offsets is None:
        pixel_offsets = [0]
        for s in shapes:
            n = 1
            for e in s:
                n *= e
            pixel_offsets.append(pixel_offsets[-1] + n)
    if maxdim is None:
        maxdim = ndim - 1
    nimg = len(shapes)
    h, _ = _context(packed.device)
    flat = [e for s in shapes for e in s]
    c_shapes = (ctypes.c_int64 * len(flat))(*flat)
    c_offs = (ctypes.c_int64 * (nimg + 1))(*pixel_offsets)
    args = [h, nimg, ctypes.c_void_p(packed.data_ptr()), c_offs, c_shapes, ndim, int(maxdim)]
    return args, ndim, nimg, pixel_offsets, shapes, maxdim


def _empty_out(n_rows: int, nimg: int, device) -> BatchedDiagram:
    return BatchedDiagram(torch.empty(n_rows, dtype=torch.int32, device=device),
                          torch.empty(n_rows, dtype=torch.float32, device=device),
                          torch.empty(n_rows, dtype=torch.float32, device=device),
                          torch.empty(n_rows, dtype=torch.int64, device=device),
                          torch.empty(n_rows, dtype=torch.int64, device=device),
                          torch.empty(nimg + 1, dtype=torch.int64, device=device),
                          torch.empty(nimg, dtype=torch.int32, device=device))


def empty_batched_output(n_rows: int, n_images: int, device) -> BatchedDiagram:
    """Output buffers for a batched call of n_images with room for n_rows rows
    (uninitialised), e.g. for persistence_batched_noalloc or check=False."""
    return _empty_out(n_rows, n_images, device)


def _out_args(out: BatchedDiagram):
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    return [p(out.dim), p(out.birth), p(out.death), p(out.birth_pixel), p(out.death_pixel), out.dim.shape[0],
            p(out.pair_offsets), p(out.status)]


def get_tuning(ndim: int, device=None) -> dict:
    """Launch parameters the context uses for ndim (see cr_tuning in cr.h)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    t = _Tuning()
    _check(lib().cr_get_tuning(h, ndim, ctypes.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def set_tuning(ndim: int, device=None, **fields) -> dict:
    """Sets some launch parameters for ndim; returns the full setting."""
    cur = get_tuning(ndim, device)
    unknown = set(fields) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    cur.update({k: int(v) for k, v in fields.items()})
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    _check(lib().cr_set_tuning(h, ndim, ctypes.byref(_Tuning(**cur))))
    return cur


def tile_shapes(ndim: int) -> list:
    """Extents (z, y, x) of the stencil tile variants for ndim."""
    out = []
    for v in range(lib().cr_tile_variants(ndim)):
        e = (ctypes.c_int32 * 3)()
        _check(lib().cr_tile_shape(ndim, v, e))
        out.append(tuple(int(x) for x in e))
    return out


def autotune(packed: torch.Tensor, shapes, pixel_offsets=None, maxdim: int | None = None,
             capacity: int | None = None, repeats: int = 2) -> dict:
    """Runs the library's autotuner on this batch (see cr_autotune_batched) and
    returns the chosen launch parameters, which the context keeps for this ndim."""
    args, ndim, nimg, offs, shapes, maxdim = _batch_prefix(packed, shapes, pixel_offsets, maxdim)
    cap = int(offs[-1]) if capacity is None else int(capacity)
    out = _empty_out(cap, nimg, packed.device)
    t = _Tuning()
    _check(lib().cr_autotune_batched(*args, _stream(packed.device), *_out_args(out), int(repeats), ctypes.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


class BatchedGraph:
    """A batched call captured once in a HIP graph (cr_batched_graph_create) and
    replayed with launch().  The packed input tensor is read at each replay, so
    refreshed pixel values of the same shapes need no new graph; the rows land in
    the fixed buffers of ``out`` (call result() after a replay)."""

    def __init__(self, packed: torch.Tensor, shapes, pixel_offsets=None, maxdim: int | None = None,
                 capacity: int | None = None):
        args, ndim, nimg, offs, shapes, maxdim = _batch_prefix(packed, shapes, pixel_offsets, maxdim)
        self.packed = packed  # keeps the captured input buffer alive
        cap = int(offs[-1]) if capacity is None else int(capacity)
        self.out = _empty_out(cap, nimg, packed.device)
        self.capture_stream = torch.cuda.Stream(packed.device)
        self.capture_stream.wait_stream(torch.cuda.current_stream(packed.device))
        g = ctypes.c_void_p()
        torch.cuda.synchronize(packed.device)
        _check(lib().cr_batched_graph_create(*args, 0, ctypes.c_void_p(self.capture_stream.cuda_stream),
                                             *_out_args(self.out), ctypes.byref(g)))
        self._g = g
        self.device = packed.device

    def launch(self, stream: torch.cuda.Stream | None = None):
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        _check(lib().cr_graph_launch(self._g, ctypes.c_void_p(s.cuda_stream)))

    def result(self, check: bool = True) -> BatchedDiagram:
        """Rows of the last replay (synchronises the current stream)."""
        s = torch.cuda.current_stream(self.device)
        code = lib().cr_graph_sync_status(self._g, ctypes.c_void_p(s.cuda_stream))
        total = int(self.out.pair_offsets[-1])
        if total > self.out.dim.shape[0]:
            raise CRError(CR_ERR_CAPACITY, f"{total} rows do not fit the capacity {self.out.dim.shape[0]}")
        if check:
            _check(code)
        o = self.out
        return BatchedDiagram(o.dim[:total], o.birth[:total], o.death[:total], o.birth_pixel[:total],
                              o.death_pixel[:total], o.pair_offsets, o.status)

    def close(self):
        if getattr(self, "_g", None) and self._g.value:
            lib().cr_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def backward(birth_pixel: torch.Tensor, death_pixel: torch.Tensor, grad_birth: torch.Tensor | None,
             grad_death: torch.Tensor | None, grad_image: torch.Tensor) -> torch.Tensor:
    """grad_image[birth_pixel] += grad_birth; grad_image[death_pixel] += grad_death (in place)."""
    h, _ = _context(grad_image.device)
    n = int(birth_pixel.shape[0])
    gb = None if grad_birth is None else grad_birth.contiguous().float()
    gd = None if grad_death is None else grad_death.contiguous().float()
    p = lambda t: ctypes.c_void_p(0 if t is None else t.data_ptr())
    _check(lib().cr_persistence_backward(h, p(birth_pixel.contiguous()), p(death_pixel.contiguous()), p(gb),
                                         p(gd), n, p(grad_image), grad_image.numel(), _stream(grad_image.device)))
    return grad_image


def workspace_size(shapes, maxdim: int | None = None, device=None) -> int:
    """Device scratch bytes a batched call of images of these shapes needs."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    shapes = [tuple(int(x) for x in s) for s in shapes]
    ndim = len(shapes[0])
    if any(len(s) != ndim for s in shapes):
        raise ValueError("all images must have the same ndim")
    flat = (ctypes.c_int64 * (ndim * len(shapes)))(*[x for s in shapes for x in s])
    out = ctypes.c_size_t()
    _check(lib().cr_batched_workspace_size(h, len(shapes), flat, ndim, ndim - 1 if maxdim is None else int(maxdim),
                                           ctypes.byref(out)))
    return int(out.value)


def reserve(nbytes: int, device=None) -> None:
    """Reserves device scratch so that batched calls needing at most nbytes allocate nothing."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    _check(lib().cr_reserve(h, int(nbytes)))


def lifetime_image(d, n_pixels: int, location: str = "birth") -> torch.Tensor:
    """The three persistence channels of the lifetime-enhanced image (Sec. 4):
    channel k holds at each pixel the largest lifetime (death - birth) of the
    bars of degree k located there (their birth or death pixel), 0 elsewhere.

    ``d`` is a Diagram or a BatchedDiagram; ``n_pixels`` the image size (or the
    packed size).  Returns a flat (3, n_pixels) float32 tensor: reshape a plain
    image's channels with ``.view(3, *shape)``; image i of a batch has
    ``out[:, pixel_offsets[i]:pixel_offsets[i + 1]]``."""
    if location not in ("birth", "death"):
        raise ValueError("location must be 'birth' or 'death'")
    dev = d.birth.device
    h, _ = _context(dev)
    out = torch.empty((3, int(n_pixels)), dtype=torch.float32, device=dev)
    t = [x.contiguous() for x in (d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel)]
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    _check(lib().cr_lifetime_image(h, *(p(x) for x in t), int(t[0].shape[0]), 1 if location == "death" else 0,
                                   p(out), int(n_pixels), _stream(dev)))
    return out


def pixel_coords(pixel: torch.Tensor, shape, base: int = 0) -> torch.Tensor:
    """(x, y, z) int32 rows of flat pixel indices (minus ``base``) in an image of
    ``shape``: the location columns of the paper's output rows; -1 gives
    (-1, -1, -1)."""
    dev = pixel.device
    h, _ = _context(dev)
    pixel = pixel.contiguous()
    n = int(pixel.shape[0])
    out = torch.empty((n, 3), dtype=torch.int32, device=dev)
    shp = (ctypes.c_int64 * len(shape))(*[int(x) for x in shape])
    _check(lib().cr_pixel_coords(h, ctypes.c_void_p(pixel.data_ptr()), n, int(base), len(shape), shp,
                                 ctypes.c_void_p(out.data_ptr()), _stream(dev)))
    return out


class PersistenceFn(torch.autograd.Function):
    """(dim, birth, death, birth_pixel, death_pixel) of an image, differentiable
    in birth and death: birth = image[birth_pixel], death = image[death_pixel]."""

    @staticmethod
    def forward(ctx, image, maxdim=None):
        d = persistence(image.detach(), maxdim)
        ctx.save_for_backward(d.birth_pixel, d.death_pixel)
        ctx.shape = image.shape
        ctx.mark_non_differentiable(d.dim, d.birth_pixel, d.death_pixel)
        return d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel

    @staticmethod
    def backward(ctx, g_dim, g_birth, g_death, g_bp, g_dp):
        bp, dp = ctx.saved_tensors
        grad = torch.zeros(ctx.shape, dtype=torch.float32, device=bp.device)
        backward(bp, dp, g_birth, g_death, grad)
        return grad, None


class PersistenceBatchedFn(torch.autograd.Function):
    """Batched form of PersistenceFn over a packed buffer."""

    @staticmethod
    def forward(ctx, packed, shapes, maxdim=None):
        d = persistence_batched(packed.detach(), shapes, maxdim=maxdim)
        ctx.save_for_backward(d.birth_pixel, d.death_pixel)
        ctx.n = packed.numel()
        ctx.mark_non_differentiable(d.dim, d.birth_pixel, d.death_pixel, d.pair_offsets)
        return d.dim, d.birth, d.death, d.birth_pixel, d.death_pixel, d.pair_offsets

    @staticmethod
    def backward(ctx, g_dim, g_birth, g_death, g_bp, g_dp, g_off):
        bp, dp = ctx.saved_tensors
        grad = torch.zeros(ctx.n, dtype=torch.float32, device=bp.device)
        backward(bp, dp, g_birth, g_death, grad)
        return grad, None, None


def stage_times(device=None) -> dict:
    """Stage durations (ms) of the last ``persistence(..., stage_times=True)`` call."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    ms = (ctypes.c_float * 6)()
    n = ctypes.c_int()
    _check(lib().cr_get_stage_times(h, ms, 6, ctypes.byref(n)))
    return {name: float(ms[i]) for i, name in enumerate(STAGES)}


def stats(device=None) -> dict:
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    h, _ = _context(dev)
    s = _Stats()
    _check(lib().cr_get_stats(h, ctypes.byref(s)))
    return {"n_pixels": s.n_pixels, "n_cells": s.n_cells, "survivors": list(s.survivors),
            "n_rows": s.n_rows, "arena_used": s.arena_used, "red_adds": s.red_adds,
            "red_merged": s.red_merged, "red_rounds": s.red_rounds,
            "arena_reruns": s.arena_reruns, "scratch_bytes": s.scratch_bytes,
            "tuning_from_cache": s.tuning_from_cache}
