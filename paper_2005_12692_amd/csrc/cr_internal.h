// Internal definitions shared by the HIP kernels and the host layer of libcr.
//
// Cells of the V-construction cubical complex (Kaji-Sudo-Ahara, Sec. 2) are
// addressed by Khalimsky coordinates k = (kz, ky, kx), 0 <= k_a < K_a = 2 n_a - 1:
// an odd coordinate means the cell extends along that axis, so dim = number of
// odd coordinates.  Its value is the maximum of its vertex pixels (the
// V-construction).  A 2D image is a volume of z extent 1.
//
// Total order of cells (a refinement of the filtration): (value, dim, kidx)
// with kidx = (kz*Ky + ky)*Kx + kx.  Within one dimension this is (value, kidx).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cr {

constexpr uint32_t TRIP_INF = 0xFFFFFFFFu;  // "never merged" level of a triplet

struct ImgDesc {
  int32_t n[3];     // pixel extents z, y, x (n[0] = 1 for a 2D image)
  int32_t K[3];     // Khalimsky extents 2n-1
  int64_t pix_off;  // index of the image's first pixel in the (packed) input
};

// Bit layout of the keys of one call (most significant field first).
//  sort key of a surviving cell:  dim(2) | img(ib) | ord32(value)(32) | kidx(kb)
//  canonical key of an output bar: img(ib) | dim(2) | birth pixel(pb) | death pixel(pb)
struct Layout {
  int kb;  // bits of kidx
  int ib;  // bits of the image index
  int pb;  // bits of a local pixel field (all ones = "no death pixel")
  int nimg;
  int ndim;
};

// Device-side status words (all zero on success).
struct Status {
  uint32_t nan_input;      // some input pixel was NaN
  uint32_t overflow;       // a capacity was exceeded: OVF_* bits
  uint32_t internal;       // an invariant of the algorithm failed (bug guard)
  uint32_t iter_cap;       // a bounded loop hit its iteration cap
  uint32_t abort;          // set together with any of the above: stop early
  uint32_t tail_round;     // degree-1 reduction: 1 + the round whose columns went to the
                           // asynchronous tail (0: none yet)
  unsigned long long adds; // column additions performed by the reduction
  unsigned long long merged;  // list entries read by those additions
};
enum : uint32_t { OVF_SURVIVORS = 1, OVF_ARENA = 2, OVF_ROWS = 4, OVF_COLUMN = 8 };

__host__ __device__ inline uint32_t ord32_bits(uint32_t u) {
  return (u >> 31) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline uint32_t unord32(uint32_t o) {
  return (o >> 31) ? (o & 0x7FFFFFFFu) : ~o;
}

__device__ inline float canon(float v) {
  // -0.0 -> +0.0; NaN is reported by the loader and replaced by +inf
  return v == 0.0f ? 0.0f : v;
}

__device__ inline uint64_t make_skey(const Layout& L, int dim, int img, uint32_t ordv, uint32_t kidx) {
  return ((uint64_t)dim << (L.ib + 32 + L.kb)) | ((uint64_t)img << (32 + L.kb)) |
         ((uint64_t)ordv << L.kb) | (uint64_t)kidx;
}
__device__ inline uint32_t skey_kidx(const Layout& L, uint64_t k) {
  return (uint32_t)(k & ((1ull << L.kb) - 1));
}
__device__ inline uint32_t skey_ord(const Layout& L, uint64_t k) { return (uint32_t)(k >> L.kb); }
__device__ inline int skey_img(const Layout& L, uint64_t k) {
  return L.ib ? (int)((k >> (32 + L.kb)) & ((1ull << L.ib) - 1)) : 0;
}

__device__ inline void kidx_coords(const ImgDesc& d, uint32_t kidx, int c[3]) {
  c[2] = (int)(kidx % (uint32_t)d.K[2]);
  uint32_t t = kidx / (uint32_t)d.K[2];
  c[1] = (int)(t % (uint32_t)d.K[1]);
  c[0] = (int)(t / (uint32_t)d.K[1]);
}
__device__ inline uint32_t coords_kidx(const ImgDesc& d, const int c[3]) {
  return ((uint32_t)c[0] * (uint32_t)d.K[1] + (uint32_t)c[1]) * (uint32_t)d.K[2] + (uint32_t)c[2];
}
__device__ inline int64_t pixel_index(const ImgDesc& d, int z, int y, int x) {
  return d.pix_off + ((int64_t)z * d.n[1] + y) * d.n[2] + x;
}
// global index of the minimal vertex of a cell (anchor of top cells and squares)
__device__ inline int64_t anchor_pixel(const ImgDesc& d, const int c[3]) {
  return pixel_index(d, c[0] >> 1, c[1] >> 1, c[2] >> 1);
}

// Value of a cell from the global image: max over its vertices.
__device__ inline float cell_value(const float* __restrict__ img, const ImgDesc& d, const int c[3]) {
  float v = -INFINITY;
  const int z0 = c[0] >> 1, y0 = c[1] >> 1, x0 = c[2] >> 1;
  const int nz = 1 + (c[0] & 1), ny = 1 + (c[1] & 1), nx = 1 + (c[2] & 1);
  for (int dz = 0; dz < nz; ++dz)
    for (int dy = 0; dy < ny; ++dy)
      for (int dx = 0; dx < nx; ++dx) {
        float p = img[pixel_index(d, z0 + dz, y0 + dy, x0 + dx)];
        p = (p != p) ? INFINITY : canon(p);
        v = fmaxf(v, p);
      }
  return v;
}

// The vertex whose value the cell takes: max value, ties to the larger flat index.
__device__ inline int64_t cell_argmax_pixel(const float* __restrict__ img, const ImgDesc& d,
                                            const int c[3]) {
  float bv = -INFINITY;
  int64_t best = -1;
  const int z0 = c[0] >> 1, y0 = c[1] >> 1, x0 = c[2] >> 1;
  const int nz = 1 + (c[0] & 1), ny = 1 + (c[1] & 1), nx = 1 + (c[2] & 1);
  for (int dz = 0; dz < nz; ++dz)
    for (int dy = 0; dy < ny; ++dy)
      for (int dx = 0; dx < nx; ++dx) {
        int64_t p = pixel_index(d, z0 + dz, y0 + dy, x0 + dx);
        float v = img[p];
        v = (v != v) ? INFINITY : canon(v);
        if (best < 0 || v > bv || (v == bv && p > best)) {
          bv = v;
          best = p;
        }
      }
  return best;
}

// ---- XCD-aware walks over a range -----------------------------------------------
// Workgroups are dispatched to the eight XCDs in turn, so workgroup b runs on
// XCD b % 8.  A range [0, n) is cut into one contiguous part per XCD (a multiple
// of `align` long) and each part is walked by that XCD's workgroups alone: the
// images an XCD works on at a time then share its L2 instead of being spread
// over all eight.  Any grid is correct; one that is not a multiple of 8 walks
// [0, n) as a single part.
struct Walk {
  uint64_t i, end, stride;
};
// Units (e.g. tiles) of the range per workgroup: i, i + stride, ... below end.
__device__ inline Walk xcd_part(uint64_t n, uint64_t align) {
  const uint32_t nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const uint32_t x = blockIdx.x % nx, b = blockIdx.x / nx;
  const uint64_t part = ((n + nx - 1) / nx + align - 1) / align * align;
  const uint64_t lo = min(n, (uint64_t)x * part), hi = min(n, lo + part);
  return {lo + b, hi, (uint64_t)(gridDim.x / nx)};
}
// Positions per thread.  chunks == 0: the whole grid strides over [0, n), so
// the positions in flight are consecutive.  Otherwise each XCD's part is cut
// into `chunks` contiguous chunks (at most one per wavefront of the XCD), each
// walked in order by its own whole wavefronts.  For the union-find merges the
// positions in flight in one image then sit at nearby levels, so fewer links
// are made out of order and later replaced.
__device__ inline Walk chunk_walk(uint64_t n, uint32_t chunks) {
  if (chunks == 0) return {blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, n, (uint64_t)gridDim.x * blockDim.x};
  const uint32_t nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const uint32_t x = blockIdx.x % nx, b = blockIdx.x / nx, nb = gridDim.x / nx;
  const uint64_t part = (n + nx - 1) / nx;
  const uint64_t lo = min(n, (uint64_t)x * part), hi = min(n, lo + part);
  const uint64_t waves = (uint64_t)nb * (blockDim.x >> 6);
  const uint64_t nc = min(waves, (uint64_t)chunks * (8 / nx));
  const uint64_t tg = (waves / nc) * 64;  // threads per chunk, whole wavefronts
  const uint64_t tx = (uint64_t)b * blockDim.x + threadIdx.x, g = tx / tg;
  if (g >= nc) return {0, 0, 1};
  const uint64_t cs = (hi - lo + nc - 1) / nc;
  const uint64_t clo = min(hi, lo + g * cs), chi = min(hi, clo + cs);
  return {clo + tx % tg, chi, tg};
}

// ---- device-scope atomics (coherent across the XCDs of one GPU) ----------------
__device__ inline uint64_t ld_acq64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_rlx64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int32_t ld_acq32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_rel64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool cas64(uint64_t* p, uint64_t expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool cas32_rel(int32_t* p, int32_t expected, int32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELEASE,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void raise_flag(Status* st, uint32_t* word, uint32_t bits = 1u) {
  atomicOr(word, bits);
  atomicOr(&st->abort, 1u);
}
__device__ inline bool aborted(const Status* st) {
  return __hip_atomic_load(&st->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

}  // namespace cr
