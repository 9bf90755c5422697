// Output assembly, backward scatter and small utility kernels.
#include "cr_internal.h"

namespace cr {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Rows from sorted canonical keys (img | dim | birth pixel | death pixel).  The
// values are read back from the image, so birth == image[birth_pixel] and
// death == image[death_pixel] bit for bit (-0.0 read as +0.0).  Pixel indices
// are indices into the input buffer (the packed buffer of a batch).
__global__ void k_gather(const uint64_t* __restrict__ cand, const unsigned long long* __restrict__ n_ptr,
                         uint64_t cap, const float* __restrict__ img, const ImgDesc* __restrict__ imgs, Layout L,
                         int32_t* __restrict__ dim, float* __restrict__ birth, float* __restrict__ death,
                         int64_t* __restrict__ bpix, int64_t* __restrict__ dpix) {
  uint64_t n = *n_ptr;
  if (n > cap) n = cap;
  const uint64_t pmask = (1ull << L.pb) - 1;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = cand[i];
    const int im = (int)(k >> (2 + 2 * L.pb));
    const ImgDesc d = imgs[im];
    const uint64_t bl = (k >> L.pb) & pmask, dl = k & pmask;
    const int64_t bp = d.pix_off + (int64_t)bl;
    dim[i] = (int32_t)((k >> (2 * L.pb)) & 3);
    bpix[i] = bp;
    birth[i] = canon(img[bp]);
    if (dl == pmask) {
      dpix[i] = -1;
      death[i] = INFINITY;
    } else {
      const int64_t dp = d.pix_off + (int64_t)dl;
      dpix[i] = dp;
      death[i] = canon(img[dp]);
    }
  }
}

// pair_offsets[0..nimg] = exclusive scan of the per-image row counts (one workgroup).
// Also sets the per-image status codes of the C ABI: CR_ERR_NAN_INPUT for an
// image with NaN; otherwise, when the call stopped early (scratch exhausted, an
// iteration cap or a failed check), CR_ERR_OUT_OF_MEMORY or CR_ERR_INTERNAL for
// every image (no image's rows are complete then); otherwise CR_ERR_CAPACITY
// for an image whose rows do not all fit below `capacity`.
__global__ __launch_bounds__(1024) void k_img_offsets(const uint32_t* __restrict__ cnt,
                                                      const uint32_t* __restrict__ img_status,
                                                      const Status* __restrict__ st, int64_t capacity, int nimg,
                                                      int64_t* __restrict__ offsets, int32_t* __restrict__ status) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int per = (nimg + 1023) / 1024;
  const int lo = tid * per, hi = lo + per < nimg ? lo + per : nimg;
  int64_t s = 0;
  for (int i = lo; i < hi; ++i) s += cnt[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t run = part[tid] - s;
  const int32_t stopped = st->abort ? (st->overflow ? 5 /* CR_ERR_OUT_OF_MEMORY */ : 7 /* CR_ERR_INTERNAL */) : 0;
  for (int i = lo; i < hi; ++i) {
    offsets[i] = run;
    run += cnt[i];
    status[i] = img_status[i] ? 2 /* CR_ERR_NAN_INPUT */ : (stopped ? stopped : (run > capacity ? 4 /* CR_ERR_CAPACITY */ : 0));
  }
  if (tid == 1023) offsets[nimg] = part[1023];
}

// grad_image[birth_pixel[i]] += grad_birth[i]; grad_image[death_pixel[i]] += grad_death[i]
// (skipping -1).  birth = image[birth_pixel] and death = image[death_pixel] make
// these the derivatives of the bar end points with respect to the pixels.
__global__ void k_backward(const int64_t* __restrict__ bpix, const int64_t* __restrict__ dpix,
                           const float* __restrict__ gb, const float* __restrict__ gd, int64_t n,
                           float* __restrict__ grad, int64_t n_pixels, uint32_t* __restrict__ bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = bpix[i], e = dpix[i];
    if (b >= 0 && b < n_pixels) {
      if (gb) atomicAdd(&grad[b], gb[i]);
    } else {
      atomicOr(bad, 1u);
    }
    if (e >= 0 && e < n_pixels) {
      if (gd) atomicAdd(&grad[e], gd[i]);
    } else if (e != -1) {
      atomicOr(bad, 1u);
    }
  }
}

// Lifetime-enhanced image channels (Sec. 4): out[k * n_pixels + p] = max over
// the bars of degree k located at pixel p of death - birth.  The location is
// the birth pixel, or the death pixel (essential bars then have none and are
// skipped).  Lifetimes are positive (bars of positive length, +inf for an
// essential bar), so the maximum is taken on their bit patterns, which order
// as unsigned integers; a non-positive or NaN lifetime leaves the pixel alone.
__global__ void k_lifetime(const int32_t* __restrict__ dim, const float* __restrict__ birth,
                           const float* __restrict__ death, const int64_t* __restrict__ loc, int64_t n,
                           float* __restrict__ out, int64_t n_pixels, int skip_missing, uint32_t* __restrict__ bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = dim[i];
    const int64_t p = loc[i];
    if (p == -1 && skip_missing) continue;
    if (k < 0 || k > 2 || p < 0 || p >= n_pixels) {
      atomicOr(bad, 1u);
      continue;
    }
    const float life = death[i] - birth[i];
    if (!(life > 0.0f)) continue;
    atomicMax(reinterpret_cast<unsigned int*>(out) + (k * n_pixels + p), __float_as_uint(life));
  }
}

// (x, y, z) of flat pixel indices (minus base) in an image of extents n[0..2]
// (z, y, x; 1 for absent axes); -1 gives (-1, -1, -1).
__global__ void k_pixel_coords(const int64_t* __restrict__ pixel, int64_t n, int64_t base, int64_t nz,
                               int64_t ny, int64_t nx, int32_t* __restrict__ xyz, uint32_t* __restrict__ bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = pixel[i];
    int32_t x = -1, y = -1, z = -1;
    if (q != -1) {
      const int64_t p = q - base;
      if (p < 0 || p >= nz * ny * nx) {
        atomicOr(bad, 1u);
      } else {
        x = (int32_t)(p % nx);
        y = (int32_t)((p / nx) % ny);
        z = (int32_t)(p / (nx * ny));
      }
    }
    xyz[3 * i] = x;
    xyz[3 * i + 1] = y;
    xyz[3 * i + 2] = z;
  }
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (!n) return;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
}

void launch_gather(int grid, const uint64_t* cand, const unsigned long long* n_ptr, uint64_t cap,
                   const float* img, const ImgDesc* imgs, Layout L, int32_t* dim, float* birth, float* death,
                   int64_t* bpix, int64_t* dpix, hipStream_t s) {
  k_gather<<<grid, 256, 0, s>>>(cand, n_ptr, cap, img, imgs, L, dim, birth, death, bpix, dpix);
}

void launch_img_offsets(const uint32_t* cnt, const uint32_t* img_status, const Status* st, int64_t capacity,
                        int nimg, int64_t* offsets, int32_t* status, hipStream_t s) {
  k_img_offsets<<<1, 1024, 0, s>>>(cnt, img_status, st, capacity, nimg, offsets, status);
}

void launch_backward(const int64_t* bpix, const int64_t* dpix, const float* gb, const float* gd, int64_t n,
                     float* grad, int64_t n_pixels, uint32_t* bad, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_backward<<<(unsigned)blocks, 256, 0, s>>>(bpix, dpix, gb, gd, n, grad, n_pixels, bad);
}

void launch_lifetime(const int32_t* dim, const float* birth, const float* death, const int64_t* loc, int64_t n,
                     float* out, int64_t n_pixels, int skip_missing, uint32_t* bad, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_lifetime<<<(unsigned)blocks, 256, 0, s>>>(dim, birth, death, loc, n, out, n_pixels, skip_missing, bad);
}

void launch_pixel_coords(const int64_t* pixel, int64_t n, int64_t base, const int64_t ext[3], int32_t* xyz,
                         uint32_t* bad, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_pixel_coords<<<(unsigned)blocks, 256, 0, s>>>(pixel, n, base, ext[0], ext[1], ext[2], xyz, bad);
}

}  // namespace cr
