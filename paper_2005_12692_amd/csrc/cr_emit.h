// Output rows of the pairing kernels (shared by the union-find and reduction stages).
#pragma once
#include "cr_internal.h"

namespace cr {

// ---- candidate output rows ---------------------------------------------------
// A bar is written as one 64-bit canonical key img | dim | birth pixel | death
// pixel (local flat indices; all ones = essential).  Birth and death values are
// read back from the image at the end, so nothing else is stored.
struct EmitCtx {
  const float* img;
  const ImgDesc* imgs;
  Layout L;
  uint64_t* cand;
  uint64_t cand_cap;
  unsigned long long* cand_count;
  uint32_t* img_pairs;
  Status* st;
};

__device__ inline uint64_t canon_key(const Layout& L, int img, int dim, uint64_t bl, uint64_t dl) {
  return ((uint64_t)img << (2 + 2 * L.pb)) | ((uint64_t)dim << (2 * L.pb)) | (bl << L.pb) | dl;
}

// The abort flag read once for the whole workgroup, so that a flag raised while
// its threads start cannot send some of them past a barrier the others skip.
__device__ inline bool aborted_block(const Status* st) {
  __shared__ int s_ab;
  if (threadIdx.x == 0) s_ab = aborted(st) ? 1 : 0;
  __syncthreads();
  return s_ab != 0;
}

// Rows of the positions [0, n) of one pairing stage; row(r, &img, &key) tells
// whether position r gives a row.  A workgroup takes tiles of ROW_PER positions
// per thread (ROW_PER * blockDim in all): it decides the rows of a tile in
// registers, reserves their places in the row buffer with one atomic, writes
// them, and adds the tile's per-image row counts with one atomic per image and
// wavefront.  A single counter bumped once per wavefront would serialise every
// wavefront of the GPU on one address.  Positions come in key order, so images
// come in runs and a tile rarely holds more than one.  Every thread of the
// workgroup must call it (it synchronises the workgroup).
constexpr int ROW_PER = 8;
constexpr int ROW_MAX_WAVES = 16;  // workgroups of at most 1024 threads

template <class F>
__device__ inline void emit_tiled(const EmitCtx& E, uint64_t n, F row) {
  __shared__ uint32_t s_wave[ROW_MAX_WAVES];
  __shared__ unsigned long long s_base;
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6, nw = blockDim.x >> 6;
  const uint64_t tile = (uint64_t)ROW_PER * blockDim.x;
  const Walk w = xcd_part((n + tile - 1) / tile, 1);
  for (uint64_t t = w.i; t < w.end; t += w.stride) {
    uint64_t ck[ROW_PER];
    int im[ROW_PER];
    uint32_t act = 0;
#pragma unroll
    for (int k = 0; k < ROW_PER; ++k) {
      const uint64_t r = t * tile + (uint64_t)k * blockDim.x + tid;
      ck[k] = 0;
      im[k] = 0;
      if (r < n && row(r, &im[k], &ck[k])) act |= 1u << k;
    }
    // places: wavefront scan of the per-thread counts, then the workgroup's
    const uint32_t cnt = __popc(act);
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t up = __shfl_up(incl, o, 64);
      if (lane >= o) incl += up;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    if (tid == 0) {
      uint32_t tot = 0;
      for (int v = 0; v < nw; ++v) tot += s_wave[v];
      s_base = tot ? atomicAdd(E.cand_count, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    uint64_t pos = s_base + incl - cnt;
    for (int v = 0; v < wv; ++v) pos += s_wave[v];
    __syncthreads();  // s_wave and s_base are rewritten by the next tile
    uint32_t stored = 0;
#pragma unroll
    for (int k = 0; k < ROW_PER; ++k)
      if (act >> k & 1u) {
        if (pos < E.cand_cap) {
          E.cand[pos] = ck[k];
          stored |= 1u << k;
        } else {
          raise_flag(E.st, &E.st->overflow, OVF_ROWS);
        }
        ++pos;
      }
    // per-image counts: the lowest image among the lanes' uncounted rows first
    while (__ballot(stored != 0)) {
      int mine = 0x7FFFFFFF;
#pragma unroll
      for (int k = ROW_PER - 1; k >= 0; --k)
        if (stored >> k & 1u) mine = min(mine, im[k]);
      int lo = mine;
#pragma unroll
      for (int o = 32; o; o >>= 1) lo = min(lo, __shfl_xor(lo, o, 64));
      uint32_t c = 0;
#pragma unroll
      for (int k = 0; k < ROW_PER; ++k)
        if ((stored >> k & 1u) && im[k] == lo) {
          ++c;
          stored &= ~(1u << k);
        }
#pragma unroll
      for (int o = 32; o; o >>= 1) c += __shfl_xor(c, o, 64);
      if (lane == 0) atomicAdd(&E.img_pairs[lo], c);
    }
  }
}

// Row for the pair (birth cell, death cell) given by their sort keys; returns
// false (no row) for a pair of length zero.
__device__ inline bool pair_row(const EmitCtx& E, uint64_t bkey, uint64_t dkey, bool essential,
                                int* img_out, uint64_t* ckey) {
  const Layout& L = E.L;
  const int im = skey_img(L, bkey);
  if (!essential && !(skey_ord(L, bkey) < skey_ord(L, dkey))) return false;  // zero length
  const ImgDesc d = E.imgs[im];
  int c[3];
  kidx_coords(d, skey_kidx(L, bkey), c);
  const int dim = (c[0] & 1) + (c[1] & 1) + (c[2] & 1);
  const uint64_t bl = (uint64_t)(cell_argmax_pixel(E.img, d, c) - d.pix_off);
  uint64_t dl = (1ull << L.pb) - 1;
  if (!essential) {
    kidx_coords(d, skey_kidx(L, dkey), c);
    dl = (uint64_t)(cell_argmax_pixel(E.img, d, c) - d.pix_off);
  }
  *img_out = im;
  *ckey = canon_key(L, im, dim, bl, dl);
  return true;
}

}  // namespace cr
