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

// Adds one to cnt[key] for every active lane with one atomic per distinct key
// in the wavefront; every lane of the wavefront must call it.
__device__ inline void wave_count(uint32_t* cnt, bool active, int key) {
  uint64_t mask = __ballot(active);
  while (mask) {
    const int leader = __ffsll((unsigned long long)mask) - 1;
    const int lk = __shfl(key, leader, 64);
    const uint64_t peers = __ballot(active && key == lk);
    if (__lane_id() == leader) atomicAdd(&cnt[lk], (uint32_t)__popcll(peers));
    mask &= ~peers;
  }
}

// Appends one row per active lane; every lane of the wavefront must call it.
__device__ inline void emit_rows(const EmitCtx& E, bool active, int img, uint64_t ckey) {
  const uint64_t mask = __ballot(active);
  if (!mask) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(E.cand_count, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader, 64);
  bool stored = false;
  if (active) {
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const unsigned long long pos = base + __popcll(mask & lt);
    if (pos < E.cand_cap) {
      E.cand[pos] = ckey;
      stored = true;
    } else {
      raise_flag(E.st, &E.st->overflow, OVF_ROWS);
    }
  }
  wave_count(E.img_pairs, stored, img);
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
