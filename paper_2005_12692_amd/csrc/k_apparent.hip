// Fused stencil pass: filtration values, apparent pairs, survivor compaction.
//
// Every cell of the V-construction complex (Sec. 2) is anchored at the pixel
// of its smallest coordinates and takes the maximum of its vertices.  A cell
// pair (s, t) is apparent iff t is the earliest cofacet of s and s is the
// latest facet of t in the total order (value, dim, kidx).  Such a pair has
// length zero (value(t) is the maximum over its facets, attained by s), so it
// emits nothing and both cells leave the problem; the remaining cells
// ("survivors") are compacted into one key array.
//
// Layout: a workgroup is RW wavefronts; wavefront w owns image row y0-1+w and
// lane l owns column x0-1+l, so the rows and lanes at the edge of the
// workgroup are a one-pixel halo and the interior is (RW-2) x 62 pixels.  In
// 3D the workgroup marches along z over ZC planes.  Per pixel and plane a
// thread keeps the record of the 8 cells anchored there (their values as
// order-preserving 32-bit keys; a cell that leaves the image has none), and
// computes for each cell the direction of its earliest cofacet and of its
// latest facet (3-bit codes: 0 -z, 1 -y, 2 -x, 3 +x, 4 +y, 5 +z, i.e. ascending
// kidx of the neighbour; 7 none).  Neighbouring records and codes come from the
// lane next door (DPP), the wavefront above or below (LDS) and the previous or
// next plane (registers).  A cell is paired iff the code of its partner points
// back at it.
//
// Two forests are written alongside:
//  * vlink[pixel]: a vertex v paired with edge e links to the other endpoint
//    of e (older than v); surviving vertices get -1 (filled in after the sort).
//    Union-find over surviving edges can start from these links: e is v's
//    earliest coface, so no surviving edge touches v before v joins its parent.
//  * tlink[anchor]: a top cell t paired with facet s links to the other
//    cofacet of s (older in the reversed order), or to the image's exterior
//    node when s lies on the boundary.  This is the same forest for the dual
//    union-find of the top dimension.
// and, for the degree-1 reduction of a volume, eapp[4 * pixel + axis] of every
// edge (axis 0 z, 1 y, 2 x; one 32-bit store per pixel): 2 * axis + (direction
// > 0) of its apparent partner square, 0xFF if none.
#include "cr_internal.h"

#include <cstdlib>

namespace cr {

constexpr uint32_t NONE = 0xFFFFFFFFu;  // key of a cell outside the image (above every value key)
constexpr uint32_t NO_CODES = 0xFFFFFFu; // eight "none" codes

// axis of direction d (0 z, 1 y, 2 x) and the bit of an axis in a cell type
// t = 4 tz + 2 ty + tx
__host__ __device__ constexpr int dir_axis(int d) { return d < 3 ? d : 5 - d; }
__host__ __device__ constexpr int abit(int a) { return 4 >> a; }
__host__ __device__ constexpr int popc3(int t) { return (t & 1) + ((t >> 1) & 1) + ((t >> 2) & 1); }

struct Rec {
  uint32_t v[8];  // keys of the 8 cells anchored at one pixel, by type
};

__device__ __forceinline__ uint32_t lane_down1(uint32_t v) {  // lane i gets lane i+1 (lane 63 keeps its own)
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_up1(uint32_t v) {  // lane i gets lane i-1 (lane 0 keeps its own)
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x138, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t pix_key(float v, bool* nan) {
  if (v != v) {
    *nan = true;
    v = INFINITY;
  }
  v = canon(v);
  uint32_t b;
  __builtin_memcpy(&b, &v, 4);
  return ord32_bits(b);
}

// Values derived from one pixel plane: the vertex, the x- and y-edges and the
// xy-square anchored at the pixel.
struct Planar {
  uint32_t v, ex, ey, sxy;
};
__device__ __forceinline__ Planar planar(uint32_t f, uint32_t fx, uint32_t fy, uint32_t fxy) {
  Planar p;
  p.v = f;
  p.ex = max(f, fx);
  p.ey = max(f, fy);
  p.sxy = max(p.ex, max(fy, fxy));
  return p;
}
__device__ __forceinline__ Rec record(const Planar& a, const Planar& b) {  // a: plane z, b: plane z+1
  Rec r;
  r.v[0] = a.v;
  r.v[1] = a.ex;
  r.v[2] = a.ey;
  r.v[3] = a.sxy;
  r.v[4] = max(a.v, b.v);
  r.v[5] = max(a.ex, b.ex);
  r.v[6] = max(a.ey, b.ey);
  r.v[7] = max(a.sxy, b.sxy);
  return r;
}

// Earliest cofacet of the cell of type T: the first direction (ascending
// kidx) of smallest value; m[a] is the record of the pixel one step down axis a.
template <int T>
__device__ __forceinline__ uint32_t ecf_code(const Rec& own, const Rec& mz, const Rec& my, const Rec& mx) {
  uint32_t best = NONE, code = 7;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int a = dir_axis(d);
    if (T & abit(a)) continue;
    const int u = T | abit(a);
    const uint32_t v = d >= 3 ? own.v[u] : (a == 0 ? mz.v[u] : (a == 1 ? my.v[u] : mx.v[u]));
    if (v < best) {
      best = v;
      code = (uint32_t)d;
    }
  }
  return code;
}

// Latest facet of the cell of type U: the last direction (ascending kidx) of
// largest value; p[a] is the record of the pixel one step up axis a.
template <int U>
__device__ __forceinline__ uint32_t lf_code(const Rec& own, const Rec& pz, const Rec& py, const Rec& px) {
  uint32_t best = 0, code = 7;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int a = dir_axis(d);
    if (!(U & abit(a))) continue;
    const int u = U ^ abit(a);
    const uint32_t v = d < 3 ? own.v[u] : (a == 0 ? pz.v[u] : (a == 1 ? py.v[u] : px.v[u]));
    if (v >= best) {
      best = v;
      code = (uint32_t)d;
    }
  }
  return code;
}

template <int T = 0>
__device__ __forceinline__ void codes_all(const Rec& own, const Rec& mz, const Rec& my, const Rec& mx,
                                          const Rec& pz, const Rec& py, const Rec& px, uint32_t* E, uint32_t* F) {
  if constexpr (T < 8) {
    *E |= (T == 7 ? 7u : ecf_code<T>(own, mz, my, mx)) << (3 * T);
    *F |= (T == 0 ? 7u : lf_code<T>(own, pz, py, px)) << (3 * T);
    codes_all<T + 1>(own, mz, my, mx, pz, py, px, E, F);
  }
}

__device__ __forceinline__ uint32_t code_of(uint32_t word, int t) { return (word >> (3 * t)) & 7u; }

// Bit 3 t set iff field t (3 bits) of the code word w equals c (c < 7; a
// missing code is 7 and never matches).
__device__ __forceinline__ uint32_t eq_code(uint32_t w, uint32_t c) {
  const uint32_t v = w ^ (c * 0x249249u);
  return ~(v | (v >> 1) | (v >> 2)) & 0x249249u;
}

template <int RW>
struct StencilLds {
  uint4 recA[RW][64];  // record fields 0, 1, 4, 5 (read by the row above: cells without a y extent)
  uint4 recB[RW][64];  // record fields 2, 3, 6, 7 (read by the row below)
  uint2 cw[2][RW][64]; // (earliest-cofacet codes, latest-facet codes), by plane parity
  uint32_t wcnt[RW];
  uint32_t woff[RW];
  unsigned long long wbase;
  unsigned long long sbase[2];  // 3D: array offsets reserved for the two staging buffers
};

// 3D: survivor keys of a plane are staged in LDS (dynamic, two buffers of
// stage_keys<RW>() keys) and written out one plane later.
template <int RW>
constexpr uint32_t stage_keys() { return 256u * RW; }

// Inclusive prefix sum over lanes 0..15 (each row of 16 lanes on its own).
__device__ __forceinline__ uint32_t row_scan16(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  return x;
}

// ROW1 (images of one row, as 1D signals run): wavefront w takes pixels
// x0 - 1 + 62 w .. of that row instead of row y0 - 1 + w, and every neighbour
// across y is outside the image.
template <int NDIM, int RW, int ZC, bool ROW1 = false>
__global__ __launch_bounds__(64 * RW) void k_stencil(
    const float* __restrict__ img, const ImgDesc* __restrict__ imgs, const int4* __restrict__ tiles,
    Layout L, uint64_t* __restrict__ surv, uint64_t surv_cap,
    unsigned long long* __restrict__ surv_count, int32_t* __restrict__ vlink, int32_t* __restrict__ tlink,
    uint8_t* __restrict__ eapp, uint32_t* __restrict__ img_status, Status* __restrict__ st, uint32_t stage_cap) {
  __shared__ StencilLds<RW> S;
  extern __shared__ uint64_t stg[];  // 3D: 2 x stage_keys<RW>() staged survivor keys
  constexpr int TOP = NDIM == 3 ? 7 : 3;  // type of the top cell
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int4 tile = tiles[blockIdx.x];
  const int im = tile.x;
  const ImgDesc d = imgs[im];
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const int z0 = tile.y, y0 = tile.z, x0 = tile.w;
  const int x = x0 - 1 + lane + (ROW1 ? 62 * row : 0), y = ROW1 ? y0 : y0 - 1 + row;
  const bool xin = x >= 0 && x < n2, x1in = x + 1 >= 0 && x + 1 < n2;
  const bool yin = y >= 0 && y < n1, y1in = y + 1 >= 0 && y + 1 < n1;
  const bool inner = lane >= 1 && lane <= 62 && (ROW1 || (row >= 1 && row <= RW - 2)) && xin && yin;
  const uint32_t K1 = (uint32_t)d.K[1], K2 = (uint32_t)d.K[2];
  const int64_t rowpix = (int64_t)n1 * n2;
  bool nan = false;

  // pixel keys of plane zz at (x, y), (x, y+1) and their right neighbours
  auto load_plane = [&](int zz, uint32_t* f, uint32_t* fy) {
    const bool zin = zz >= 0 && zz < n0;
    const int64_t base = d.pix_off + (int64_t)zz * rowpix + (int64_t)y * n2 + x;
    *f = (zin && xin && yin) ? pix_key(img[base], &nan) : NONE;
    *fy = (zin && xin && y1in) ? pix_key(img[base + n2], &nan) : NONE;
  };
  auto planar_of = [&](int zz, uint32_t f, uint32_t fy) {
    uint32_t fx = lane_down1(f), fxy = lane_down1(fy);
    if (lane == 63) {  // the right neighbour lies beyond the wavefront
      const bool zin = zz >= 0 && zz < n0;
      const int64_t base = d.pix_off + (int64_t)zz * rowpix + (int64_t)y * n2 + x + 1;
      fx = (zin && x1in && yin) ? pix_key(img[base], &nan) : NONE;
      fxy = (zin && x1in && y1in) ? pix_key(img[base + n2], &nan) : NONE;
    }
    return planar(f, fx, fy, fxy);
  };

  // Exchanges the record of plane kk with the rows above and below; returns
  // the earliest-cofacet and latest-facet codes of the cells at plane kk.
  auto codes_of_plane = [&](const Rec& R0, const Rec& Rm, const Rec& Rp, uint32_t* E, uint32_t* F) {
    S.recA[row][lane] = make_uint4(R0.v[0], R0.v[1], R0.v[4], R0.v[5]);
    S.recB[row][lane] = make_uint4(R0.v[2], R0.v[3], R0.v[6], R0.v[7]);
    __syncthreads();
    Rec ym, yp, xm, xp;
    const uint4 b = !ROW1 && row > 0 ? S.recB[row - 1][lane] : make_uint4(NONE, NONE, NONE, NONE);
    const uint4 a = !ROW1 && row < RW - 1 ? S.recA[row + 1][lane] : make_uint4(NONE, NONE, NONE, NONE);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      ym.v[t] = NONE;
      yp.v[t] = NONE;
      xm.v[t] = lane_up1(R0.v[t]);
      xp.v[t] = lane_down1(R0.v[t]);
    }
    ym.v[2] = b.x; ym.v[3] = b.y; ym.v[6] = b.z; ym.v[7] = b.w;
    yp.v[0] = a.x; yp.v[1] = a.y; yp.v[4] = a.z; yp.v[5] = a.w;
    *E = 0;
    *F = 0;
    codes_all(R0, Rm, ym, xm, Rp, yp, xp, E, F);
  };

  // Classifies the cells anchored at (plane zc, y, x) from the codes of this
  // pixel (E0, F0), of the pixels one step down each axis (latest-facet words
  // Fm*) and one step up (earliest-cofacet words Ep*).  Every type at once: a
  // code word holds eight 3-bit fields, and eq_code marks the fields equal to
  // a direction with bit 3 t, so a pairing condition is a shift and an AND of
  // such marks (the field of type t | A sits 3 A bits above that of t).
  // Writes the links and the edges' partner codes; returns the survivor mask,
  // bit 3 t for type t.
  auto classify = [&](int zc, const Rec& R, uint32_t E0, uint32_t F0, uint32_t Fmz, uint32_t Fmy, uint32_t Fmx,
                      uint32_t Epz, uint32_t Epy, uint32_t Epx) -> uint32_t {
    const int32_t pix = (int32_t)(d.pix_off + (int64_t)zc * rowpix + (int64_t)y * n2 + x);
    const int32_t st_z = (int32_t)rowpix, st_y = n2;
    // earliest cofacet of (p, t) in direction d: eE[d]; latest facet of (p, u): eF[d]
    const uint32_t eE0 = eq_code(E0, 0), eE1 = eq_code(E0, 1), eE2 = eq_code(E0, 2);
    const uint32_t eE3 = eq_code(E0, 3), eE4 = eq_code(E0, 4), eE5 = eq_code(E0, 5);
    const uint32_t eF0 = eq_code(F0, 0), eF1 = eq_code(F0, 1), eF2 = eq_code(F0, 2);
    const uint32_t eF3 = eq_code(F0, 3), eF4 = eq_code(F0, 4), eF5 = eq_code(F0, 5);
    // (p, t) with its earliest cofacet t | A above it (+a: same anchor, whose
    // latest facet must be -a) or below it (-a: anchor p - e_a, whose latest
    // facet must be +a)
    const uint32_t pf = (eE5 & (eF0 >> 12)) | (eE0 & (eq_code(Fmz, 5) >> 12)) |  // z
                        (eE4 & (eF1 >> 6)) | (eE1 & (eq_code(Fmy, 4) >> 6)) |    // y
                        (eE3 & (eF2 >> 3)) | (eE2 & (eq_code(Fmx, 3) >> 3));     // x
    // (p, u) with its latest facet u - B below it (-b: same anchor, whose
    // earliest cofacet must be +b) or above it (+b: anchor p + e_b, whose
    // earliest cofacet must be -b)
    const uint32_t pc = (eF0 & (eE5 << 12)) | (eF5 & (eq_code(Epz, 0) << 12)) |  // z
                        (eF1 & (eE4 << 6)) | (eF4 & (eq_code(Epy, 1) << 6)) |    // y
                        (eF2 & (eE3 << 3)) | (eF3 & (eq_code(Epx, 2) << 3));     // x
    uint32_t exists = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) exists |= R.v[t] != NONE ? (1u << (3 * t)) : 0u;
    // axis of a direction code (0 z, 1 y, 2 x), read from a table so that it
    // compiles to selects rather than branches
    auto axis_of = [](uint32_t c) { return (0x012210u >> (4 * c)) & 3u; };
    // vertex: link to the other end of its edge
    {
      const uint32_t e = E0 & 7u, a = axis_of(e);
      const int32_t step = a == 0 ? st_z : (a == 1 ? st_y : 1);
      const int32_t to = e >= 3 ? pix + step : pix - step;
      vlink[pix] = (pf & 1u) ? to : -1;
    }
    // top cell: link to the other cofacet of its latest facet, or the exterior
    {
      const uint32_t f = (F0 >> (3 * TOP)) & 7u, b = axis_of(f);
      const int32_t step = b == 0 ? st_z : (b == 1 ? st_y : 1);
      const int pb = b == 0 ? zc : (b == 1 ? y : x);
      const int nb = b == 0 ? n0 : (b == 1 ? n1 : n2);
      const bool ext = f < 3 ? pb < 1 : pb + 2 >= nb;
      const int32_t to = ext ? -(im + 2) : (f < 3 ? pix - step : pix + step);
      const int32_t link = ((pc >> (3 * TOP)) & 1u) ? to : -1;
      if (R.v[TOP] != NONE) tlink[pix] = link;
    }
    // the partner squares of the three edges (byte axis: 0 z, 1 y, 2 x) as
    // 2 * axis + (direction > 0), 0xFF if none: one word per pixel
    if (NDIM == 3 && eapp) {
      // direction code d -> 2 * axis + (d >= 3): 0, 2, 4, 5, 3, 1
      auto part = [&](int t) -> uint32_t {
        const uint32_t e = (E0 >> (3 * t)) & 7u;
        return ((pf >> (3 * t)) & 1u) ? ((0x135420u >> (4 * e)) & 15u) : 0xFFu;
      };
      reinterpret_cast<uint32_t*>(eapp)[pix] = part(4) | (part(2) << 8) | (part(1) << 16) | 0xFF000000u;
    }
    return exists & ~(pf | pc);
  };

  // Appends the survivors of this step (mask bit 3 t for type t) with one
  // atomic per workgroup.
  auto flush = [&](int zc, const Rec& R, uint32_t mask) {
    const uint32_t cnt = (uint32_t)__popc(mask);
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
      const uint64_t bm = __ballot((cnt >> bit) & 1u);
      pre += __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u)) << bit;
      tot += (uint32_t)__popcll(bm) << bit;
    }
    if (lane == 0) S.wcnt[row] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t run = 0;
      for (int w = 0; w < RW; ++w) {
        S.woff[w] = run;
        run += S.wcnt[w];
      }
      const unsigned long long base = run ? atomicAdd(surv_count, (unsigned long long)run) : 0ull;
      if (base + run > surv_cap) raise_flag(st, &st->overflow, OVF_SURVIVORS);  // what fits is kept
      S.wbase = base;
    }
    __syncthreads();
    if (!mask) return;
    unsigned long long pos = S.wbase + S.woff[row] + pre;
    const unsigned long long lim = surv_cap;
    const uint32_t kbase = ((uint32_t)(2 * zc) * K1 + (uint32_t)(2 * y)) * K2 + (uint32_t)(2 * x);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if ((mask >> (3 * t)) & 1u) {
        const uint32_t kidx = kbase + ((t & 4) ? K1 * K2 : 0u) + ((t & 2) ? K2 : 0u) + (uint32_t)(t & 1);
        if (pos < lim) surv[pos] = make_skey(L, popc3(t), im, R.v[t], kidx);
        ++pos;
      }
    }
  };

  // 3D form of flush: the survivors of a plane go to an LDS staging buffer,
  // and thread 0 issues the workgroup's reservation without waiting for it;
  // the next call (or drain) copies them out, coalesced, once the reservation
  // has returned.  So no wavefront waits on the atomic's round trip, where
  // flush holds the whole workgroup at a barrier for it on every plane.  A
  // plane with more survivors than a buffer holds is written as in flush.
  constexpr uint32_t STG = stage_keys<RW>();  // stage_cap <= STG keys are staged
  unsigned long long res = 0;  // thread 0: the reservation of the staged plane
  uint32_t prev = 0;           // keys staged by the previous call (0: none)
  uint32_t pb = 0;             // staging buffer of this call
  auto copy_out = [&](uint32_t b) {  // after a barrier that follows the write of S.sbase[b]
    const unsigned long long base = S.sbase[b];
    const uint64_t* src = stg + (size_t)b * STG;
    for (uint32_t i = threadIdx.x; i < prev; i += 64 * RW)
      if (base + i < surv_cap) surv[base + i] = src[i];
  };
  auto publish = [&]() {  // thread 0, before a barrier: the previous call's reservation
    if (threadIdx.x == 0 && prev) {
      S.sbase[pb ^ 1u] = res;
      if (res + prev > surv_cap) raise_flag(st, &st->overflow, OVF_SURVIVORS);  // what fits is kept
    }
  };
  auto flush_staged = [&](int zc, const Rec& R, uint32_t mask) {
    const uint32_t cnt = (uint32_t)__popc(mask);
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
      const uint64_t bm = __ballot((cnt >> bit) & 1u);
      pre += __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u)) << bit;
      tot += (uint32_t)__popcll(bm) << bit;
    }
    if (lane == 0) S.wcnt[row] = tot;
    publish();
    __syncthreads();
    if (prev) copy_out(pb ^ 1u);
    // the wavefronts' offsets within the plane and its total, by every wavefront
    static_assert(RW <= 16, "one DPP row holds the wavefront counts");
    const uint32_t incl = row_scan16(lane < RW ? S.wcnt[lane] : 0u);
    const uint32_t run = (uint32_t)__builtin_amdgcn_readlane((int)incl, RW - 1);
    const uint32_t woff = row ? (uint32_t)__builtin_amdgcn_readlane((int)incl, row - 1) : 0u;
    const uint32_t kbase = ((uint32_t)(2 * zc) * K1 + (uint32_t)(2 * y)) * K2 + (uint32_t)(2 * x);
    if (run > stage_cap) {  // too many to stage: reserve now and write them straight out
      if (threadIdx.x == 0) {
        const unsigned long long base = atomicAdd(surv_count, (unsigned long long)run);
        if (base + run > surv_cap) raise_flag(st, &st->overflow, OVF_SURVIVORS);
        S.wbase = base;
      }
      __syncthreads();
      unsigned long long pos = S.wbase + woff + pre;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if ((mask >> (3 * t)) & 1u) {
          const uint32_t kidx = kbase + ((t & 4) ? K1 * K2 : 0u) + ((t & 2) ? K2 : 0u) + (uint32_t)(t & 1);
          if (pos < surv_cap) surv[pos] = make_skey(L, popc3(t), im, R.v[t], kidx);
          ++pos;
        }
      }
      prev = 0;
      return;
    }
    if (threadIdx.x == 0 && run) res = atomicAdd(surv_count, (unsigned long long)run);  // read by the next call
    uint64_t* dst = stg + (size_t)pb * STG + woff + pre;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if ((mask >> (3 * t)) & 1u) {
        const uint32_t kidx = kbase + ((t & 4) ? K1 * K2 : 0u) + ((t & 2) ? K2 : 0u) + (uint32_t)(t & 1);
        *dst++ = make_skey(L, popc3(t), im, R.v[t], kidx);
      }
    }
    prev = run;
    pb ^= 1u;
  };
  auto drain = [&]() {  // the last staged plane
    publish();
    __syncthreads();
    if (prev) copy_out(pb ^ 1u);
  };

  if constexpr (NDIM == 2) {
    uint32_t f, fy;
    load_plane(0, &f, &fy);
    const Planar p0 = planar_of(0, f, fy);
    const Planar none = {NONE, NONE, NONE, NONE};
    const Rec R0 = record(p0, none);
    Rec Rn;
#pragma unroll
    for (int t = 0; t < 8; ++t) Rn.v[t] = NONE;
    uint32_t E, F;
    codes_of_plane(R0, Rn, Rn, &E, &F);
    S.cw[0][row][lane] = make_uint2(E, F);
    __syncthreads();
    const uint32_t Fmy = !ROW1 && row > 0 ? S.cw[0][row - 1][lane].y : NO_CODES;
    const uint32_t Epy = !ROW1 && row < RW - 1 ? S.cw[0][row + 1][lane].x : NO_CODES;
    const uint32_t Fmx = lane_up1(F), Epx = lane_down1(E);
    uint32_t mask = 0;
    if (inner) mask = classify(0, R0, E, F, NO_CODES, Fmy, Fmx, NO_CODES, Epy, Epx);
    flush(0, R0, mask);
  } else {
    const int zend = z0 + ZC < n0 ? z0 + ZC : n0;
    // rolling state: planar values of plane kk+1, records of planes kk-1..kk+1,
    // codes of planes kk-2 (latest-facet word) and kk-1, and the prefetched plane
    uint32_t f, fy, nf, nfy;
    load_plane(z0 - 2, &f, &fy);
    Planar pcur = planar_of(z0 - 2, f, fy);
    load_plane(z0 - 1, &nf, &nfy);
    Rec Rm, R0, Rp;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      Rm.v[t] = NONE;
      R0.v[t] = NONE;
      Rp.v[t] = NONE;
    }
    uint32_t Ec = NO_CODES, Fc = NO_CODES, Fcm = NO_CODES;
    for (int kk = z0 - 3; kk <= zend; ++kk) {
      // plane kk+2 was prefetched; start the load of plane kk+3
      f = nf;
      fy = nfy;
      load_plane(kk + 3, &nf, &nfy);
      const Planar pnext = planar_of(kk + 2, f, fy);
      Rm = R0;
      R0 = Rp;
      Rp = record(pcur, pnext);  // record of plane kk+1
      pcur = pnext;
      if (kk < z0 - 1) continue;
      uint32_t E, F;
      codes_of_plane(R0, Rm, Rp, &E, &F);  // codes of plane kk
      S.cw[kk & 1][row][lane] = make_uint2(E, F);
      uint32_t mask = 0;
      const int zc = kk - 1;
      if (zc >= z0) {
        // neighbours of plane zc: their codes were stored in the previous step,
        // before this step's barrier
        const uint32_t Fmy = row > 0 ? S.cw[zc & 1][row - 1][lane].y : NO_CODES;
        const uint32_t Epy = row < RW - 1 ? S.cw[zc & 1][row + 1][lane].x : NO_CODES;
        const uint32_t Fmx = lane_up1(Fc), Epx = lane_down1(Ec);
        if (inner) mask = classify(zc, Rm, Ec, Fc, Fcm, Fmy, Fmx, E, Epy, Epx);
      }
      Fcm = Fc;
      Ec = E;
      Fc = F;
      flush_staged(kk - 1, Rm, mask);  // also the barrier before the next step's record exchange
    }
    drain();
  }
  if (__ballot(nan) && lane == 0) {
    atomicOr(&img_status[im], 1u);
    atomicOr(&st->nan_input, 1u);
  }
}

template <int NDIM, int RW, int ZC, bool ROW1 = false>
void launch_stencil_t(int ntiles, const float* img, const ImgDesc* imgs, const int4* tiles, Layout L,
                      uint64_t* surv, uint64_t surv_cap, unsigned long long* surv_count, int32_t* vlink,
                      int32_t* tlink, uint8_t* eapp, uint32_t* img_status, Status* st, hipStream_t stream) {
  // CR_STAGE_KEYS lowers the staging capacity (0: every plane is written straight out)
  uint32_t stage_cap = stage_keys<RW>();
  if (const char* v = getenv("CR_STAGE_KEYS")) {
    const unsigned long c = strtoul(v, nullptr, 10);
    if (c < stage_cap) stage_cap = (uint32_t)c;
  }
  const size_t dyn = NDIM == 3 ? 2 * stage_keys<RW>() * sizeof(uint64_t) : 0;
  static bool attr_set = false;
  if (dyn && !attr_set) {
    (void)hipFuncSetAttribute((const void*)k_stencil<NDIM, RW, ZC, ROW1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)dyn);
    attr_set = true;
  }
  k_stencil<NDIM, RW, ZC, ROW1><<<ntiles, 64 * RW, dyn, stream>>>(img, imgs, tiles, L, surv, surv_cap, surv_count, vlink,
                                                            tlink, eapp, img_status, st, stage_cap);
}

constexpr int ROW1_VARIANT = 3;  // the one-row layout (not a tuning choice)

// Tile shapes: RW wavefronts (RW-2 interior rows of 62 pixels) and ZC planes.
struct TileVariant {
  int rw, zc;
};
constexpr TileVariant TILES2[3] = {{16, 1}, {8, 1}, {4, 1}};
constexpr TileVariant TILES3[3] = {{16, 32}, {16, 16}, {8, 32}};

void launch_apparent(int ndim, int variant, int ntiles, const float* img, const ImgDesc* imgs, const int4* tiles,
                     Layout L, uint64_t* surv, uint64_t surv_cap, unsigned long long* surv_count,
                     int32_t* vlink, int32_t* tlink, uint8_t* eapp, uint32_t* img_status, Status* st,
                     hipStream_t stream) {
  if (ntiles <= 0) return;
#define CR_STENCIL(N, R, Z) \
  launch_stencil_t<N, R, Z>(ntiles, img, imgs, tiles, L, surv, surv_cap, surv_count, vlink, tlink, eapp, img_status, st, stream)
  if (ndim == 2 && variant == ROW1_VARIANT) {
    launch_stencil_t<2, 16, 1, true>(ntiles, img, imgs, tiles, L, surv, surv_cap, surv_count, vlink, tlink, eapp,
                                     img_status, st, stream);
  } else if (ndim == 2) {
    if (variant == 1) CR_STENCIL(2, 8, 1);
    else if (variant == 2) CR_STENCIL(2, 4, 1);
    else CR_STENCIL(2, 16, 1);
  } else {
    if (variant == 1) CR_STENCIL(3, 16, 16);
    else if (variant == 2) CR_STENCIL(3, 8, 32);
    else CR_STENCIL(3, 16, 32);
  }
#undef CR_STENCIL
}

// Extents (z, y, x) of the interior of a tile of the one-row layout (variant
// ROW1_VARIANT of ndim 2, chosen by the library for calls whose images all have
// one row).
void stencil_tile_row1(int ext[3]) {
  ext[0] = 1;
  ext[1] = 1;
  ext[2] = 62 * 16;
}

// Extents (z, y, x) of the interior of stencil tile `variant` for ndim; false if there is no such variant.
bool stencil_tile(int ndim, int variant, int ext[3]) {
  if (variant < 0 || variant >= 3 || (ndim != 2 && ndim != 3)) return false;
  const TileVariant v = ndim == 2 ? TILES2[variant] : TILES3[variant];
  ext[0] = v.zc;
  ext[1] = v.rw - 2;
  ext[2] = 62;
  return true;
}

// Segment sizes of the sorted survivors: dim_count[d] = number of keys whose
// top field (the dimension) is d, by binary search for each boundary.
__global__ void k_dim_bounds(const uint64_t* __restrict__ keys, const unsigned long long* __restrict__ n_ptr,
                             uint64_t cap, Layout L, unsigned long long* __restrict__ dim_count) {
  __shared__ uint64_t first[5];
  const int t = threadIdx.x;
  const uint64_t n = *n_ptr < cap ? *n_ptr : cap;
  const int shift = L.ib + 32 + L.kb;
  if (t < 5) {
    // first index whose dimension is >= t
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
      const uint64_t m = (lo + hi) >> 1;
      if ((int)(keys[m] >> shift) < t) lo = m + 1;
      else hi = m;
    }
    first[t] = t == 4 ? n : lo;
  }
  __syncthreads();
  if (t < 4) dim_count[t] = first[t + 1] - first[t];
}

// ---- host launchers ----------------------------------------------------------
void launch_dim_bounds(const uint64_t* keys, const unsigned long long* n_ptr, uint64_t cap, Layout L,
                       unsigned long long* dim_count, hipStream_t s) {
  k_dim_bounds<<<1, 64, 0, s>>>(keys, n_ptr, cap, L, dim_count);
}

}  // namespace cr
