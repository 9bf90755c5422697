// Fused stencil pass: filtration values, apparent pairs, survivor compaction.
//
// One workgroup owns a tile of pixels and every cell anchored at them (cell k
// is anchored at pixel floor(k/2)).  It stages the pixel tile plus a halo in
// LDS (reads are coalesced along x), derives the value of every cell within
// Khalimsky distance 2 of the tile -- the maximum over the cell's vertices,
// the V-construction of Sec. 2 -- and then decides for each owned cell whether
// it belongs to an apparent pair:
//   (s, t) is apparent iff t is the earliest cofacet of s and s is the latest
//   facet of t, in the total order (value, dim, kidx).
// An apparent pair is a persistence pair of length zero (value(t) is the
// maximum over its facets, attained by its latest facet s), so it emits nothing
// and both cells leave the problem.  The remaining cells ("survivors") are
// compacted with wave64 ballots into one key array, dimension-major.
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
#include "cr_internal.h"

namespace cr {

template <int NDIM, int TX, int TY, int TZ>
struct ApparentTile {
  static constexpr int PX = TX + 3, PY = TY + 3, PZ = (NDIM == 3) ? TZ + 3 : 1;
  static constexpr int RX = 2 * TX + 4, RY = 2 * TY + 4, RZ = (NDIM == 3) ? 2 * TZ + 4 : 1;
  static constexpr int NT = TX * TY * TZ;
};

__device__ inline bool key_less(float va, uint32_t ka, float vb, uint32_t kb) {
  return va < vb || (va == vb && ka < kb);
}

template <int NDIM, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_apparent(
    const float* __restrict__ img, const ImgDesc* __restrict__ imgs, const int4* __restrict__ tiles,
    Layout L, uint64_t* __restrict__ surv, uint64_t surv_cap,
    unsigned long long* __restrict__ surv_count, int32_t* __restrict__ vlink, int32_t* __restrict__ tlink,
    uint8_t* __restrict__ eapp, uint32_t* __restrict__ img_status, Status* __restrict__ st) {
  using T = ApparentTile<NDIM, TX, TY, TZ>;
  __shared__ float pix[T::PZ * T::PY * T::PX];
  __shared__ float kv[T::RZ * T::RY * T::RX];
  __shared__ unsigned int wtot[T::NT / 64];
  __shared__ unsigned long long bbase;
  __shared__ unsigned int nan_seen;

  const int tid = threadIdx.x;
  const int4 tile = tiles[blockIdx.x];
  const int im = tile.x;
  const ImgDesc d = imgs[im];
  const int z0 = (NDIM == 3) ? tile.y : 0, y0 = tile.z, x0 = tile.w;
  if (tid == 0) nan_seen = 0;

  // ---- stage pixels (tile origin minus one, plus a halo of two after) ----
  const int pz0 = (NDIM == 3) ? z0 - 1 : 0;
  for (int i = tid; i < T::PZ * T::PY * T::PX; i += T::NT) {
    const int px = i % T::PX, py = (i / T::PX) % T::PY, pz = i / (T::PX * T::PY);
    const int gx = x0 - 1 + px, gy = y0 - 1 + py, gz = pz0 + pz;
    float v = INFINITY;
    if (gx >= 0 && gx < d.n[2] && gy >= 0 && gy < d.n[1] && gz >= 0 && gz < d.n[0]) {
      v = img[pixel_index(d, gz, gy, gx)];
      if (v != v) {
        nan_seen = 1;
        v = INFINITY;
      }
      v = canon(v);
    }
    pix[i] = v;
  }
  __syncthreads();
  if (tid == 0 && nan_seen) {
    atomicOr(&img_status[im], 1u);
    atomicOr(&st->nan_input, 1u);
  }

  // ---- values of all cells within Khalimsky distance 2 of the tile ----
  const int bz = (NDIM == 3) ? 2 * z0 - 2 : 0, by = 2 * y0 - 2, bx = 2 * x0 - 2;
  for (int i = tid; i < T::RZ * T::RY * T::RX; i += T::NT) {
    const int lx = i % T::RX, ly = (i / T::RX) % T::RY, lz = i / (T::RX * T::RY);
    const int kx = bx + lx, ky = by + ly, kz = bz + lz;
    float v = 0.0f;
    if (kx >= 0 && kx < d.K[2] && ky >= 0 && ky < d.K[1] && kz >= 0 && kz < d.K[0]) {
      const int qx = (kx >> 1) - (x0 - 1), qy = (ky >> 1) - (y0 - 1), qz = (kz >> 1) - pz0;
      v = -INFINITY;
      for (int dz = 0; dz <= (kz & 1); ++dz)
        for (int dy = 0; dy <= (ky & 1); ++dy)
          for (int dx = 0; dx <= (kx & 1); ++dx)
            v = fmaxf(v, pix[((qz + dz) * T::PY + qy + dy) * T::PX + qx + dx]);
    }
    kv[i] = v;
  }
  __syncthreads();

  // ---- classify the cells anchored at this thread's pixel ----
  constexpr int NCELL = 1 << NDIM;
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  const bool pix_in = gx < d.n[2] && gy < d.n[1] && gz < d.n[0];
  uint32_t surv_mask = 0;
  uint64_t keys[NCELL];
  const int Kd[3] = {d.K[0], d.K[1], d.K[2]};
  const int base[3] = {bz, by, bx};
  auto lidx = [&](const int k[3]) { return ((k[0] - base[0]) * T::RY + (k[1] - base[1])) * T::RX + (k[2] - base[2]); };
  auto kid = [&](const int k[3]) {
    return ((uint32_t)k[0] * (uint32_t)Kd[1] + (uint32_t)k[1]) * (uint32_t)Kd[2] + (uint32_t)k[2];
  };

#pragma unroll
  for (int cs = 0; cs < NCELL; ++cs) {
    const int dx = cs & 1, dy = (cs >> 1) & 1, dz = (NDIM == 3) ? (cs >> 2) & 1 : 0;
    int k[3] = {2 * gz + dz, 2 * gy + dy, 2 * gx + dx};
    if (!pix_in || k[0] >= Kd[0] || k[1] >= Kd[1] || k[2] >= Kd[2]) continue;
    const int dim = dx + dy + dz;
    const float vc = kv[lidx(k)];
    const uint32_t kc = kid(k);
    bool paired = false;

    // (a) as the facet of an apparent pair: earliest cofacet t, then is k the latest facet of t?
    if (dim < NDIM) {
      int ta = -1, ts = 0;
      float tv = 0.0f;
      uint32_t tk = 0;
      for (int a = 0; a < 3; ++a) {
        if (k[a] & 1) continue;
        for (int s = -1; s <= 1; s += 2) {
          int t[3] = {k[0], k[1], k[2]};
          t[a] += s;
          if (t[a] < 0 || t[a] >= Kd[a]) continue;
          const float v = kv[lidx(t)];
          const uint32_t kk = kid(t);
          if (ta < 0 || key_less(v, kk, tv, tk)) {
            ta = a; ts = s; tv = v; tk = kk;
          }
        }
      }
      bool latest = false;
      if (ta >= 0) {
        int t[3] = {k[0], k[1], k[2]};
        t[ta] += ts;
        latest = true;
        for (int b = 0; b < 3 && latest; ++b) {
          if (!(t[b] & 1)) continue;
          for (int s = -1; s <= 1; s += 2) {
            int f[3] = {t[0], t[1], t[2]};
            f[b] += s;
            if (f[0] == k[0] && f[1] == k[1] && f[2] == k[2]) continue;
            if (key_less(vc, kc, kv[lidx(f)], kid(f))) {
              latest = false;
              break;
            }
          }
        }
      }
      if (NDIM == 3 && dim == 1 && eapp) {
        // apparent-partner code of an edge for the degree-1 reduction:
        // 2 * axis + (direction > 0) of its partner square, 0xFF if none
        const int oa = (k[0] & 1) ? 0 : ((k[1] & 1) ? 1 : 2);
        eapp[3 * pixel_index(d, k[0] >> 1, k[1] >> 1, k[2] >> 1) + oa] =
            latest ? (uint8_t)(2 * ta + (ts > 0 ? 1 : 0)) : (uint8_t)0xFF;
      }
      if (latest) {
        paired = true;
        if (dim == 0) {  // vertex: link to the other endpoint of its edge
          int o[3] = {k[0], k[1], k[2]};
          o[ta] += 2 * ts;
          vlink[pixel_index(d, k[0] >> 1, k[1] >> 1, k[2] >> 1)] =
              (int32_t)pixel_index(d, o[0] >> 1, o[1] >> 1, o[2] >> 1);
        }
      }
    }
    // (b) as the cofacet of an apparent pair: latest facet s, then is k the earliest cofacet of s?
    if (!paired && dim >= 1) {
      int sa = -1, ss = 0;
      float sv = 0.0f;
      uint32_t sk = 0;
      for (int a = 0; a < 3; ++a) {
        if (!(k[a] & 1)) continue;
        for (int s = -1; s <= 1; s += 2) {
          int f[3] = {k[0], k[1], k[2]};
          f[a] += s;
          const float v = kv[lidx(f)];
          const uint32_t kk = kid(f);
          if (sa < 0 || key_less(sv, sk, v, kk)) {
            sa = a; ss = s; sv = v; sk = kk;
          }
        }
      }
      int f[3] = {k[0], k[1], k[2]};
      f[sa] += ss;
      bool earliest = true;
      for (int b = 0; b < 3 && earliest; ++b) {
        if (f[b] & 1) continue;
        for (int s = -1; s <= 1; s += 2) {
          int g[3] = {f[0], f[1], f[2]};
          g[b] += s;
          if (g[b] < 0 || g[b] >= Kd[b]) continue;
          if (g[0] == k[0] && g[1] == k[1] && g[2] == k[2]) continue;
          if (key_less(kv[lidx(g)], kid(g), vc, kc)) {
            earliest = false;
            break;
          }
        }
      }
      if (earliest) {
        paired = true;
        if (dim == NDIM) {  // top cell: link to the other cofacet of its facet, or the exterior
          int o[3] = {k[0], k[1], k[2]};
          o[sa] += 2 * ss;
          int32_t to;
          if (o[sa] < 0 || o[sa] >= Kd[sa]) to = -(im + 2);
          else to = (int32_t)pixel_index(d, o[0] >> 1, o[1] >> 1, o[2] >> 1);
          tlink[pixel_index(d, k[0] >> 1, k[1] >> 1, k[2] >> 1)] = to;
        }
      }
    }
    if (!paired) {
      surv_mask |= 1u << cs;
      uint32_t bits;
      __builtin_memcpy(&bits, &vc, 4);
      keys[cs] = make_skey(L, dim, im, ord32_bits(bits), kc);
      if (dim == 0) vlink[pixel_index(d, k[0] >> 1, k[1] >> 1, k[2] >> 1)] = -1;
      if (dim == NDIM) tlink[pixel_index(d, k[0] >> 1, k[1] >> 1, k[2] >> 1)] = -1;
    }
  }

  // ---- append this workgroup's survivors with one atomic ----
  const uint32_t mine = __popc(surv_mask);
  const int lane = __lane_id(), wave = tid >> 6;
  uint32_t incl = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t up = __shfl_up(incl, off, 64);
    if (lane >= off) incl += up;
  }
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int w = 0; w < T::NT / 64; ++w) {
      const uint32_t t = wtot[w];
      wtot[w] = run;
      run += t;
    }
    bbase = run ? atomicAdd(surv_count, (unsigned long long)run) : 0ull;
  }
  __syncthreads();
  unsigned long long pos = bbase + wtot[wave] + incl - mine;
#pragma unroll
  for (int cs = 0; cs < NCELL; ++cs) {
    if (surv_mask & (1u << cs)) {
      if (pos < surv_cap) surv[pos] = keys[cs];
      else raise_flag(st, &st->overflow, OVF_SURVIVORS);
      ++pos;
    }
  }
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

// ---- host launcher ----------------------------------------------------------
void launch_apparent(int ndim, int variant, int ntiles, const float* img, const ImgDesc* imgs, const int4* tiles,
                     Layout L, uint64_t* surv, uint64_t surv_cap, unsigned long long* surv_count,
                     int32_t* vlink, int32_t* tlink, uint8_t* eapp, uint32_t* img_status, Status* st,
                     hipStream_t stream) {
  if (ntiles <= 0) return;
#define CR_APPARENT(N, X, Y, Z)                                                                     \
  k_apparent<N, X, Y, Z><<<ntiles, X * Y * Z, 0, stream>>>(img, imgs, tiles, L, surv, surv_cap, surv_count, \
                                                         vlink, tlink, eapp, img_status, st)
  // tile shapes (x, y, z extents) indexed by variant; they must match stencil_tile()
  if (ndim == 2) {
    if (variant == 1) CR_APPARENT(2, 64, 4, 1);
    else if (variant == 2) CR_APPARENT(2, 16, 16, 1);
    else CR_APPARENT(2, 32, 8, 1);
  } else {
    if (variant == 1) CR_APPARENT(3, 32, 4, 2);
    else if (variant == 2) CR_APPARENT(3, 8, 8, 4);
    else CR_APPARENT(3, 16, 4, 4);
  }
#undef CR_APPARENT
}

// Extents (z, y, x) of stencil tile `variant` for ndim; returns false if there is no such variant.
bool stencil_tile(int ndim, int variant, int ext[3]) {
  static const int t2[3][3] = {{1, 8, 32}, {1, 4, 64}, {1, 16, 16}};
  static const int t3[3][3] = {{4, 4, 16}, {2, 4, 32}, {4, 8, 8}};
  if (variant < 0 || variant >= 3 || (ndim != 2 && ndim != 3)) return false;
  const int* t = ndim == 2 ? t2[variant] : t3[variant];
  ext[0] = t[0];
  ext[1] = t[1];
  ext[2] = t[2];
  return true;
}

void launch_dim_bounds(const uint64_t* keys, const unsigned long long* n_ptr, uint64_t cap, Layout L,
                       unsigned long long* dim_count, hipStream_t s) {
  k_dim_bounds<<<1, 64, 0, s>>>(keys, n_ptr, cap, L, dim_count);
}

}  // namespace cr
