// Degree 0 and the top degree by union-find with the elder rule.
//
// Degree 0 (Sec. 2, Fig. 2): the surviving edges are visited in filtration
// order and an edge joining two components kills the younger one.  The top
// degree (1-cycles of an image, 2-cycles of a volume) is the same computation
// on the dual graph -- top cells plus one exterior node per image, joined by
// the (top-1)-cells -- in the reversed order, where the exterior node is the
// oldest (Alexander duality, Remark 2.1).  Both run here as one kernel.
//
// Sequential Kruskal order is replaced by a merge structure whose final state
// does not depend on the order in which edges are inserted: every node x holds
// one 64-bit word T[x] = (level s, node v) meaning "x is joined to the older
// node v by level s".  rep(x, s) follows these words while their level is <= s.
// Inserting edge (a, b) at level s: take r_a = rep(a, s), r_b = rep(b, s); if
// they differ, the younger y of the two is relinked to the older o at level s
// by one 64-bit CAS, and the fact it held before (y joined to v at a higher
// level s') is re-inserted as (o, v, s').  Levels only decrease in each word,
// so every loop terminates, and once all edges are in, T[x].s is the level at
// which x first meets an older node -- exactly the elder-rule death of x.  The
// edges can therefore be inserted by all threads at once, lock-free.
#include "cr_emit.h"

namespace cr {

constexpr uint32_t ITER_CAP = 1u << 22;

// ---- the merge structure -------------------------------------------------------
__device__ inline uint32_t trip_rep(uint64_t* T, uint32_t x, uint32_t s, Status* st) {
  for (uint32_t it = 0; it < ITER_CAP; ++it) {
    const uint64_t t = ld_rlx64(&T[x]);
    if ((uint32_t)(t >> 32) <= s) x = (uint32_t)t;
    else return x;
  }
  raise_flag(st, &st->iter_cap);
  return x;
}

__device__ inline void trip_merge(uint64_t* T, uint32_t a, uint32_t b, uint32_t s, Status* st) {
  for (uint32_t it = 0; it < ITER_CAP; ++it) {
    a = trip_rep(T, a, s, st);
    b = trip_rep(T, b, s, st);
    if (a == b) return;
    const uint32_t y = a > b ? a : b, o = a > b ? b : a;
    const uint64_t old = ld_rlx64(&T[y]);
    const uint32_t os = (uint32_t)(old >> 32);
    if (os <= s) continue;  // y was relinked meanwhile; walk again
    if (cas64(&T[y], old, ((uint64_t)s << 32) | o)) {
      if (os == TRIP_INF) return;
      a = o;
      b = (uint32_t)old;
      s = os;
    }
    if ((it & 15) == 15 && aborted(st)) return;
  }
  raise_flag(st, &st->iter_cap);
}

__global__ void k_trip_init(uint64_t* __restrict__ T, const unsigned long long* __restrict__ cnt,
                            int cnt_index, uint32_t extra) {
  const uint64_t n = cnt[cnt_index] + extra;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    T[i] = ((uint64_t)TRIP_INF << 32) | (uint32_t)i;
}

// Segment [off, off + n) of dimension dm in the sorted survivor array.
__device__ inline void segment(const unsigned long long* dim_count, int dm, uint64_t* off, uint64_t* n) {
  uint64_t o = 0;
  for (int i = 0; i < dm; ++i) o += dim_count[i];
  *off = o;
  *n = dim_count[dm];
}

// Surviving vertices become forest roots: vlink[pixel] = -(rank + 2).
__global__ void k_vroot_init(const uint64_t* __restrict__ skeys, const unsigned long long* __restrict__ dim_count,
                             const ImgDesc* __restrict__ imgs, Layout L, int32_t* __restrict__ vlink,
                             const Status* __restrict__ st) {
  if (aborted(st)) return;
  uint64_t off, n;
  segment(dim_count, 0, &off, &n);
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n;
       r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = skeys[off + r];
    const ImgDesc d = imgs[skey_img(L, k)];
    int c[3];
    kidx_coords(d, skey_kidx(L, k), c);
    vlink[anchor_pixel(d, c)] = -(int32_t)(r + 2);
  }
}

// Surviving top cells become dual roots: tlink[anchor] = -(id + 2), where the
// dual node id of the cell at ascending rank r is nimg + (ntop - 1 - r) (the
// exterior nodes 0..nimg-1 are the oldest; larger keys are older).
__global__ void k_troot_init(const uint64_t* __restrict__ skeys, const unsigned long long* __restrict__ dim_count,
                             int top, const ImgDesc* __restrict__ imgs, Layout L, int32_t* __restrict__ tlink,
                             const Status* __restrict__ st) {
  if (aborted(st)) return;
  uint64_t off, n;
  segment(dim_count, top, &off, &n);
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n;
       r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = skeys[off + r];
    const ImgDesc d = imgs[skey_img(L, k)];
    int c[3];
    kidx_coords(d, skey_kidx(L, k), c);
    tlink[anchor_pixel(d, c)] = -(int32_t)(L.nimg + (n - 1 - r) + 2);
  }
}

// Roots of the forest nodes x and y, walked together (their loads overlap); a
// side with `done` set is not walked and keeps the value in *rx / *ry.
__device__ inline void forest_roots2(const int32_t* link, int64_t x, int64_t y, bool dx, bool dy,
                                     uint32_t* rx, uint32_t* ry, Status* st) {
  for (uint32_t it = 0; it < ITER_CAP; ++it) {
    if (dx && dy) return;
    const int32_t vx = dx ? 0 : link[x];
    const int32_t vy = dy ? 0 : link[y];
    if (!dx) {
      if (vx == -1) {  // a root that was never numbered: inconsistent state
        raise_flag(st, &st->internal);
        *rx = 0;
        dx = true;
      } else if (vx < 0) {
        *rx = (uint32_t)(-(vx + 2));
        dx = true;
      } else {
        x = vx;
      }
    }
    if (!dy) {
      if (vy == -1) {
        raise_flag(st, &st->internal);
        *ry = 0;
        dy = true;
      } else if (vy < 0) {
        *ry = (uint32_t)(-(vy + 2));
        dy = true;
      } else {
        y = vy;
      }
    }
  }
  raise_flag(st, &st->iter_cap);
  *rx = 0;
  *ry = 0;
}

// Degree 0: insert every surviving edge (level = its rank among edges).
__global__ void k_h0_merge(const uint64_t* __restrict__ skeys, const unsigned long long* __restrict__ dim_count,
                           const ImgDesc* __restrict__ imgs, Layout L, const int32_t* __restrict__ vlink,
                           uint64_t* __restrict__ T, uint32_t chunks, Status* __restrict__ st) {
  uint64_t off, n;
  segment(dim_count, 1, &off, &n);
  uint32_t j = 0;
  const Walk w = chunk_walk(n, chunks);
  for (uint64_t i = w.i; i < w.end; i += w.stride) {
    if ((j++ & 15) == 0 && aborted(st)) return;  // (a flag read costs a round trip to L2)
    const uint64_t k = skeys[off + i];
    const ImgDesc d = imgs[skey_img(L, k)];
    int c[3];
    kidx_coords(d, skey_kidx(L, k), c);
    const int a = (c[0] & 1) ? 0 : ((c[1] & 1) ? 1 : 2);
    int p[3] = {c[0], c[1], c[2]}, q[3] = {c[0], c[1], c[2]};
    p[a] -= 1;
    q[a] += 1;
    uint32_t ra = 0, rb = 0;
    forest_roots2(vlink, anchor_pixel(d, p), anchor_pixel(d, q), false, false, &ra, &rb, st);
    trip_merge(T, ra, rb, (uint32_t)i, st);
  }
}

// Degree 0 rows; marks edges that kill a component (they are not 1-columns).
__global__ void k_h0_emit(const uint64_t* __restrict__ skeys, const unsigned long long* __restrict__ dim_count,
                          const uint64_t* __restrict__ T, uint8_t* __restrict__ neg, EmitCtx E) {
  if (aborted_block(E.st)) return;
  uint64_t off0, n0, off1, n1;
  segment(dim_count, 0, &off0, &n0);
  segment(dim_count, 1, &off1, &n1);
  emit_tiled(E, n0, [&](uint64_t r, int* im, uint64_t* ck) {
    const uint64_t t = T[r];
    const uint32_t s = (uint32_t)(t >> 32);
    const bool ess = s == TRIP_INF;
    if (!ess) {
      if (s >= n1) {
        raise_flag(E.st, &E.st->internal);
        return false;
      }
      neg[s] = 1;
    }
    return pair_row(E, skeys[off0 + r], ess ? 0 : skeys[off1 + s], ess, im, ck);
  });
}

// Top degree on the dual graph.  For an image (top = 2) the columns are the
// surviving edges that kill no component (clearing).  For a volume (top = 3)
// every surviving square is a column: a square whose column would reduce to
// zero closes a cycle of the dual graph and merges nothing, so no clearing is
// needed, and degree 2 can run before degree 1.
// level = n - 1 - i (larger key = earlier in the reversed order).
__device__ inline bool dual_col_skipped(int top, uint64_t i, const uint8_t* neg) {
  return top == 2 && neg[i] != 0;
}

__global__ void k_dual_merge(int top, const uint64_t* __restrict__ skeys,
                             const unsigned long long* __restrict__ dim_count,
                             const ImgDesc* __restrict__ imgs, Layout L, const int32_t* __restrict__ tlink,
                             const uint8_t* __restrict__ neg, uint64_t* __restrict__ T, Status* __restrict__ st) {
  uint64_t off, n;
  segment(dim_count, top - 1, &off, &n);
  uint32_t jj = 0;
  const Walk w = chunk_walk(n, ~0u);  // one chunk per wavefront
  for (uint64_t i = w.i; i < w.end; i += w.stride) {
    if ((jj++ & 15) == 0 && aborted(st)) return;  // (a flag read costs a round trip to L2)
    const uint64_t k = skeys[off + i];
    const int im = skey_img(L, k);
    const ImgDesc d = imgs[im];
    int c[3];
    kidx_coords(d, skey_kidx(L, k), c);
    if (dual_col_skipped(top, i, neg)) continue;
    // the one even axis of the cell within the image's own dimensions (selects,
    // not an index: an indexed local array would be placed in LDS)
    const int a = (top == 2) ? ((c[1] & 1) ? 2 : 1) : (!(c[0] & 1) ? 0 : (!(c[1] & 1) ? 1 : 2));
    const int ka = a == 0 ? d.K[0] : a == 1 ? d.K[1] : d.K[2];
    const int ca = a == 0 ? c[0] : a == 1 ? c[1] : c[2];
    if (ka == 1) continue;  // no cofacet at all (a flat image): a loop at the exterior node
    // the two top cofacets differ from c by -1 and +1 along a; one outside the
    // image is the exterior node
    const int lo[3] = {c[0] - (a == 0), c[1] - (a == 1), c[2] - (a == 2)};
    const int hi[3] = {c[0] + (a == 0), c[1] + (a == 1), c[2] + (a == 2)};
    const bool out0 = ca == 0, out1 = ca + 1 >= ka;
    uint32_t e0 = (uint32_t)im, e1 = (uint32_t)im;
    forest_roots2(tlink, out0 ? 0 : anchor_pixel(d, lo), out1 ? 0 : anchor_pixel(d, hi), out0, out1, &e0, &e1,
                  st);
    trip_merge(T, e0, e1, (uint32_t)(n - 1 - i), st);
  }
}

// Rows of the top degree; with `mark`, also flags each column that gives birth
// to a class (mark[column position] = 1), the clearing set of degree top-1.
__global__ void k_dual_emit(int top, const uint64_t* __restrict__ skeys,
                            const unsigned long long* __restrict__ dim_count, const uint64_t* __restrict__ T,
                            uint8_t* __restrict__ mark, int emit, EmitCtx E) {
  if (aborted_block(E.st)) return;
  uint64_t offc, nc, offt, nt;
  segment(dim_count, top - 1, &offc, &nc);
  segment(dim_count, top, &offt, &nt);
  emit_tiled(E, nt, [&](uint64_t r, int* im, uint64_t* ck) {
    const uint64_t id = E.L.nimg + (nt - 1 - r);
    const uint64_t t = T[id];
    const uint32_t s = (uint32_t)(t >> 32);
    if (s == TRIP_INF || s >= nc) {
      raise_flag(E.st, &E.st->internal);  // a top cell that never dies: impossible in a box
      return false;
    }
    if (mark) mark[nc - 1 - s] = 1;
    return emit != 0 && pair_row(E, skeys[offc + (nc - 1 - s)], skeys[offt + r], false, im, ck);
  });
}

// ---- host launchers ------------------------------------------------------------
void launch_h0(int grid, const uint64_t* skeys, const unsigned long long* dim_count, const ImgDesc* imgs,
               Layout L, int32_t* vlink, uint64_t* T, uint8_t* neg, const EmitCtx& E, Status* st,
               hipStream_t s) {
  k_vroot_init<<<grid, 256, 0, s>>>(skeys, dim_count, imgs, L, vlink, st);
  k_trip_init<<<grid, 256, 0, s>>>(T, dim_count, 0, 0);
  // degree 0: a single image is walked by the whole grid at once (measured
  // best on a 256^3 volume); a batch gets about one chunk per image
  const uint32_t chunks = L.nimg < 8 ? 0u : (uint32_t)((L.nimg + 7) / 8);
  k_h0_merge<<<grid, 256, 0, s>>>(skeys, dim_count, imgs, L, vlink, T, chunks, st);
  k_h0_emit<<<grid, 256, 0, s>>>(skeys, dim_count, T, neg, E);
}

void launch_dual(int grid, int top, const uint64_t* skeys, const unsigned long long* dim_count,
                 const ImgDesc* imgs, Layout L, int32_t* tlink, const uint8_t* neg, uint8_t* mark, int emit,
                 uint64_t* T, const EmitCtx& E, Status* st, hipStream_t s) {
  k_troot_init<<<grid, 256, 0, s>>>(skeys, dim_count, top, imgs, L, tlink, st);
  k_trip_init<<<grid, 256, 0, s>>>(T, dim_count, top, (uint32_t)L.nimg);
  k_dual_merge<<<grid, 256, 0, s>>>(top, skeys, dim_count, imgs, L, tlink, neg, T, st);
  k_dual_emit<<<grid, 256, 0, s>>>(top, skeys, dim_count, T, mark, emit, E);
}

}  // namespace cr
