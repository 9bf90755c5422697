// Degree 1 of a volume: reduction of the coboundary matrix over Z/2 (Sec. 2).
//
// Columns are the surviving edges that kill no component (clearing: the deaths
// of degree 0 reduce to zero), ordered by decreasing key -- column id 0 is the
// latest edge.  A column holds the squares of a coboundary, enumerated from
// the image on the fly (at most four per edge), as an ascending list of keys;
// its pivot is the smallest key.  Column j is reduced while its pivot t is
// owned by a column to its left:
//   * t belongs to an apparent pair (s, t): s is to the left of every column
//     that can reach t, and its column is its raw coboundary -- add that;
//   * owner[t] = k < j: add the published column of k;
//   * owner[t] = k > j: j takes t over (CAS) and the thread goes on to reduce k,
//     which has just lost its pivot;
//   * no owner: j publishes its column and claims t (CAS).
// Every addition adds a column to its left, so whatever order the threads run
// in, the end state is a reduced matrix and -- the pivots of a reduced matrix
// being unique -- the pairing is the one the sequential reduction gives.
//
// Columns live in an append-only arena: a column version is written once and
// published by a release store of (offset, length); readers acquire it, so a
// column can be read while its owner is rewritten.
#include "cr_emit.h"

namespace cr {

constexpr uint32_t RED_ITER_CAP = 1u << 24;

struct RedCtx {
  const float* img;
  const ImgDesc* imgs;
  Layout L;
  const uint64_t* skeys;
  const unsigned long long* dim_count;
  const uint8_t* neg;
  int32_t* owner;     // per square (3 * anchor pixel + orientation): owning column, or -1
  uint64_t* piv;      // per column: key of its pivot square
  uint64_t* col_ptr;  // per column: (arena offset << 24) | length
  uint64_t* arena;
  uint64_t arena_cap;
  unsigned long long* arena_top;
  Status* st;
};

__device__ inline uint64_t sq_key(const RedCtx& R, int im, const ImgDesc& d, const int c[3]) {
  const float v = cell_value(R.img, d, c);
  uint32_t bits;
  __builtin_memcpy(&bits, &v, 4);
  return make_skey(R.L, 2, im, ord32_bits(bits), coords_kidx(d, c));
}
__device__ inline uint64_t edge_key(const RedCtx& R, int im, const ImgDesc& d, const int c[3]) {
  const float v = cell_value(R.img, d, c);
  uint32_t bits;
  __builtin_memcpy(&bits, &v, 4);
  return make_skey(R.L, 1, im, ord32_bits(bits), coords_kidx(d, c));
}
__device__ inline int64_t sq_slot(const ImgDesc& d, const int c[3]) {
  const int orient = !(c[0] & 1) ? 0 : (!(c[1] & 1) ? 1 : 2);
  return 3 * anchor_pixel(d, c) + orient;
}

// Cofacets (squares) of edge c, ascending.
__device__ inline int edge_cob(const RedCtx& R, int im, const ImgDesc& d, const int c[3], uint64_t out[4]) {
  int n = 0;
  for (int b = 0; b < 3; ++b) {
    if (c[b] & 1) continue;
    for (int s = -1; s <= 1; s += 2) {
      int t[3] = {c[0], c[1], c[2]};
      t[b] += s;
      if (t[b] < 0 || t[b] >= d.K[b]) continue;
      out[n++] = sq_key(R, im, d, t);
    }
  }
  for (int i = 1; i < n; ++i) {
    const uint64_t v = out[i];
    int j = i - 1;
    while (j >= 0 && out[j] > v) {
      out[j + 1] = out[j];
      --j;
    }
    out[j + 1] = v;
  }
  return n;
}

// If square t is in an apparent pair (s, t), writes the coboundary of s into
// cob and returns its length; returns 0 otherwise.
__device__ inline int apparent_cob(const RedCtx& R, int im, const ImgDesc& d, const int tc[3],
                                   uint64_t tkey, uint64_t cob[4]) {
  int best[3] = {0, 0, 0};
  uint64_t bk = 0;
  bool have = false;
  for (int a = 0; a < 3; ++a) {
    if (!(tc[a] & 1)) continue;
    for (int s = -1; s <= 1; s += 2) {
      int f[3] = {tc[0], tc[1], tc[2]};
      f[a] += s;
      const uint64_t k = edge_key(R, im, d, f);
      if (!have || k > bk) {
        have = true;
        bk = k;
        best[0] = f[0]; best[1] = f[1]; best[2] = f[2];
      }
    }
  }
  const int n = edge_cob(R, im, d, best, cob);
  return (n > 0 && cob[0] == tkey) ? n : 0;
}

__device__ inline uint64_t arena_alloc(const RedCtx& R, uint32_t len) {
  const unsigned long long off = atomicAdd(R.arena_top, (unsigned long long)len);
  if (off + len > R.arena_cap) {
    raise_flag(R.st, &R.st->overflow);
    return ~0ull;
  }
  return off;
}

// out = a XOR b for ascending lists; returns the length.
__device__ inline uint32_t xor_lists(const uint64_t* a, uint32_t na, const uint64_t* b, uint32_t nb,
                                     uint64_t* out) {
  uint32_t i = 0, j = 0, m = 0;
  while (i < na && j < nb) {
    const uint64_t x = a[i], y = b[j];
    if (x < y) { out[m++] = x; ++i; }
    else if (y < x) { out[m++] = y; ++j; }
    else { ++i; ++j; }
  }
  while (i < na) out[m++] = a[i++];
  while (j < nb) out[m++] = b[j++];
  return m;
}

__device__ inline uint64_t pack_col(uint64_t off, uint32_t len) { return (off << 24) | len; }

// Reduce column c (and every column it takes a pivot from).
__device__ void reduce_column(const RedCtx& R, uint32_t c, uint64_t off1, uint64_t n1) {
  // initial column: the coboundary of the edge
  uint64_t woff, wlen;
  {
    const uint64_t ek = R.skeys[off1 + (n1 - 1 - c)];
    const int im = skey_img(R.L, ek);
    const ImgDesc d = R.imgs[im];
    int ec[3];
    kidx_coords(d, skey_kidx(R.L, ek), ec);
    uint64_t cob[4];
    const int n = edge_cob(R, im, d, ec, cob);
    woff = arena_alloc(R, 4);
    if (woff == ~0ull) return;
    for (int i = 0; i < n; ++i) R.arena[woff + i] = cob[i];
    wlen = n;
  }
  for (uint32_t it = 0; it < RED_ITER_CAP; ++it) {
    if ((it & 63) == 63 && aborted(R.st)) return;
    if (wlen == 0) {  // would be an essential class of degree 1: impossible in a box
      raise_flag(R.st, &R.st->internal);
      return;
    }
    const uint64_t t = R.arena[woff];
    const int im = skey_img(R.L, t);
    const ImgDesc d = R.imgs[im];
    int tc[3];
    kidx_coords(d, skey_kidx(R.L, t), tc);
    uint64_t cob[4];
    const int na = apparent_cob(R, im, d, tc, t, cob);
    if (na > 0) {  // owner: the apparent partner, whose column is its raw coboundary
      const uint64_t noff = arena_alloc(R, (uint32_t)(wlen + na));
      if (noff == ~0ull) return;
      wlen = xor_lists(R.arena + woff, (uint32_t)wlen, cob, (uint32_t)na, R.arena + noff);
      woff = noff;
      continue;
    }
    int32_t* slot = R.owner + sq_slot(d, tc);
    const int32_t o = ld_acq32(slot);
    if (o < 0 || (uint32_t)o > c) {
      // publish this column, then claim t (or take it over from column o > c)
      if (wlen >= (1u << 24)) {
        raise_flag(R.st, &R.st->overflow);
        return;
      }
      st_rel64(&R.col_ptr[c], pack_col(woff, (uint32_t)wlen));
      R.piv[c] = t;
      if (cas32_rel(slot, o, (int32_t)c)) {
        if (o < 0) return;
        // column o lost its pivot: reduce it next, from its published version
        c = (uint32_t)o;
        const uint64_t p = ld_acq64(&R.col_ptr[c]);
        woff = p >> 24;
        wlen = p & ((1u << 24) - 1);
      }
      continue;
    }
    if ((uint32_t)o == c) {  // cannot happen: c is held by this thread
      raise_flag(R.st, &R.st->internal);
      return;
    }
    // o < c: add the column of o
    const uint64_t p = ld_acq64(&R.col_ptr[o]);
    const uint64_t ooff = p >> 24;
    const uint32_t olen = (uint32_t)(p & ((1u << 24) - 1));
    const uint64_t noff = arena_alloc(R, (uint32_t)(wlen + olen));
    if (noff == ~0ull) return;
    wlen = xor_lists(R.arena + woff, (uint32_t)wlen, R.arena + ooff, olen, R.arena + noff);
    woff = noff;
  }
  raise_flag(R.st, &R.st->iter_cap);
}

__global__ void k_h1_reduce(RedCtx R) {
  if (aborted(R.st)) return;
  const uint64_t off1 = R.dim_count[0];
  const uint64_t n1 = R.dim_count[1];
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < n1;
       c += (uint64_t)gridDim.x * blockDim.x) {
    if (aborted(R.st)) return;
    if (R.neg[n1 - 1 - c]) continue;
    reduce_column(R, (uint32_t)c, off1, n1);
  }
}

// Degree-1 rows of a volume: column c pairs its edge with its final pivot.
__global__ void k_h1_emit(RedCtx R, EmitCtx E) {
  if (aborted(R.st)) return;
  const uint64_t off1 = R.dim_count[0];
  const uint64_t n1 = R.dim_count[1];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t nr = (n1 + 63) & ~63ull;
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < nr; c += stride) {
    bool active = false;
    int im = 0;
    uint64_t ck = 0;
    if (c < n1 && !R.neg[n1 - 1 - c]) {
      const uint64_t t = R.piv[c];
      const ImgDesc d = R.imgs[skey_img(R.L, t)];
      int tc[3];
      kidx_coords(d, skey_kidx(R.L, t), tc);
      if (R.owner[sq_slot(d, tc)] != (int32_t)c) raise_flag(R.st, &R.st->internal);
      else active = pair_row(E, R.skeys[off1 + (n1 - 1 - c)], t, false, &im, &ck);
    }
    emit_rows(E, active, im, ck);
  }
}

void launch_h1_reduce_raw(int grid, const float* img, const ImgDesc* imgs, Layout L, const uint64_t* skeys,
                          const unsigned long long* dim_count, const uint8_t* neg, int32_t* owner,
                          uint64_t* piv, uint64_t* col_ptr, uint64_t* arena, uint64_t arena_cap,
                          unsigned long long* arena_top, Status* st, const EmitCtx& E, hipStream_t s) {
  RedCtx R;
  R.img = img;
  R.imgs = imgs;
  R.L = L;
  R.skeys = skeys;
  R.dim_count = dim_count;
  R.neg = neg;
  R.owner = owner;
  R.piv = piv;
  R.col_ptr = col_ptr;
  R.arena = arena;
  R.arena_cap = arena_cap;
  R.arena_top = arena_top;
  R.st = st;
  k_h1_reduce<<<grid, 256, 0, s>>>(R);
  k_h1_emit<<<grid, 256, 0, s>>>(R, E);
}

}  // namespace cr
