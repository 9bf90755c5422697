// Degree 1 of a volume: reduction of the boundary matrix over Z/2 (Sec. 2).
//
// The pivots of any reduced matrix give the same pairing, and the pairing of
// the boundary matrix (homology) is the one of the coboundary matrix
// (cohomology) the paper describes; degree 1 of a volume is reduced here in
// homology, where a working column is a 1-chain (a loop of edges) rather than
// a 2-cochain, which keeps columns short.
//
// Columns are the surviving squares that are not births of degree 2 (clearing:
// those reduce to zero; the dual union-find of degree 2 runs first and marks
// them).  Column id = rank of the square (ascending key), so "left" is
// "smaller id".  A column is the list of its boundary edges (4 per square,
// enumerated from the image); its pivot is its largest key.
//
// The reduction runs in rounds.  During a round the owner table and the
// columns of finished ("done") columns are read-only, so every thread reads
// them with plain cached loads; kernel boundaries publish what a round wrote.
// In a round every active column j is reduced while its pivot e is owned by a
// column to its left:
//   * e belongs to an apparent pair (e, s): s is e's earliest cofacet, hence to
//     the left of every column holding e, and its column is its raw boundary;
//   * owner[e] = k < j: add the column of k;
// and when e has no owner, or its owner lies to the right, j stores its column
// and proposes itself for e (atomicMin).  The commit step makes the leftmost
// proposer the owner; a column that loses, and an owner that was displaced,
// stay active for the next round.  Every addition adds a column to its left, so
// the rounds end in a reduced matrix with the unique pivots of the sequential
// reduction.
//
// A working column is kept in two sorted parts: a short front list F (at most
// FCAP entries plus one addend) that absorbs small additions, and a tail T.
// The pivot is the larger of the two last entries after cancelling equal ones,
// so adding a 4-entry boundary to a long column costs O(FCAP), not O(length);
// F is merged into T only when it overflows.  Stored columns live in an
// append-only arena.
#include "cr_reduce.h"

namespace cr {


__device__ inline uint64_t cell_key(const RedCtx& R, int dim, int im, const ImgDesc& d, const int c[3]) {
  const float v = cell_value(R.img, d, c);
  uint32_t bits;
  __builtin_memcpy(&bits, &v, 4);
  return make_skey(R.L, dim, im, ord32_bits(bits), coords_kidx(d, c));
}
__device__ inline int64_t edge_slot(const ImgDesc& d, const int c[3]) {
  const int axis = (c[0] & 1) ? 0 : ((c[1] & 1) ? 1 : 2);
  return 3 * anchor_pixel(d, c) + axis;
}

__device__ inline void sort_small(uint64_t* a, int n) {
  for (int i = 1; i < n; ++i) {
    const uint64_t v = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > v) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = v;
  }
}

// Boundary (edges) of square c, ascending.
__device__ inline int sq_boundary(const RedCtx& R, int im, const ImgDesc& d, const int c[3], uint64_t out[4]) {
  int n = 0;
  for (int a = 0; a < 3; ++a) {
    if (!(c[a] & 1)) continue;
    for (int s = -1; s <= 1; s += 2) {
      int f[3] = {c[0], c[1], c[2]};
      f[a] += s;
      out[n++] = cell_key(R, 1, im, d, f);
    }
  }
  sort_small(out, n);
  return n;
}

// If edge e is in an apparent pair (e, s) -- s its earliest cofacet and e the
// latest facet of s -- writes the boundary of s into bnd and returns its length.
__device__ inline int apparent_bnd(const RedCtx& R, int im, const ImgDesc& d, const int ec[3], uint64_t ekey,
                                   uint64_t bnd[4]) {
  int best[3] = {0, 0, 0};
  uint64_t bk = 0;
  bool have = false;
  for (int a = 0; a < 3; ++a) {
    if (ec[a] & 1) continue;
    for (int s = -1; s <= 1; s += 2) {
      int t[3] = {ec[0], ec[1], ec[2]};
      t[a] += s;
      if (t[a] < 0 || t[a] >= d.K[a]) continue;
      const uint64_t k = cell_key(R, 2, im, d, t);
      if (!have || k < bk) {
        have = true;
        bk = k;
        best[0] = t[0]; best[1] = t[1]; best[2] = t[2];
      }
    }
  }
  if (!have) return 0;
  const int n = sq_boundary(R, im, d, best, bnd);
  return bnd[n - 1] == ekey ? n : 0;
}

__device__ inline uint64_t arena_alloc(const RedCtx& R, uint32_t len) {
  const unsigned long long off = atomicAdd(R.arena_top, (unsigned long long)len);
  if (off + len > R.arena_cap) {
    raise_flag(R.st, &R.st->overflow, OVF_ARENA);
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

struct Work {
  uint64_t* fbuf[2];
  uint64_t* tbuf[2];
  uint64_t* F;
  uint32_t nf;
  const uint64_t* T;
  uint32_t nt;
  int tsel;  // which private tail buffer T is in, or -1
  unsigned long long adds, merged;
  uint32_t maxlen;
};

// T ^= B into fresh storage (the other private tail buffer, or the arena).
__device__ inline bool tail_add(const RedCtx& R, Work& W, const uint64_t* b, uint32_t nb) {
  const uint32_t need = W.nt + nb;
  uint64_t* out;
  int sel = -1;
  if (need <= PCAP) {
    sel = W.tsel == 0 ? 1 : 0;
    out = W.tbuf[sel];
  } else {
    const uint64_t off = arena_alloc(R, need);
    if (off == ~0ull) return false;
    out = R.arena + off;
  }
  W.nt = xor_lists(W.T, W.nt, b, nb, out);
  W.T = out;
  W.tsel = sel;
  W.merged += need;
  return true;
}

// W ^= B.  Returns false on arena exhaustion.
__device__ inline bool work_add(const RedCtx& R, Work& W, const uint64_t* b, uint32_t nb) {
  W.adds += 1;
  if (nb > FCAP) {
    if (!tail_add(R, W, b, nb)) return false;
  } else {
    uint64_t* out = (W.F == W.fbuf[0]) ? W.fbuf[1] : W.fbuf[0];
    W.merged += W.nf + nb;
    W.nf = xor_lists(W.F, W.nf, b, nb, out);
    W.F = out;
    if (W.nf > FCAP) {
      if (!tail_add(R, W, W.F, W.nf)) return false;
      W.nf = 0;
    }
  }
  if (W.nf + W.nt > W.maxlen) W.maxlen = W.nf + W.nt;
  return true;
}

// Cancels equal last entries of F and T; returns false if the column is zero.
__device__ inline bool work_pivot(Work& W, uint64_t* piv) {
  while (W.nf && W.nt && W.F[W.nf - 1] == W.T[W.nt - 1]) {
    --W.nf;
    --W.nt;
  }
  if (!W.nf && !W.nt) return false;
  if (!W.nf) *piv = W.T[W.nt - 1];
  else if (!W.nt) *piv = W.F[W.nf - 1];
  else *piv = W.F[W.nf - 1] > W.T[W.nt - 1] ? W.F[W.nf - 1] : W.T[W.nt - 1];
  return true;
}

// Writes F XOR T to the arena; afterwards the working column is that list.
__device__ inline uint64_t work_publish(const RedCtx& R, Work& W, uint32_t* len) {
  const uint32_t need = W.nf + W.nt;
  const uint64_t off = arena_alloc(R, need ? need : 1);
  if (off == ~0ull) return ~0ull;
  *len = xor_lists(W.F, W.nf, W.T, W.nt, R.arena + off);
  W.T = R.arena + off;
  W.nt = *len;
  W.tsel = -1;
  W.nf = 0;
  return off;
}

__device__ inline void work_load(Work& W, const RedCtx& R, uint64_t p) {
  W.T = R.arena + (p >> 24);
  W.nt = (uint32_t)(p & ((1u << 24) - 1));
  W.tsel = -1;
  W.nf = 0;
}

// One round of column c: reduce it against the columns done before this
// round, then store it and propose it as the owner of its pivot.
__device__ void reduce_round(const RedCtx& R, uint32_t c, bool first, uint64_t off2, Work& W) {
  if (first) {  // initial column: the boundary of the square
    const uint64_t k = R.skeys[off2 + c];
    const int im = skey_img(R.L, k);
    const ImgDesc d = R.imgs[im];
    int sc[3];
    kidx_coords(d, skey_kidx(R.L, k), sc);
    W.F = W.fbuf[0];
    W.nf = (uint32_t)sq_boundary(R, im, d, sc, W.F);
    W.T = W.tbuf[0];
    W.nt = 0;
    W.tsel = 0;
  } else {
    W.F = W.fbuf[0];
    work_load(W, R, R.col_ptr[c]);
  }
  for (uint32_t it = 0; it < RED_ITER_CAP; ++it) {
    if ((it & 63) == 63 && aborted(R.st)) return;
    uint64_t e;
    if (!work_pivot(W, &e)) {  // a zero column would be a birth of degree 2: those were cleared
      raise_flag(R.st, &R.st->internal);
      return;
    }
    const int im = skey_img(R.L, e);
    const ImgDesc d = R.imgs[im];
    int ec[3];
    kidx_coords(d, skey_kidx(R.L, e), ec);
    uint64_t bnd[4];
    const int na = apparent_bnd(R, im, d, ec, e, bnd);
    if (na > 0) {  // owner: the apparent partner, whose column is its raw boundary
      if (!work_add(R, W, bnd, (uint32_t)na)) return;
      continue;
    }
    const int64_t slot = edge_slot(d, ec);
    const int32_t o = R.owner[slot];
    if (o >= 0 && (uint32_t)o < c) {  // add the column of o
      const uint64_t p = R.col_ptr[o];
      if (!work_add(R, W, R.arena + (p >> 24), (uint32_t)(p & ((1u << 24) - 1)))) return;
      continue;
    }
    if ((uint32_t)o == c) {  // cannot happen: an active column owns nothing
      raise_flag(R.st, &R.st->internal);
      return;
    }
    // store the column and propose c as the owner of e
    uint32_t len = 0;
    const uint64_t off = work_publish(R, W, &len);
    if (off == ~0ull) return;
    if (len >= (1u << 24)) {
      raise_flag(R.st, &R.st->overflow, OVF_COLUMN);
      return;
    }
    R.col_ptr[c] = pack_col(off, len);
    R.piv[c] = e;
    atomicMin(&R.claim[slot], (int32_t)c);
    return;
  }
  raise_flag(R.st, &R.st->iter_cap);
}

// Round kernel.  Round 0 runs every column that is not cleared (list = all
// squares); later rounds run the columns in `list` (count in *n_list).
__global__ void k_fill_count(unsigned long long* c) { *c = 0; }

__global__ __launch_bounds__(256) void k_red_round(RedCtx R, const uint32_t* __restrict__ list,
                                                   const unsigned long long* __restrict__ n_list, int first) {
  if (aborted(R.st)) return;
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  const uint64_t n = first ? R.dim_count[2] : *n_list;
  if (n == 0) return;
  const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  Work W;
  uint64_t* base = R.pbuf + gtid * PBUF_PER_THREAD;
  W.fbuf[0] = base;
  W.fbuf[1] = base + FBUF;
  W.tbuf[0] = base + 2 * FBUF;
  W.tbuf[1] = base + 2 * FBUF + PCAP;
  W.adds = 0;
  W.merged = 0;
  W.maxlen = 0;
  for (uint64_t i = gtid; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    if (aborted(R.st)) break;
    const uint32_t c = first ? (uint32_t)i : list[i];
    if (first && R.cleared[c]) continue;
    reduce_round(R, c, first != 0, off2, W);
  }
  if (W.adds) {
    atomicAdd(&R.st->adds, W.adds);
    atomicAdd(&R.st->merged, W.merged);
    atomicMax(&R.st->max_col, W.maxlen);
  }
}

__device__ inline int64_t pivot_slot(const RedCtx& R, uint64_t e) {
  const ImgDesc d = R.imgs[skey_img(R.L, e)];
  int ec[3];
  kidx_coords(d, skey_kidx(R.L, e), ec);
  return edge_slot(d, ec);
}

__device__ inline void push_list(uint32_t* list, unsigned long long* n, uint32_t c) {
  const unsigned long long at = atomicAdd(n, 1ull);
  list[at] = c;
}

// Commit: the leftmost proposer of each pivot becomes its owner; losers and
// displaced owners form the next round's list.
__global__ void k_red_commit(RedCtx R, const uint32_t* __restrict__ list, const unsigned long long* __restrict__ n_list,
                             int first, uint32_t* __restrict__ next, unsigned long long* __restrict__ n_next) {
  if (aborted(R.st)) return;
  const uint64_t n = first ? R.dim_count[2] : *n_list;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t c = first ? (uint32_t)i : list[i];
    if (first && R.cleared[c]) continue;
    const int64_t slot = pivot_slot(R, R.piv[c]);
    if (R.claim[slot] == (int32_t)c) {
      const int32_t old = R.owner[slot];
      R.owner[slot] = (int32_t)c;
      if (old >= 0) push_list(next, n_next, (uint32_t)old);
    } else {
      push_list(next, n_next, c);
    }
  }
}

// Clears the proposals of the round that was just committed.
__global__ void k_red_reset(RedCtx R, const uint32_t* __restrict__ list, const unsigned long long* __restrict__ n_list,
                            int first) {
  if (aborted(R.st)) return;
  const uint64_t n = first ? R.dim_count[2] : *n_list;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t c = first ? (uint32_t)i : list[i];
    if (first && R.cleared[c]) continue;
    R.claim[pivot_slot(R, R.piv[c])] = 0x7FFFFFFF;
  }
}

// Degree-1 rows of a volume: column c pairs its final pivot edge (birth) with
// its square (death).
__global__ void k_h1_emit(RedCtx R, EmitCtx E) {
  if (aborted(R.st)) return;
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  const uint64_t n2 = R.dim_count[2];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t nr = (n2 + 63) & ~63ull;
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < nr; c += stride) {
    bool active = false;
    int im = 0;
    uint64_t ck = 0;
    if (c < n2 && !R.cleared[c]) {
      const uint64_t e = R.piv[c];
      const ImgDesc d = R.imgs[skey_img(R.L, e)];
      int ec[3];
      kidx_coords(d, skey_kidx(R.L, e), ec);
      if (R.owner[edge_slot(d, ec)] != (int32_t)c) raise_flag(R.st, &R.st->internal);
      else active = pair_row(E, e, R.skeys[off2 + c], false, &im, &ck);
    }
    emit_rows(E, active, im, ck);
  }
}

RedCtx make_redctx(const float* img, const ImgDesc* imgs, Layout L, const uint64_t* skeys,
                   const unsigned long long* dim_count, const uint8_t* cleared, int32_t* owner, int32_t* claim,
                   uint64_t* piv, uint64_t* col_ptr, uint64_t* arena, uint64_t arena_cap,
                   unsigned long long* arena_top, uint64_t* pbuf, Status* st) {
  RedCtx R;
  R.img = img;
  R.imgs = imgs;
  R.L = L;
  R.skeys = skeys;
  R.dim_count = dim_count;
  R.cleared = cleared;
  R.owner = owner;
  R.claim = claim;
  R.piv = piv;
  R.col_ptr = col_ptr;
  R.arena = arena;
  R.arena_cap = arena_cap;
  R.arena_top = arena_top;
  R.pbuf = pbuf;
  R.st = st;
  return R;
}

void launch_h1_rounds(int grid, const RedCtx& R, uint32_t* lists[2], unsigned long long* counts, int round0,
                      int nrounds, hipStream_t s) {
  for (int r = round0; r < round0 + nrounds; ++r) {
    const int cur = r & 1, nxt = (r + 1) & 1;
    const int first = r == 0;
    k_fill_count<<<1, 1, 0, s>>>(counts + nxt);
    k_red_round<<<grid, 256, 0, s>>>(R, lists[cur], counts + cur, first);
    k_red_commit<<<grid, 256, 0, s>>>(R, lists[cur], counts + cur, first, lists[nxt], counts + nxt);
    k_red_reset<<<grid, 256, 0, s>>>(R, lists[cur], counts + cur, first);
  }
}

void launch_h1_emit(int grid, const RedCtx& R, const EmitCtx& E, hipStream_t s) {
  k_h1_emit<<<grid, 256, 0, s>>>(R, E);
}

}  // namespace cr
