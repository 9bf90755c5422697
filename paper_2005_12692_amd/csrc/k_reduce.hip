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
// latest facet of s, as recorded by the stencil pass -- writes the boundary of
// s into bnd and returns its length; returns 0 otherwise.
__device__ inline int apparent_bnd(const RedCtx& R, int im, const ImgDesc& d, const int ec[3], uint64_t ekey,
                                   uint64_t bnd[4]) {
  (void)ekey;
  const uint8_t code = R.eapp[edge_slot(d, ec)];
  if (code == 0xFF) return 0;
  int t[3] = {ec[0], ec[1], ec[2]};
  t[code >> 1] += (code & 1) ? 1 : -1;
  return sq_boundary(R, im, d, t, bnd);
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

constexpr uint64_t YIELDED = ~0ull;      // piv[c] of a column that stored its state without proposing

__device__ inline void push_list(uint32_t* list, unsigned long long* n, uint32_t c) {
  const unsigned long long at = atomicAdd(n, 1ull);
  list[at] = c;
}

// Wave-aggregated append of c for every active lane (all lanes must call it).
__device__ inline void wave_push(uint32_t* list, unsigned long long* n, bool active, uint32_t c) {
  const uint64_t mask = __ballot(active);
  if (!mask) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(n, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (active) {
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    list[base + __popcll(mask & lt)] = c;
  }
}

// Stores W as column c and proposes c as the owner of e (or yields if e == YIELDED).
__device__ inline bool store_and_propose(const RedCtx& R, Work& W, uint32_t c, uint64_t e, int64_t slot) {
  uint32_t len = 0;
  const uint64_t off = work_publish(R, W, &len);
  if (off == ~0ull) return false;
  if (len >= (1u << 24)) {
    raise_flag(R.st, &R.st->overflow, OVF_COLUMN);
    return false;
  }
  R.col_ptr[c] = pack_col(off, len);
  R.piv[c] = e;
  if (e != YIELDED) atomicMin(&R.claim[slot], (int32_t)c);
  return true;
}

// One round of column c in thread mode: reduce it against the columns done
// before this round, then store it and propose it as the owner of its pivot.
// A column whose tail grows past R.long_len keys, or that needs more than
// R.yield_iters additions, stores its state and moves to the block-mode list
// (a single thread merges long lists at one memory latency per key).
__device__ void reduce_round(const RedCtx& R, uint32_t c, bool first, uint64_t off2, Work& W,
                             uint32_t* long_next, unsigned long long* n_long_next) {
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
    if (it >= R.yield_iters || W.nt > R.long_len) {
      if (store_and_propose(R, W, c, YIELDED, 0)) push_list(long_next, n_long_next, c);
      return;
    }
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
    store_and_propose(R, W, c, e, slot);
    return;
  }
  raise_flag(R.st, &R.st->iter_cap);
}

__global__ void k_fill_count(unsigned long long* c) {
  c[0] = 0;
  c[1] = 0;
}

// Thread-mode round.  Round 0 runs every column that is not cleared; later
// rounds run the short-column list.
__global__ __launch_bounds__(256) void k_red_round(RedCtx R, const uint32_t* __restrict__ list,
                                                   const unsigned long long* __restrict__ n_list, int first,
                                                   uint32_t* __restrict__ long_next,
                                                   unsigned long long* __restrict__ n_long_next) {
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
    reduce_round(R, c, first != 0, off2, W, long_next, n_long_next);
  }
  if (W.adds) {
    atomicAdd(&R.st->adds, W.adds);
    atomicAdd(&R.st->merged, W.merged);
    atomicMax(&R.st->max_col, W.maxlen);
  }
}

// ---- block mode: one workgroup per long column ---------------------------------
//
// The front list F lives in LDS (two buffers of FB_CAP keys); the tail T is a
// sorted list in global memory.  Small additions are merged into F by rank
// computations in LDS (every thread places some elements); F is merged into T
// when it passes FB_LIM, and long addends are merged into T directly, by a
// tiled merge: tiles of both inputs are staged in LDS with coalesced loads,
// merged by ranks, equal pairs cancelled, and the survivors written out with a
// block-wide scan.
constexpr int BT = 256;
constexpr uint32_t FB_CAP = 7168;
constexpr uint32_t FB_LIM = FB_CAP - 2048;  // room for an addend of up to STAGE keys
constexpr uint32_t STAGE = 2048;            // longest addend merged in LDS
constexpr int TILE = 256;
constexpr int BLOCK_GRID = 512;          // workgroups of the block-mode round

struct BlockLds {
  uint64_t F[2][FB_CAP];
  uint64_t stage[STAGE];
  uint32_t pref[STAGE + 1];
  uint64_t tA[TILE + 1], tB[TILE + 1];
  uint64_t tM[2 * TILE + 2];
  uint32_t keep[2 * TILE + 2];
  uint32_t part[BT + 1];
  uint64_t bnd[4];
  uint64_t e, tlast;
  unsigned long long off;
  int64_t slot;
  int32_t o;
  uint32_t nf, cur, nt, n_out, ka, kb, act, na;
  const uint64_t* T;
  unsigned long long adds, merged;
};

// Exclusive scan of one value per thread across the workgroup (wave shuffles,
// then the four wave totals); returns the prefix and writes the total.
__device__ inline uint32_t blk_excl(uint32_t v, uint32_t* part, uint32_t* total) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t up = __shfl_up(incl, off, 64);
    if (lane >= (uint32_t)off) incl += up;
  }
  if (lane == 63) part[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (uint32_t w = 0; w < BT / 64; ++w) {
    const uint32_t x = part[w];
    if (w < wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// Exclusive scan of flags[0..n) into out[0..n] (out[n] = total); returns the total.
__device__ inline uint32_t blk_scan(const uint32_t* flags, uint32_t n, uint32_t* out, uint32_t* part) {
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (n + BT - 1) / BT;
  const uint32_t lo = tid * per < n ? tid * per : n, hi = lo + per < n ? lo + per : n;
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += flags[i];
  uint32_t total;
  uint32_t run = blk_excl(s, part, &total);
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = flags[i];
    out[i] = run;
    run += v;
  }
  if (tid == 0) out[n] = total;
  __syncthreads();
  return total;
}

__device__ inline uint32_t lower_bound_lds(const uint64_t* a, uint32_t n, uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if (a[m] < v) lo = m + 1;
    else hi = m;
  }
  return lo;
}
__device__ inline uint32_t upper_bound_lds(const uint64_t* a, uint32_t n, uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if (a[m] <= v) lo = m + 1;
    else hi = m;
  }
  return lo;
}

// out = A XOR B, with A and B sorted lists in LDS (|B| <= STAGE); out in LDS.
// Returns the length.  Uses S.pref for the cancellation prefix over B.
__device__ uint32_t blk_xor_lds(BlockLds& S, const uint64_t* A, uint32_t na, const uint64_t* B, uint32_t nb,
                                uint64_t* out) {
  const uint32_t tid = threadIdx.x;
  // flags over B: B[j] also in A (these values cancel)
  for (uint32_t j = tid; j < nb; j += BT) {
    const uint32_t q = lower_bound_lds(A, na, B[j]);
    S.pref[j] = (q < na && A[q] == B[j]) ? 1u : 0u;
  }
  __syncthreads();
  // exclusive prefix of the cancel flags, in place (pref[j] = # cancels in B[0:j])
  {
    const uint32_t per = (nb + BT - 1) / BT;
    const uint32_t lo = tid * per < nb ? tid * per : nb, hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += S.pref[i];
    uint32_t total;
    uint32_t run = blk_excl(s, S.part, &total);
    for (uint32_t i = lo; i < hi; ++i) {
      const uint32_t v = S.pref[i];
      S.pref[i] = run;
      run += v;
    }
    if (tid == 0) S.pref[nb] = total;
    __syncthreads();
  }
  const uint32_t ncancel = S.pref[nb];
  for (uint32_t i = tid; i < na; i += BT) {
    const uint64_t v = A[i];
    const uint32_t r = lower_bound_lds(B, nb, v);
    if (r < nb && B[r] == v) continue;  // cancelled
    out[i + r - 2 * S.pref[r]] = v;
  }
  for (uint32_t j = tid; j < nb; j += BT) {
    const uint64_t v = B[j];
    const uint32_t q = lower_bound_lds(A, na, v);
    if (q < na && A[q] == v) continue;
    out[j + q - 2 * S.pref[j]] = v;
  }
  __syncthreads();
  return na + nb - 2 * ncancel;
}

// out = A XOR B for sorted lists anywhere (global or LDS); out in global
// memory.  Tiled merge in key order; returns the length.
__device__ uint32_t blk_xor_tiled(BlockLds& S, const uint64_t* A, uint32_t na, const uint64_t* B, uint32_t nb,
                                  uint64_t* out) {
  const uint32_t tid = threadIdx.x;
  const uint64_t INF = ~0ull;
  uint32_t ia = 0, ib = 0, o = 0;
  while (ia < na || ib < nb) {
    const uint32_t la = na - ia < (uint32_t)TILE ? na - ia : TILE;
    const uint32_t lb = nb - ib < (uint32_t)TILE ? nb - ib : TILE;
    S.tA[tid] = tid < la ? A[ia + tid] : INF;
    S.tB[tid] = tid < lb ? B[ib + tid] : INF;
    if (tid == 0) {
      S.tA[TILE] = INF;
      S.tB[TILE] = INF;
    }
    __syncthreads();
    if (tid == 0) {
      // the next d outputs of the merge come from tA[0:ka] and tB[0:kb]
      uint32_t d = la + lb < (uint32_t)TILE ? la + lb : TILE;
      uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
      while (lo < hi) {  // smallest ka with tA[ka] >= tB[d - ka - 1]
        const uint32_t ka = (lo + hi) >> 1;
        if (S.tA[ka] < S.tB[d - ka - 1]) lo = ka + 1;
        else hi = ka;
      }
      uint32_t ka = lo, kb = d - lo;
      // keep an equal pair in one tile
      if (ka < la && kb > 0 && S.tA[ka] == S.tB[kb - 1]) ++ka;
      else if (kb < lb && ka > 0 && S.tB[kb] == S.tA[ka - 1]) ++kb;
      S.ka = ka;
      S.kb = kb;
    }
    __syncthreads();
    const uint32_t ka = S.ka, kb = S.kb, m = ka + kb;
    if (tid < ka) S.tM[tid + lower_bound_lds(S.tB, kb, S.tA[tid])] = S.tA[tid];
    if (tid < kb) S.tM[tid + upper_bound_lds(S.tA, ka, S.tB[tid])] = S.tB[tid];
    if (tid + BT < ka) S.tM[tid + BT + lower_bound_lds(S.tB, kb, S.tA[tid + BT])] = S.tA[tid + BT];
    if (tid + BT < kb) S.tM[tid + BT + upper_bound_lds(S.tA, ka, S.tB[tid + BT])] = S.tB[tid + BT];
    __syncthreads();
    for (uint32_t p = tid; p < m; p += BT) {
      const uint64_t v = S.tM[p];
      const bool dup = (p > 0 && S.tM[p - 1] == v) || (p + 1 < m && S.tM[p + 1] == v);
      S.keep[p] = dup ? 0u : 1u;
    }
    __syncthreads();
    uint32_t* pos = S.pref;  // reuse as scan output (m + 1 <= STAGE)
    const uint32_t kept = blk_scan(S.keep, m, pos, S.part);
    for (uint32_t p = tid; p < m; p += BT)
      if (S.keep[p]) out[o + pos[p]] = S.tM[p];
    o += kept;
    ia += ka;
    ib += kb;
    __syncthreads();
  }
  return o;
}

// Allocates n arena entries for the block (thread 0) and broadcasts the offset.
__device__ inline uint64_t blk_alloc(const RedCtx& R, BlockLds& S, uint32_t n) {
  if (threadIdx.x == 0) {
    const unsigned long long off = atomicAdd(R.arena_top, (unsigned long long)(n ? n : 1));
    if (off + n > R.arena_cap) {
      raise_flag(R.st, &R.st->overflow, OVF_ARENA);
      S.off = ~0ull;
    } else {
      S.off = off;
    }
  }
  __syncthreads();
  return S.off;
}

// T = T XOR src (any memory), into the arena.  Returns false on exhaustion.
__device__ inline bool blk_tail_add(const RedCtx& R, BlockLds& S, const uint64_t* src, uint32_t n) {
  const uint64_t off = blk_alloc(R, S, S.nt + n);
  if (off == ~0ull) return false;
  const uint32_t len = blk_xor_tiled(S, S.T, S.nt, src, n, R.arena + off);
  if (threadIdx.x == 0) {
    S.T = R.arena + off;
    S.nt = len;
    S.merged += len + n;
  }
  __syncthreads();
  return true;
}

// F = F XOR B (B in LDS, |B| <= STAGE); flushes F into T past FB_LIM.
__device__ inline bool blk_front_add(const RedCtx& R, BlockLds& S, const uint64_t* B, uint32_t nb) {
  const uint32_t cur = S.cur;
  const uint32_t n = blk_xor_lds(S, S.F[cur], S.nf, B, nb, S.F[cur ^ 1]);
  if (threadIdx.x == 0) {
    S.cur = cur ^ 1;
    S.nf = n;
    S.merged += n + nb;
  }
  __syncthreads();
  if (S.nf > FB_LIM) {
    if (!blk_tail_add(R, S, S.F[S.cur], S.nf)) return false;
    if (threadIdx.x == 0) S.nf = 0;
    __syncthreads();
  }
  return true;
}

static_assert(sizeof(BlockLds) <= 160 * 1024, "block-mode LDS exceeds the workgroup limit");

enum { ACT_APP = 1, ACT_OWNER = 2, ACT_PROPOSE = 3, ACT_STOP = 4 };

__global__ __launch_bounds__(BT) void k_red_round_block(RedCtx R, const uint32_t* __restrict__ list,
                                                        const unsigned long long* __restrict__ n_list) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  BlockLds& S = *reinterpret_cast<BlockLds*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  // every exit decision is taken by thread 0 and broadcast, so all threads of
  // the workgroup reach the same barriers
  if (tid == 0) {
    S.adds = 0;
    S.merged = 0;
    S.act = aborted(R.st) ? ACT_STOP : 0;
  }
  __syncthreads();
  if (S.act == ACT_STOP) return;
  const uint64_t n = *n_list;
  for (uint64_t li = blockIdx.x; li < n; li += gridDim.x) {
    const uint32_t c = list[li];
    // load the stored column: into F if it fits, else as the tail
    const uint64_t p = R.col_ptr[c];
    const uint32_t len = (uint32_t)(p & ((1u << 24) - 1));
    const uint64_t* src = R.arena + (p >> 24);
    if (len <= FB_LIM) {
      for (uint32_t i = tid; i < len; i += BT) S.F[0][i] = src[i];
      if (tid == 0) {
        S.nf = len;
        S.nt = 0;
        S.T = src;
      }
    } else if (tid == 0) {
      S.nf = 0;
      S.T = src;
      S.nt = len;
    }
    if (tid == 0) S.cur = 0;
    __syncthreads();
    bool ok = true;
    for (uint32_t it = 0; ok; ++it) {
      if (tid == 0) {
        uint32_t act = ACT_STOP;
        if (it >= RED_ITER_CAP) {
          raise_flag(R.st, &R.st->iter_cap);
        } else if (!aborted(R.st)) {
          // pivot: cancel equal last entries of F and T
          const uint64_t* F = S.F[S.cur];
          uint32_t nf = S.nf, nt = S.nt;
          while (nf && nt && F[nf - 1] == S.T[nt - 1]) {
            --nf;
            --nt;
          }
          S.nf = nf;
          S.nt = nt;
          if (!nf && !nt) {
            raise_flag(R.st, &R.st->internal);
          } else {
            uint64_t e;
            if (!nf) e = S.T[nt - 1];
            else if (!nt) e = F[nf - 1];
            else e = F[nf - 1] > S.T[nt - 1] ? F[nf - 1] : S.T[nt - 1];
            S.e = e;
            const int im = skey_img(R.L, e);
            const ImgDesc d = R.imgs[im];
            int ec[3];
            kidx_coords(d, skey_kidx(R.L, e), ec);
            const int na = apparent_bnd(R, im, d, ec, e, S.bnd);
            if (na > 0) {
              S.na = (uint32_t)na;
              act = ACT_APP;
            } else {
              const int64_t slot = edge_slot(d, ec);
              const int32_t o = R.owner[slot];
              S.slot = slot;
              S.o = o;
              if (o >= 0 && (uint32_t)o < c) act = ACT_OWNER;
              else if ((uint32_t)o == c) raise_flag(R.st, &R.st->internal);
              else act = ACT_PROPOSE;
            }
          }
        }
        S.act = act;
        if (act == ACT_APP || act == ACT_OWNER) S.adds += 1;
      }
      __syncthreads();
      const uint32_t act = S.act;
      if (act == ACT_STOP) {
        ok = false;
      } else if (act == ACT_APP) {
        ok = blk_front_add(R, S, S.bnd, S.na);
      } else if (act == ACT_OWNER) {
        const uint64_t q = R.col_ptr[S.o];
        const uint32_t ql = (uint32_t)(q & ((1u << 24) - 1));
        const uint64_t* qs = R.arena + (q >> 24);
        if (ql <= STAGE) {
          for (uint32_t i = tid; i < ql; i += BT) S.stage[i] = qs[i];
          __syncthreads();
          ok = blk_front_add(R, S, S.stage, ql);
        } else {
          ok = blk_tail_add(R, S, qs, ql);
        }
      } else {  // ACT_PROPOSE: store F XOR T and propose c for e
        const uint64_t off = blk_alloc(R, S, S.nf + S.nt);
        if (off != ~0ull) {
          const uint32_t l = blk_xor_tiled(S, S.F[S.cur], S.nf, S.T, S.nt, R.arena + off);
          if (tid == 0) {
            if (l >= (1u << 24)) {
              raise_flag(R.st, &R.st->overflow, OVF_COLUMN);
            } else {
              R.col_ptr[c] = pack_col(off, l);
              R.piv[c] = S.e;
              atomicMin(&R.claim[S.slot], (int32_t)c);
            }
          }
        }
        ok = false;
      }
      __syncthreads();
    }
  }
  if (tid == 0 && S.adds) {
    atomicAdd(&R.st->adds, S.adds);
    atomicAdd(&R.st->merged, S.merged);
  }
}

__device__ inline int64_t pivot_slot(const RedCtx& R, uint64_t e) {
  const ImgDesc d = R.imgs[skey_img(R.L, e)];
  int ec[3];
  kidx_coords(d, skey_kidx(R.L, e), ec);
  return edge_slot(d, ec);
}

// Commit: the leftmost proposer of each pivot becomes its owner; losers and
// displaced owners go to the next round's lists (long stored columns to the
// block-mode list).  Yielded columns were already listed.
__global__ void k_red_commit(RedCtx R, const uint32_t* __restrict__ list_t, const unsigned long long* __restrict__ n_t,
                             const uint32_t* __restrict__ list_b, const unsigned long long* __restrict__ n_b,
                             int first, uint32_t* next_t, uint32_t* next_b, unsigned long long* __restrict__ n_next) {
  if (aborted(R.st)) return;
  const uint64_t nt = first ? R.dim_count[2] : *n_t;
  const uint64_t nb = first ? 0 : *n_b;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t nr = (nt + nb + 63) & ~63ull;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nr; i += stride) {
    bool again_short = false, again_long = false;
    uint32_t again = 0;
    if (i < nt + nb) {
      uint32_t c;
      bool skip = false;
      if (i < nt) {
        c = first ? (uint32_t)i : list_t[i];
        skip = first && R.cleared[c];
      } else {
        c = list_b[i - nt];
      }
      const uint64_t e = skip ? YIELDED : R.piv[c];
      if (e != YIELDED) {
        const int64_t slot = pivot_slot(R, e);
        bool push = true;
        if (R.claim[slot] == (int32_t)c) {
          const int32_t old = R.owner[slot];
          R.owner[slot] = (int32_t)c;
          push = old >= 0;
          again = (uint32_t)old;
        } else {
          again = c;
        }
        if (push) {
          const bool lng = (uint32_t)(R.col_ptr[again] & ((1u << 24) - 1)) > R.long_len;
          again_long = lng;
          again_short = !lng;
        }
      }
    }
    wave_push(next_t, n_next, again_short, again);
    wave_push(next_b, n_next + 1, again_long, again);
  }
}

// Clears the proposals of the round that was just committed.
__global__ void k_red_reset(RedCtx R, const uint32_t* __restrict__ list_t, const unsigned long long* __restrict__ n_t,
                            const uint32_t* __restrict__ list_b, const unsigned long long* __restrict__ n_b,
                            int first) {
  if (aborted(R.st)) return;
  const uint64_t nt = first ? R.dim_count[2] : *n_t;
  const uint64_t nb = first ? 0 : *n_b;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nt + nb; i += stride) {
    uint32_t c;
    if (i < nt) {
      c = first ? (uint32_t)i : list_t[i];
      if (first && R.cleared[c]) continue;
    } else {
      c = list_b[i - nt];
    }
    const uint64_t e = R.piv[c];
    if (e != YIELDED) R.claim[pivot_slot(R, e)] = 0x7FFFFFFF;
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
                   const unsigned long long* dim_count, const uint8_t* cleared, const uint8_t* eapp,
                   int32_t* owner, int32_t* claim,
                   uint64_t* piv, uint64_t* col_ptr, uint64_t* arena, uint64_t arena_cap,
                   unsigned long long* arena_top, uint64_t* pbuf, Status* st) {
  RedCtx R;
  R.img = img;
  R.imgs = imgs;
  R.L = L;
  R.skeys = skeys;
  R.dim_count = dim_count;
  R.cleared = cleared;
  R.eapp = eapp;
  R.owner = owner;
  R.claim = claim;
  R.piv = piv;
  R.col_ptr = col_ptr;
  R.arena = arena;
  R.arena_cap = arena_cap;
  R.arena_top = arena_top;
  R.pbuf = pbuf;
  R.st = st;
  R.long_len = 128;
  R.yield_iters = 32;
  return R;
}

void launch_h1_rounds(int grid, const RedCtx& R, uint32_t* lists[4], unsigned long long* counts, int round0,
                      int nrounds, hipStream_t s) {
  static bool lds_set = false;
  if (!lds_set) {
    (void)hipFuncSetAttribute((const void*)k_red_round_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(BlockLds));
    lds_set = true;
  }
  for (int r = round0; r < round0 + nrounds; ++r) {
    const int cur = r & 1, nxt = (r + 1) & 1;
    const int first = r == 0;
    // lists[2*k + 0] short (thread mode), lists[2*k + 1] long (block mode); counts likewise
    uint32_t* lt = lists[2 * cur];
    uint32_t* lb = lists[2 * cur + 1];
    unsigned long long* ct = counts + 2 * cur;
    unsigned long long* cnx = counts + 2 * nxt;
    k_fill_count<<<1, 1, 0, s>>>(cnx);
    k_red_round<<<grid, 256, 0, s>>>(R, lt, ct, first, lists[2 * nxt + 1], cnx + 1);
    if (!first) k_red_round_block<<<BLOCK_GRID, BT, sizeof(BlockLds), s>>>(R, lb, ct + 1);
    k_red_commit<<<grid, 256, 0, s>>>(R, lt, ct, lb, ct + 1, first, lists[2 * nxt], lists[2 * nxt + 1], cnx);
    k_red_reset<<<grid, 256, 0, s>>>(R, lt, ct, lb, ct + 1, first);
  }
}

void launch_h1_emit(int grid, const RedCtx& R, const EmitCtx& E, hipStream_t s) {
  k_h1_emit<<<grid, 256, 0, s>>>(R, E);
}

}  // namespace cr
