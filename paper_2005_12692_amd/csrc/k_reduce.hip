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
// reduction.  Once few columns are left, the asynchronous tail (below) reduces
// them to the end without rounds, claiming pivots by compare-and-swap.
//
// Short columns are reduced one per thread; a column that grows long, or needs
// many additions, continues in wave mode (one wavefront per column).  Stored
// columns live in an append-only arena as a length word followed by the keys.
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
// The byte of an edge in the stencil's partner codes: four per anchor pixel.
__device__ inline int64_t eapp_slot(const ImgDesc& d, const int c[3]) {
  const int axis = (c[0] & 1) ? 0 : ((c[1] & 1) ? 1 : 2);
  return 4 * anchor_pixel(d, c) + axis;
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
__device__ inline int apparent_bnd(const RedCtx& R, int im, const ImgDesc& d, const int ec[3], uint64_t bnd[4]) {
  const uint8_t code = R.eapp[eapp_slot(d, ec)];
  if (code == 0xFF) return 0;
  int t[3] = {ec[0], ec[1], ec[2]};
  t[code >> 1] += (code & 1) ? 1 : -1;
  return sq_boundary(R, im, d, t, bnd);
}

__device__ inline uint64_t arena_alloc(const RedCtx& R, uint64_t len) {
  const unsigned long long off = atomicAdd(R.arena_top, (unsigned long long)len);
  if (off + len > R.arena_cap) {
    raise_flag(R.st, &R.st->overflow, OVF_ARENA);
    return ~0ull;
  }
  return off;
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

template <typename T>
__device__ __forceinline__ T sel3(int i, T a, T b, T c) { return i == 0 ? a : (i == 1 ? b : c); }

// x / d for x < 2^30 and 1 <= d < 2^22, with rd = 1.0 / d: the product in
// double precision is within 2^-22 of x / d, so its integer part is the
// quotient or one below it (only when x / d is an integer); one remainder
// check corrects that.  Cheaper than a 32-bit integer division.
__device__ __forceinline__ uint32_t udiv_rcp(uint32_t x, uint32_t d, double rd) {
  uint32_t q = (uint32_t)((double)x * rd);
  if (x - q * d >= d) ++q;
  return q;
}

__device__ __forceinline__ uint32_t ord_of(float v) {
  uint32_t bits;
  __builtin_memcpy(&bits, &v, 4);
  return ord32_bits(bits);
}
__device__ __forceinline__ float pix_val(const float* img, int64_t p) {
  const float v = img[p];
  return (v != v) ? INFINITY : canon(v);
}

// ---- thread mode: one thread per column, the column in registers -----------------
//
// A column of at most TC keys is kept sorted in descending order in registers
// (w[0] is the pivot).  XOR-inserting a key compares it with every slot and
// shifts by selects, so nothing is indexed dynamically.  A column that would
// grow past TC keys, or needs more than yield_iters additions in one round, is
// stored and continues in wave mode -- except that in the first round, which
// runs with a smaller TC, a column that outgrows it continues in thread mode.
template <int TC>
struct RegCol {
  uint64_t w[TC];
  uint32_t n;
};

template <int TC>
__device__ __forceinline__ void rc_pop(RegCol<TC>& C) {
#pragma unroll
  for (int i = 0; i + 1 < TC; ++i) C.w[i] = C.w[i + 1];
  C.w[TC - 1] = 0;
  --C.n;
}

// C ^= {k}; when k is absent the column must have a free slot.  Empty slots
// hold 0, below every key, so they need no bounds test.
template <int TC>
__device__ __forceinline__ void rc_xor(RegCol<TC>& C, uint64_t k) {
  bool eq = false;
#pragma unroll
  for (int i = 0; i < TC; ++i) eq = eq || C.w[i] == k;
  // one pass, in place, from the top: slot i keeps its key while that is above
  // k; below, it takes the next key (k removed), or k at the first such slot
  // and the previous key after it (k inserted)
  uint64_t prev = 0;
  bool prev_above = true;
#pragma unroll
  for (int i = 0; i < TC; ++i) {
    const uint64_t cur = C.w[i];
    const uint64_t next = i + 1 < TC ? C.w[i + 1 < TC ? i + 1 : i] : 0ull;
    const bool above = cur > k;
    C.w[i] = above ? cur : (eq ? next : (prev_above ? k : prev));
    prev = cur;
    prev_above = above;
  }
  C.n = eq ? C.n - 1 : C.n + 1;
}

// Writes the column to the arena as a stored list (ascending); returns its offset.
template <int TC>
__device__ __forceinline__ uint64_t rc_store(const RedCtx& R, const RegCol<TC>& C) {
  const uint64_t off = arena_alloc(R, (uint64_t)C.n + 1);
  if (off == ~0ull) return off;
  R.arena[off] = C.n;
#pragma unroll
  for (int i = 0; i < TC; ++i)
    if ((uint32_t)i < C.n) R.arena[off + C.n - i] = C.w[i];
  return off;
}

constexpr int THREAD_CAP_FIRST = 16;  // keys of a thread-mode column in the first round
constexpr int THREAD_CAP = 32;        // ... in later rounds

template <int TC>
__device__ void reduce_round_reg(const RedCtx& R, uint32_t c, bool first, uint64_t off2, uint32_t* short_next,
                                 unsigned long long* n_short_next, uint32_t* long_next,
                                 unsigned long long* n_long_next, unsigned long long* adds) {
  const uint64_t sq = R.skeys[off2 + c];
  const int im = skey_img(R.L, sq);
  const ImgDesc d = R.imgs[im];
  const uint32_t K1 = (uint32_t)d.K[1], K2 = (uint32_t)d.K[2];
  const int64_t ps0 = (int64_t)d.n[1] * d.n[2], ps1 = d.n[2];
  const uint32_t ks0 = K1 * K2, ks1 = K2;
  const double rK1 = 1.0 / (double)K1, rK2 = 1.0 / (double)K2;
  RegCol<TC> C;
#pragma unroll
  for (int i = 0; i < TC; ++i) C.w[i] = 0;
  if (first) {  // the boundary of the square: its four edges, from its four vertices
    const uint32_t sk = skey_kidx(R.L, sq);
    const uint32_t sx = sk % K2, st1 = sk / K2;
    const uint32_t sy = st1 % K1, sz = st1 / K1;
    const int a0 = (sz & 1) ? 0 : 1;                 // the two odd axes a0 < a1 of the square
    const int a1 = (sx & 1) ? 2 : 1;
    const int64_t p00 = pixel_index(d, (int)(sz >> 1), (int)(sy >> 1), (int)(sx >> 1));
    const int64_t pa = sel3(a0, ps0, ps1, (int64_t)1), pb = sel3(a1, ps0, ps1, (int64_t)1);
    const uint32_t ka = sel3(a0, ks0, ks1, 1u), kb = sel3(a1, ks0, ks1, 1u);
    const float f00 = pix_val(R.img, p00), f10 = pix_val(R.img, p00 + pa);
    const float f01 = pix_val(R.img, p00 + pb), f11 = pix_val(R.img, p00 + pa + pb);
    // edges along a1 at a0 = low / high, along a0 at a1 = low / high
    C.w[0] = make_skey(R.L, 1, im, ord_of(fmaxf(f00, f01)), sk - ka);
    C.w[1] = make_skey(R.L, 1, im, ord_of(fmaxf(f10, f11)), sk + ka);
    C.w[2] = make_skey(R.L, 1, im, ord_of(fmaxf(f00, f10)), sk - kb);
    C.w[3] = make_skey(R.L, 1, im, ord_of(fmaxf(f01, f11)), sk + kb);
    // descending sorting network on four keys
    auto cx = [](uint64_t& x, uint64_t& y) {
      const uint64_t hi = x > y ? x : y, lo = x > y ? y : x;
      x = hi;
      y = lo;
    };
    cx(C.w[0], C.w[1]);
    cx(C.w[2], C.w[3]);
    cx(C.w[0], C.w[2]);
    cx(C.w[1], C.w[3]);
    cx(C.w[1], C.w[2]);
    C.n = 4;
  } else {
    const uint64_t off = R.col_ptr[c];
    const uint32_t len = (uint32_t)R.arena[off];
    if (len > (uint32_t)TC) {  // too long for registers: straight to wave mode
      R.piv[c] = YIELDED;
      push_list(long_next, n_long_next, c);
      return;
    }
#pragma unroll
    for (int i = 0; i < TC; ++i)
      if ((uint32_t)i < len) C.w[i] = R.arena[off + len - i];
    C.n = len;
  }
  auto yield = [&](bool full) {  // full: the column outgrew TC
    const uint64_t off = rc_store(R, C);
    if (off == ~0ull) return;
    R.col_ptr[c] = off;
    R.piv[c] = YIELDED;
    if (full && TC < THREAD_CAP) push_list(short_next, n_short_next, c);
    else push_list(long_next, n_long_next, c);
  };
  for (uint32_t it = 0;; ++it) {
    if (it >= R.yield_iters) {
      yield(false);
      return;
    }
    if (C.n == 0) {  // a zero column would be a birth of degree 2: those were cleared
      raise_flag(R.st, &R.st->internal);
      return;
    }
    const uint64_t e = C.w[0];
    const uint32_t kidx = skey_kidx(R.L, e);
    const uint32_t t1 = udiv_rcp(kidx, K2, rK2), kx = kidx - t1 * K2;
    const uint32_t kz = udiv_rcp(t1, K1, rK1), ky = t1 - kz * K1;
    if ((e >> (R.L.ib + 32 + R.L.kb)) != 1 || skey_img(R.L, e) != im || kz >= (uint32_t)d.K[0] ||
        ((kz & 1) + (ky & 1) + (kx & 1)) != 1) {
      raise_flag(R.st, &R.st->internal);
      return;
    }
    const int ax = (kz & 1) ? 0 : ((ky & 1) ? 1 : 2);
    const int64_t anchor = pixel_index(d, (int)(kz >> 1), (int)(ky >> 1), (int)(kx >> 1));
    const int64_t slot = 3 * anchor + ax;
    const uint8_t code = R.eapp[4 * anchor + ax];
    const uint64_t ow = R.owner[slot];
    if (code != 0xFF) {  // the apparent partner s of e: its boundary is e and three older edges
      if (C.n + 2 > (uint32_t)TC) {
        yield(true);
        return;
      }
      const int bb = code >> 1;
      const int sg = (code & 1) ? 1 : -1;
      const int64_t pax = sel3(ax, ps0, ps1, (int64_t)1), pbb = sel3(bb, ps0, ps1, (int64_t)1);
      const float v0 = pix_val(R.img, anchor), v1 = pix_val(R.img, anchor + pax);
      const float w0 = pix_val(R.img, anchor + sg * pbb), w1 = pix_val(R.img, anchor + pax + sg * pbb);
      const uint32_t kax = sel3(ax, ks0, ks1, 1u);
      const uint32_t kb = (uint32_t)((int)sel3(bb, ks0, ks1, 1u) * sg);
      const uint64_t kw = make_skey(R.L, 1, im, ord_of(fmaxf(w0, w1)), kidx + 2 * kb);
      const uint64_t ka0 = make_skey(R.L, 1, im, ord_of(fmaxf(v0, w0)), kidx - kax + kb);
      const uint64_t ka1 = make_skey(R.L, 1, im, ord_of(fmaxf(v1, w1)), kidx + kax + kb);
      if (kw >= e || ka0 >= e || ka1 >= e) {  // e must be the latest facet of s
        raise_flag(R.st, &R.st->internal);
        return;
      }
      rc_pop(C);
      rc_xor(C, kw);
      rc_xor(C, ka0);
      rc_xor(C, ka1);
      *adds += 1;
      continue;
    }
    const int32_t o = ow == NO_OWNER ? -1 : (int32_t)(ow >> 32);
    if (o >= 0 && (uint32_t)o < c) {  // add the column of o; its top key is e
      const uint64_t* q = R.arena + (uint32_t)ow;
      const uint32_t m = (uint32_t)q[0] - 1;
      if (C.n - 1 + m > (uint32_t)TC) {
        yield(true);
        return;
      }
      rc_pop(C);
      for (uint32_t i0 = 0; i0 < m; i0 += 4) {  // four loads in flight, then four inserts
        uint64_t k[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) k[j] = i0 + j < m ? q[1 + i0 + j] : 0ull;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (i0 + j < m) rc_xor(C, k[j]);
      }
      *adds += 1;
      continue;
    }
    if ((uint32_t)o == c) {  // cannot happen: an active column owns nothing
      raise_flag(R.st, &R.st->internal);
      return;
    }
    const uint64_t off = rc_store(R, C);
    if (off == ~0ull) return;
    R.col_ptr[c] = off;
    R.piv[c] = e;
    atomicMax(reinterpret_cast<unsigned long long*>(&R.claim[slot]), claim_word(R.round, c));
    return;
  }
}

// Whether a key of the spatial order is a cleared column's.
__device__ __forceinline__ bool spatial_none(const RedCtx& R, uint64_t key) {
  return (key & 0xFFFFFFFFull) == (1ull << (R.L.ib + R.L.kb)) - 1;
}

// Whether a round's kernels leave its columns to the asynchronous tail: a
// round after the first with at most async_max columns (its commit records it
// in st->tail_round), and every round after that one.  ct: the round's counts.
__device__ __forceinline__ bool in_tail(const RedCtx& R, const unsigned long long* ct, int first) {
  if (first || R.async_max == 0) return false;
  if (R.st->tail_round) return true;
  const uint64_t n = ct[0] + ct[1];
  return n > 0 && n <= R.async_max;
}

// Thread-mode round.  Round 0 runs every column that is not cleared; later
// rounds run the short-column list unless it is short enough for wave mode.
template <int TC>
__global__ __launch_bounds__(256) void k_red_round(RedCtx R, const uint32_t* __restrict__ list,
                                                   const unsigned long long* __restrict__ n_list, int first,
                                                   uint32_t* __restrict__ short_next,
                                                   unsigned long long* __restrict__ n_short_next,
                                                   uint32_t* __restrict__ long_next,
                                                   unsigned long long* __restrict__ n_long_next) {
  if (aborted(R.st) || in_tail(R, n_list, first)) return;
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  // the first round takes the columns in the spatial order when it was built
  const uint64_t nsp = first && R.spatial ? *R.n_spatial : 0;
  const uint64_t n = first ? (nsp ? nsp : R.dim_count[2]) : *n_list;
  if (n == 0 || (!first && n <= R.wave_short)) return;
  unsigned long long adds = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    if (aborted(R.st)) break;
    const uint64_t sk = nsp ? R.spatial[i] : 0;
    if (nsp && spatial_none(R, sk)) continue;  // cleared (they sort last)
    const uint32_t c = first ? (nsp ? (uint32_t)(sk >> 32) : (uint32_t)i) : list[i];
    if (first && !nsp && R.cleared[c]) continue;
    reduce_round_reg<TC>(R, c, first != 0, off2, short_next, n_short_next, long_next, n_long_next, &adds);
  }
  if (adds) atomicAdd(&R.st->adds, adds);
}

// ---- wave mode: one wavefront per column -----------------------------------------
//
// The working column is the XOR of four sorted lists, each level absorbing the
// one before it when that fills (a log-structured merge):
//   P -- at most 128 keys in registers, lane i holding the i-th and the
//        (64 + i)-th smallest; the three new edges of an apparent addition and
//        short owner columns go here;
//   F -- the front list in this wavefront's LDS (at most front_cap keys), which
//        absorbs P when it fills and owner columns too long for P (merged
//        straight from the arena);
//   U -- the middle list in the arena, which absorbs F when F fills and owner
//        columns longer than half of F, and is folded into T when it would
//        grow past mid_cap keys;
//   T -- the tail in the arena.
// Arena lists are immutable (a merge into one writes a new list); the top 64
// keys of U and of T are kept in register windows.  The pivot is the largest
// key present an odd number of times among the tops of the four lists.  An
// iteration issues its loads together: the apparent code of the pivot edge,
// its owner word, and the ten pixels that the four squares around the edge can
// have as vertices, so an apparent addition costs one memory latency and an
// owner addition two.  Merges are merge-path XOR merges: a fixed number of
// positions per lane, equal pairs dropped, never split between lanes.  Every
// step is wave-synchronous: no workgroup barriers.
//
// Two configurations: the wide one (large stage and front list, few
// wavefronts per CU) for rounds with few, long columns, and the narrow one
// (small LDS footprint, four wavefronts per SIMD to hide memory latency) for
// rounds with many columns.
constexpr int WPB = 2;                 // wavefronts per workgroup
constexpr int PER_WIDE = 16;           // merge positions per lane per step of a merge into F
constexpr int PER_NARROW = 2;          // ... of a merge into P
constexpr uint64_t KEY_INF = ~0ull;    // above every key
constexpr uint32_t PCAP = 128;         // keys of P: two per lane
template <int PER_>
struct WaveCfg {
  static constexpr int PER = PER_;              // merge positions per lane per step of a merge with an arena list
  static constexpr uint32_t CHUNK = 64 * PER;   // keys per chunk of the ring
  static constexpr uint32_t RING = 4;           // chunks of the ring (two in use, one arriving, one spare)
  static constexpr uint32_t XN = RING * CHUNK;  // the stage: the ring of a merge with an arena list
  static_assert((XN & (XN - 1)) == 0, "the ring is indexed with a mask");
};
using WideCfg = WaveCfg<8>;
using NarrowCfg = WaveCfg<2>;
static_assert(WPB * 8 * (2 * FRONT_CAP_MAX + WideCfg::XN + PCAP) <= 160 * 1024, "wave-mode LDS exceeds a workgroup's share");
static_assert(WPB * 8 * (2 * FRONT_CAP_NARROW_MAX + NarrowCfg::XN + PCAP) * 8 <= 160 * 1024,
              "narrow wave mode: eight workgroups per CU");

template <class C>
__host__ __device__ __forceinline__ size_t wave_lds_words(uint32_t front_cap) { return 2 * (size_t)front_cap + C::XN + PCAP; }

struct WaveBufs {
  uint64_t* F0;      // the two front buffers (the front list and its merge target)
  uint64_t* F1;
  uint64_t* X;       // the stage
  uint64_t* ps;      // PCAP words: P staged for a merge
  uint64_t* hx;      // 64 words: a short owner column staged for a merge into P
  uint64_t* po;      // PCAP words: the output of that merge (null: F's spare buffer)
  uint32_t cap;
};

__device__ __forceinline__ uint64_t* fbuf(const WaveBufs& S, uint32_t i) { return i ? S.F1 : S.F0; }

// An arena list with a register window over its top: lane i holds v[b + i]
// for b + i < n.
struct Tail {
  const uint64_t* v;
  uint64_t w;
  uint32_t n, b;
};
// The wave-mode kernel's RedCtx argument (its first, so at the start of the
// kernel argument segment) through a pointer that the compiler may not assume
// unchanged: fields read through it are loaded (scalar loads) where they are
// used instead of occupying scalar registers for the whole column loop.  For
// fields that the per-iteration path does not touch; only code called from
// k_red_round_wave uses it.
using KargCtx = const __attribute__((address_space(4))) RedCtx;
__device__ __forceinline__ KargCtx* cold(const RedCtx&) {
  KargCtx* p = (KargCtx*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return p;
}

struct WState {
  uint64_t p0, p1;   // P: this lane's keys lane and 64 + lane (below np)
  Tail U, T;
  uint32_t np, nf, cur;
  unsigned long long adds, merged;  // statistics, counted in lane 0 (vector registers)
};
__device__ __forceinline__ void w_count(unsigned long long& acc, uint32_t v, int lane) {
  acc += lane == 0 ? v : 0u;
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// After global stores that other lanes of the wave read back.
__device__ __forceinline__ void wsync_global() {
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
// Wave-uniform 64-bit value kept in scalar registers (so branches on it are scalar).
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, uint32_t i) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)i);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---- P, the register list: key i in lane i (i < 64) or lane i - 64 of p1 ----
__device__ __forceinline__ uint64_t p_top(const WState& W) {
  return W.np == 0 ? 0 : (W.np <= 64 ? rdlane64(W.p0, W.np - 1) : rdlane64(W.p1, W.np - 65));
}
// Writes P ascending to dst[0..np).
__device__ __forceinline__ void p_stage(const WState& W, uint64_t* dst, int lane) {
  if ((uint32_t)lane < W.np) dst[lane] = W.p0;
  if ((uint32_t)lane + 64 < W.np) dst[64 + lane] = W.p1;
}
// P = src[0..n), n <= PCAP.
__device__ __forceinline__ void p_load(WState& W, const uint64_t* src, uint32_t n, int lane) {
  W.p0 = (uint32_t)lane < n ? src[lane] : 0;
  W.p1 = (uint32_t)lane + 64 < n ? src[64 + lane] : 0;
  W.np = n;
}
// P ^= {k0, k1, k2} for three distinct wave-uniform keys, P holding at most
// PCAP - 3 keys: each kept key and each new key goes to its rank through the
// LDS slot ps, with no branches on the data.
__device__ __forceinline__ void p_insert3(const WaveBufs& S, WState& W, uint64_t k0, uint64_t k1, uint64_t k2,
                                          int lane) {
  {
    // The common case: the three keys (the rest of the boundary of the square
    // paired with the pivot just removed) all lie above P's top.  They cannot
    // be in P, so they go on top in ascending order, with no exchange through
    // LDS.  Slots beyond np are never read.
    uint64_t a = k0, b = k1, c = k2;
    if (a > b) { const uint64_t t = a; a = b; b = t; }
    if (b > c) { const uint64_t t = b; b = c; c = t; }
    if (a > b) { const uint64_t t = a; a = b; b = t; }
    const uint32_t n = W.np;
    if (a > p_top(W) && n + 3 <= PCAP) {
      const uint32_t l0 = (uint32_t)lane, l1 = (uint32_t)lane + 64;
      W.p0 = l0 == n ? a : (l0 == n + 1 ? b : (l0 == n + 2 ? c : W.p0));
      W.p1 = l1 == n ? a : (l1 == n + 1 ? b : (l1 == n + 2 ? c : W.p1));
      W.np = n + 3;
      return;
    }
  }
  const bool in0 = (uint32_t)lane < W.np, in1 = (uint32_t)lane + 64 < W.np;
  const bool h0 = (wballot(in0 && W.p0 == k0) | wballot(in1 && W.p1 == k0)) != 0;
  const bool h1 = (wballot(in0 && W.p0 == k1) | wballot(in1 && W.p1 == k1)) != 0;
  const bool h2 = (wballot(in0 && W.p0 == k2) | wballot(in1 && W.p1 == k2)) != 0;
  const uint64_t km0 = wballot(in0 && W.p0 != k0 && W.p0 != k1 && W.p0 != k2);  // lanes whose key stays
  const uint64_t km1 = wballot(in1 && W.p1 != k0 && W.p1 != k1 && W.p1 != k2);
  const bool n0 = !h0, n1 = !h1, n2 = !h2;  // keys that are new
  auto below = [&](uint64_t k) {  // kept keys below k
    return (uint32_t)__popcll(km0 & wballot(W.p0 < k)) + (uint32_t)__popcll(km1 & wballot(W.p1 < k));
  };
  const uint32_t r0 = below(k0) + (n1 && k1 < k0) + (n2 && k2 < k0);
  const uint32_t r1 = below(k1) + (n0 && k0 < k1) + (n2 && k2 < k1);
  const uint32_t r2 = below(k2) + (n0 && k0 < k2) + (n1 && k1 < k2);
  const uint32_t c0 = (uint32_t)__popcll(km0);
  if ((km0 >> lane) & 1)
    S.ps[mbcnt64(km0) + (n0 && k0 < W.p0) + (n1 && k1 < W.p0) + (n2 && k2 < W.p0)] = W.p0;
  if ((km1 >> lane) & 1)
    S.ps[c0 + mbcnt64(km1) + (n0 && k0 < W.p1) + (n1 && k1 < W.p1) + (n2 && k2 < W.p1)] = W.p1;
  if (lane < 3 && sel3(lane, n0, n1, n2)) S.ps[sel3(lane, r0, r1, r2)] = sel3(lane, k0, k1, k2);
  wsync();
  p_load(W, S.ps, c0 + (uint32_t)__popcll(km1) + n0 + n1 + n2, lane);
  wsync();
}

// Exclusive prefix over the wave of a count below 2^BITS per lane, from one
// ballot per bit; sets *total.
template <int BITS>
__device__ __forceinline__ uint32_t w_excl_small(uint32_t v, uint32_t* total) {
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int bit = 0; bit < BITS; ++bit) {
    const uint64_t bm = wballot(((v >> bit) & 1u) != 0);
    pre += mbcnt64(bm) << bit;
    tot += (uint32_t)__popcll(bm) << bit;
  }
  *total = tot;
  return pre;
}

// Pointers with an explicit address space.  In code compiled out of line the
// compiler cannot see where a pointer came from and accesses it with flat
// instructions, which are slower to LDS and count against both the LDS and the
// vector memory counters (a wait for an LDS value then also waits for every
// global load in flight); the merges below take their LDS and arena operands
// through these instead.
using lds64 = __attribute__((address_space(3))) uint64_t;
using glb64 = __attribute__((address_space(1))) uint64_t;
__device__ __forceinline__ lds64* to_lds(const uint64_t* p) { return (lds64*)(uint64_t*)p; }
__device__ __forceinline__ glb64* to_glb(const uint64_t* p) { return (glb64*)(uint64_t*)p; }

// A sorted list seen through an index map: a plain LDS array, or a window of
// a ring of N slots in LDS (key i of the window is ring slot (base + i) mod N).
struct Lin {
  const lds64* p;
  __device__ __forceinline__ uint64_t operator[](uint32_t i) const { return p[i]; }
};
template <uint32_t N>
struct RingN {
  const lds64* p;
  uint32_t base;
  __device__ __forceinline__ uint64_t operator[](uint32_t i) const { return p[(base + i) & (N - 1)]; }
};

// Number of A elements among the first d positions of the merge of A and B,
// ties taken from A first.
template <class AA, class BB>
__device__ __forceinline__ uint32_t mp_split(const AA& A, uint32_t na, const BB& B, uint32_t nb, uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if (A[m] <= B[d - m - 1]) lo = m + 1;
    else hi = m;
  }
  return lo;
}

// Writes the XOR of the first d merge positions of A and B (LDS, ascending;
// equal pairs dropped) ascending to out, d <= 64 * P.  An equal pair is never
// split: if position d falls between its two copies the second is consumed
// too.  A or B may be a tile of a longer list as long as it holds at least d
// keys or all that remain.  Sets *ka, *kb to the keys consumed; returns the
// number written.
struct SegResult {
  uint32_t written, ka, kb;
};
template <int P, class AA, class BB, class O>
__device__ __forceinline__ SegResult w_merge_seg(const AA& A, uint32_t na, const BB& B, uint32_t nb,
                                                 uint32_t d, O* out, int lane) {
  const uint32_t dend = (uint32_t)(lane + 1) * P < d ? (uint32_t)(lane + 1) * P : d;
  const uint32_t ie = mp_split(A, na, B, nb, dend);
  uint32_t je = dend - ie;
  if (ie > 0 && je < nb && A[ie - 1] == B[je]) ++je;
  uint32_t is = __shfl_up(ie, 1, 64), js = __shfl_up(je, 1, 64);
  if (lane == 0) {
    is = 0;
    js = 0;
  }
  uint32_t i = is, j = js;
  uint64_t a = i < ie ? A[i] : KEY_INF;
  uint64_t b = j < je ? B[j] : KEY_INF;
  uint64_t buf[P + 1];
  uint32_t keep = 0;
#pragma unroll
  for (int t = 0; t <= P; ++t) {
    buf[t] = 0;
    if (a < b) {
      buf[t] = a;
      keep |= 1u << t;
      ++i;
      a = i < ie ? A[i] : KEY_INF;
    } else if (b < a) {
      buf[t] = b;
      keep |= 1u << t;
      ++j;
      b = j < je ? B[j] : KEY_INF;
    } else if (a != KEY_INF) {  // an equal pair: both dropped
      ++i;
      ++j;
      a = i < ie ? A[i] : KEY_INF;
      b = j < je ? B[j] : KEY_INF;
    }
  }
  uint32_t total;
  uint32_t pos = w_excl_small<(P < 8 ? 3 : (P < 16 ? 4 : 5))>((uint32_t)__popc(keep), &total);
#pragma unroll
  for (int t = 0; t <= P; ++t)
    if (keep & (1u << t)) out[pos++] = buf[t];
  SegResult r;
  r.written = total;
  r.ka = (uint32_t)__builtin_amdgcn_readlane((int)ie, 63);
  r.kb = (uint32_t)__builtin_amdgcn_readlane((int)je, 63);
  return r;
}

// out = A XOR B for sorted lists in LDS; out (LDS) distinct from both.  Out of
// line (like the global merge) to keep the per-iteration code compact.
template <int P>
__device__ __noinline__ uint32_t w_xor_lds(const uint64_t* A_, uint32_t na, const uint64_t* B_, uint32_t nb,
                                           uint64_t* out_, int lane) {
  const lds64* A = to_lds(A_);
  const lds64* B = to_lds(B_);
  lds64* out = to_lds(out_);
  uint32_t ia = 0, ib = 0, o = 0;
  while (ia < na || ib < nb) {
    const uint32_t rem = (na - ia) + (nb - ib);
    const SegResult r = w_merge_seg<P>(Lin{A + ia}, na - ia, Lin{B + ib}, nb - ib, rem < 64u * P ? rem : 64u * P,
                                       out + o, lane);
    o += r.written;
    ia += r.ka;
    ib += r.kb;
  }
  wsync();
  return o;
}

// out = T XOR F, T in the arena, F in LDS, out in the arena (OUT_LDS false) or
// in LDS (OUT_LDS true: an owner column merged into the front list).  T is read through a ring
// of RING chunks in the stage: the chunks holding the next CHUNK keys are
// resident, and the chunk after them is loaded into registers during each
// merge step and stored into the ring when it is needed, so the load latency
// overlaps the merging.
template <class C, bool OUT_LDS>
__device__ __noinline__ uint32_t w_merge_tail(uint64_t* X_, const uint64_t* T_, uint32_t nt, const uint64_t* F_,
                                              uint32_t nf, uint64_t* out_, int lane) {
  lds64* X = to_lds(X_);
  const glb64* T = to_glb(T_);
  const lds64* F = to_lds(F_);
  auto out = [&] {
    if constexpr (OUT_LDS) return to_lds(out_);
    else return to_glb(out_);
  }();
  constexpr int PER = C::PER;
  constexpr uint32_t CHUNK = C::CHUNK, RING = C::RING;
  const uint32_t nch = (nt + CHUNK - 1) / CHUNK;
  uint64_t pre[PER];
  auto load_chunk = [&](uint32_t c) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t i = c * CHUNK + (uint32_t)(j * 64 + lane);
      pre[j] = (c < nch && i < nt) ? T[i] : 0ull;
    }
  };
  auto store_chunk = [&](uint32_t c) {
    lds64* slot = X + (c % RING) * CHUNK;
#pragma unroll
    for (int j = 0; j < PER; ++j) slot[j * 64 + lane] = pre[j];
  };
  load_chunk(0);
  store_chunk(0);
  load_chunk(1);
  store_chunk(1);
  uint32_t next = 2;  // the chunk in flight in pre[]
  load_chunk(next);
  wsync();
  uint32_t ia = 0, ib = 0, o = 0;
  while (ia < nt || ib < nf) {
    const uint32_t la = nt - ia < CHUNK ? nt - ia : CHUNK;
    const uint32_t lb = nf - ib < CHUNK ? nf - ib : CHUNK;
    const SegResult r = w_merge_seg<PER>(RingN<C::XN>{X, ia}, la, Lin{F + ib}, lb, la + lb < CHUNK ? la + lb : CHUNK, out + o,
                                         lane);
    o += r.written;
    ia += r.ka;
    ib += r.kb;
    // the next step reads chunks ia / CHUNK and the one after; the ring slot of
    // the arriving chunk last held a chunk below ia / CHUNK
    if (next < nch && next <= ia / CHUNK + 1) {
      wsync();
      store_chunk(next);
      ++next;
      load_chunk(next);
    }
    wsync();
  }
  wsync_global();
  return o;
}

// out (arena) = A XOR B, both in the arena: as w_merge_tail, with the stage
// split into one ring per input and chunks of half the size.
template <class C>
__device__ __noinline__ uint32_t w_merge_gg(uint64_t* X_, const uint64_t* A_, uint32_t na, const uint64_t* B_,
                                            uint32_t nb, uint64_t* out_, int lane) {
  const glb64* A = to_glb(A_);
  const glb64* B = to_glb(B_);
  glb64* out = to_glb(out_);
  constexpr uint32_t RING = C::RING;
  constexpr uint32_t HN = C::XN / 2;       // words of each ring
  constexpr uint32_t HCH = HN / RING;      // keys per chunk
  constexpr int HP = (int)(HCH / 64);      // merge positions per lane per step
  lds64* XA = to_lds(X_);
  lds64* XB = XA + HN;
  const uint32_t nca = (na + HCH - 1) / HCH, ncb = (nb + HCH - 1) / HCH;
  uint64_t pa[HP], pb[HP];
  auto load = [&](const glb64* src, uint32_t n, uint32_t nch, uint32_t c, uint64_t* pre) {
#pragma unroll
    for (int j = 0; j < HP; ++j) {
      const uint32_t i = c * HCH + (uint32_t)(j * 64 + lane);
      pre[j] = (c < nch && i < n) ? src[i] : 0ull;
    }
  };
  auto store = [&](lds64* ring, uint32_t c, const uint64_t* pre) {
    lds64* slot = ring + (c % RING) * HCH;
#pragma unroll
    for (int j = 0; j < HP; ++j) slot[j * 64 + lane] = pre[j];
  };
  load(A, na, nca, 0, pa);
  load(B, nb, ncb, 0, pb);
  store(XA, 0, pa);
  store(XB, 0, pb);
  load(A, na, nca, 1, pa);
  load(B, nb, ncb, 1, pb);
  store(XA, 1, pa);
  store(XB, 1, pb);
  uint32_t nexta = 2, nextb = 2;  // the chunks in flight in pa[] / pb[]
  load(A, na, nca, nexta, pa);
  load(B, nb, ncb, nextb, pb);
  wsync();
  uint32_t ia = 0, ib = 0, o = 0;
  while (ia < na || ib < nb) {
    const uint32_t la = na - ia < HCH ? na - ia : HCH;
    const uint32_t lb = nb - ib < HCH ? nb - ib : HCH;
    const SegResult r = w_merge_seg<HP>(RingN<HN>{XA, ia}, la, RingN<HN>{XB, ib}, lb, la + lb < HCH ? la + lb : HCH,
                                        out + o, lane);
    o += r.written;
    ia += r.ka;
    ib += r.kb;
    // each input advances by at most one chunk per step
    const bool sa = nexta < nca && nexta <= ia / HCH + 1;
    const bool sb = nextb < ncb && nextb <= ib / HCH + 1;
    if (sa || sb) {
      wsync();
      if (sa) {
        store(XA, nexta, pa);
        ++nexta;
        load(A, na, nca, nexta, pa);
      }
      if (sb) {
        store(XB, nextb, pb);
        ++nextb;
        load(B, nb, ncb, nextb, pb);
      }
    }
    wsync();
  }
  wsync_global();
  return o;
}

// Allocates n arena entries (lane 0) and broadcasts the offset (~0 on overflow).
__device__ __forceinline__ uint64_t w_alloc(const RedCtx& R, uint64_t n, int lane) {
  unsigned long long off = 0;
  if (lane == 0) {
    const auto* C = cold(R);
    n = n ? n : 1;
    off = atomicAdd(C->arena_top, (unsigned long long)n);
    if (off + n > C->arena_cap) {
      raise_flag(C->st, &C->st->overflow, OVF_ARENA);
      off = ~0ull;
    }
  }
  return rdlane64(off, 0);
}

// Waits for this wavefront's outstanding vector memory operations.  Registers
// loaded from global memory in a loop body are otherwise taken as possibly in
// flight wherever the loop reads them, and the compiler waits there for every
// load issued since -- in the pivot search, for the loads started ahead for
// the next pivot, which then save nothing.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0xF70); }  // vmcnt(0)

__device__ __forceinline__ void tail_window(Tail& t, int lane) {
  t.b = t.n > 64 ? t.n - 64 : 0;
  t.w = (t.b + (uint32_t)lane < t.n) ? t.v[t.b + lane] : 0;
  wait_vm();  // read at once by the pivot search
}
__device__ __forceinline__ void tail_set(Tail& t, const uint64_t* v, uint32_t n, int lane) {
  t.v = v;
  t.n = n;
  tail_window(t, lane);
}
__device__ __forceinline__ uint64_t tail_top(const Tail& t) { return t.n ? rdlane64(t.w, t.n - 1 - t.b) : 0; }
__device__ __forceinline__ void tail_pop(Tail& t, int lane) {
  --t.n;
  if (t.n > 0 && t.n == t.b) tail_window(t, lane);
}

// T ^= U (U becomes empty).
template <class C>
__device__ __forceinline__ bool w_fold_mid(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
  if (W.U.n == 0) return true;
  if (W.T.n == 0) {
    W.T = W.U;
  } else {
    const uint64_t off = w_alloc(R, (uint64_t)W.T.n + W.U.n, lane);
    if (off == ~0ull) return false;
    const uint32_t len = uni(w_merge_gg<C>(S.X, W.T.v, W.T.n, W.U.v, W.U.n, R.arena + off, lane));
    w_count(W.merged, W.T.n + W.U.n, lane);
    tail_set(W.T, R.arena + off, len, lane);
  }
  W.U.n = 0;
  return true;
}

// U ^= F (F becomes empty), folding U into T first if U would outgrow mid_cap.
template <class C>
__device__ __forceinline__ bool w_push_front(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
  if (W.nf == 0) return true;
  if (W.U.n + W.nf > cold(R)->mid_cap && !w_fold_mid<C>(R, S, W, lane)) return false;
  const uint64_t off = w_alloc(R, (uint64_t)W.U.n + W.nf, lane);
  if (off == ~0ull) return false;
  const uint32_t len = uni(w_merge_tail<C, false>(S.X, W.U.v, W.U.n, fbuf(S, W.cur), W.nf, R.arena + off, lane));
  w_count(W.merged, W.U.n + W.nf, lane);
  W.nf = 0;
  tail_set(W.U, R.arena + off, len, lane);
  return true;
}

// F ^= X[0..m) (X in LDS), pushing F into T first if the result might not fit.
template <class C>
__device__ __forceinline__ bool w_front_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* X, uint32_t m,
                            int lane) {
  if (W.nf + m > S.cap && !w_push_front<C>(R, S, W, lane)) return false;
  w_count(W.merged, W.nf + m, lane);
  W.nf = uni(w_xor_lds<PER_WIDE>(fbuf(S, W.cur), W.nf, X, m, fbuf(S, W.cur ^ 1), lane));
  W.cur ^= 1;
  return true;
}

// Adds a sorted arena list Q[0..m) (an owner column) to the column: into F,
// streamed through the stage, or, for a list of more than half of F's
// capacity, into U (which becomes Q itself when it is empty: arena lists are
// immutable).
template <class C>
__device__ __forceinline__ bool w_owner_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* Q,
                                            uint32_t m, int lane) {
  if (2 * m > S.cap) {
    if (W.U.n + m > cold(R)->mid_cap && !w_fold_mid<C>(R, S, W, lane)) return false;
    if (W.U.n == 0) {
      tail_set(W.U, Q, m, lane);
      return true;
    }
    const uint64_t off = w_alloc(R, (uint64_t)W.U.n + m, lane);
    if (off == ~0ull) return false;
    const uint32_t len = uni(w_merge_gg<C>(S.X, W.U.v, W.U.n, Q, m, R.arena + off, lane));
    w_count(W.merged, W.U.n + m, lane);
    tail_set(W.U, R.arena + off, len, lane);
    return true;
  }
  if (W.nf + m > S.cap && !w_push_front<C>(R, S, W, lane)) return false;
  w_count(W.merged, W.nf + m, lane);
  W.nf = uni(w_merge_tail<C, true>(S.X, Q, m, fbuf(S, W.cur), W.nf, fbuf(S, W.cur ^ 1), lane));
  W.cur ^= 1;
  return true;
}

// F ^= P (P becomes empty).
template <class C>
__device__ __forceinline__ bool w_flush_p(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
  if (W.np == 0) return true;
  p_stage(W, S.ps, lane);
  wsync();
  const uint32_t np = W.np;
  W.np = 0;
  return w_front_add<C>(R, S, W, S.ps, np, lane);
}

// P ^= {k0, k1, k2} for three distinct wave-uniform keys (flushing P first if
// it might overflow): each kept key and each new key goes to its rank through
// the LDS pending slot, with no branches on the data.
template <class C>
__device__ __forceinline__ bool w_insert3(const RedCtx& R, const WaveBufs& S, WState& W, uint64_t k0, uint64_t k1,
                                          uint64_t k2, int lane) {
  if (W.np > PCAP - 3 && !w_flush_p<C>(R, S, W, lane)) return false;
  p_insert3(S, W, k0, k1, k2, lane);
  return true;
}

// P ^= X[0..m) for a staged list with np + m <= PCAP; the output goes through
// S.po, or F's spare buffer.
__device__ __forceinline__ void w_p_add(const WaveBufs& S, WState& W, const uint64_t* X, uint32_t m, int lane) {
  p_stage(W, S.ps, lane);
  wsync();
  uint64_t* out = S.po ? S.po : fbuf(S, W.cur ^ 1);
  const uint32_t n = uni(w_xor_lds<PER_NARROW>(S.ps, W.np, X, m, out, lane));
  w_count(W.merged, W.np + m, lane);
  p_load(W, out, n, lane);
  wsync();
}

// Largest key present an odd number of times among the tops of P, F, U and
// T, after dropping equal pairs (0 if the column is empty); *where names the
// list that holds it afterwards (0 = P, 1 = F, 2 = U, 3 = T).
__device__ __forceinline__ uint64_t w_pivot(const WaveBufs& S, WState& W, int lane, int* where) {
  for (;;) {
    const uint64_t a = p_top(W);
    const uint64_t b = W.nf ? uni64(fbuf(S, W.cur)[W.nf - 1]) : 0;
    const uint64_t u = tail_top(W.U);
    const uint64_t c = tail_top(W.T);
    uint64_t m = a > b ? a : b;
    m = m > u ? m : u;
    m = m > c ? m : c;
    if (m == 0) return 0;
    const bool ha = a == m, hb = b == m, hu = u == m, hc = c == m;
    // copies cancel in pairs; an odd count leaves the one in the deepest list
    const int keep = ((int)ha + (int)hb + (int)hu + (int)hc) & 1 ? (hc ? 3 : (hu ? 2 : (hb ? 1 : 0))) : -1;
    if (ha && keep != 0) --W.np;
    if (hb && keep != 1) --W.nf;
    if (hu && keep != 2) tail_pop(W.U, lane);
    if (hc && keep != 3) tail_pop(W.T, lane);
    if (keep >= 0) {
      *where = keep;
      return m;
    }
  }
}

__device__ __forceinline__ void w_pop(WState& W, int where, int lane) {
  if (where == 0) --W.np;
  else if (where == 1) --W.nf;
  else if (where == 2) tail_pop(W.U, lane);
  else tail_pop(W.T, lane);
}

__device__ __forceinline__ float rdlane_f(float v, uint32_t i) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)i));
}
// The steps of a column reduction that differ between one wavefront per
// column and a workgroup per column.
template <class C>
struct WaveOps {
  static constexpr bool kAsync = false;  // the asynchronous tail (claims by compare-and-swap)
  // whether the list at this arena offset was stored during the asynchronous tail
  __device__ static bool fresh(const RedCtx&, uint32_t) { return false; }
  __device__ static bool leader(int lane) { return lane == 0; }
  // the round of this launch and the additions after which a column yields
  __device__ static uint32_t round(const RedCtx& R) { return cold(R)->round; }
  __device__ static uint32_t wave_yield(const RedCtx& R) { return cold(R)->wave_yield; }
  __device__ static bool aborted(const RedCtx& R, const WaveBufs&) { return cr::aborted(cold(R)->st); }
  __device__ static uint64_t alloc(const RedCtx& R, const WaveBufs&, uint64_t n, int lane) { return w_alloc(R, n, lane); }
  __device__ static bool insert3(const RedCtx& R, const WaveBufs& S, WState& W, uint64_t k0, uint64_t k1, uint64_t k2,
                                 int lane) {
    return w_insert3<C>(R, S, W, k0, k1, k2, lane);
  }
  __device__ static bool flush_p(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
    return w_flush_p<C>(R, S, W, lane);
  }
  __device__ static bool push_front(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
    return w_push_front<C>(R, S, W, lane);
  }
  __device__ static bool front_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* X, uint32_t m,
                                   int lane) {
    return w_front_add<C>(R, S, W, X, m, lane);
  }
  __device__ static uint32_t merge_tail(const WaveBufs& S, const uint64_t* T, uint32_t nt, const uint64_t* F,
                                        uint32_t nf, uint64_t* out, int lane) {
    return uni(w_merge_tail<C, false>(S.X, T, nt, F, nf, out, lane));  // out: the arena
  }
  __device__ static uint32_t merge_gg(const WaveBufs& S, const uint64_t* A, uint32_t na, const uint64_t* B,
                                      uint32_t nb, uint64_t* out, int lane) {
    return uni(w_merge_gg<C>(S.X, A, na, B, nb, out, lane));
  }
  __device__ static void copy_in(const WaveBufs&, uint64_t* dst, const uint64_t* src, uint32_t n, int lane) {
    for (uint32_t i = (uint32_t)lane; i < n; i += 64) dst[i] = src[i];
    wsync();
  }
  __device__ static bool owner_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* Q, uint32_t m,
                                   int lane) {
    return w_owner_add<C>(R, S, W, Q, m, lane);
  }
  __device__ static void copy_out(const WaveBufs&, uint64_t* dst, const uint64_t* src, uint32_t n, int lane) {
    for (uint32_t i = (uint32_t)lane; i < n; i += 64) dst[i] = src[i];
  }
};

// The geometry of one image that the load group of an edge needs.
struct EdgeGeom {
  int kb;                              // bits of the key's index field
  uint32_t K0, K1, K2;                 // Khalimsky extents z, y, x
  double rK1, rK2;                     // their reciprocals
  uint32_t n0, n1, n2, ps0, ps1;       // pixel extents and strides
  const float* img;                    // the image's pixels
  const uint8_t* eapp;                 // its edges' apparent codes (4 bytes per anchor pixel)
  const uint64_t* owner;               // its edges' owner words
};
// What a lane loads for edge e in role r (the value only once it is used):
// roles 0 and 1 the edge's endpoints, 2..9 the far vertices of the four
// squares around it (role 2 + 4h + 2s + o: the other axis h, side s, endpoint
// o; other roles and vertices off the image read the anchor); every role the
// edge's apparent code and owner word.
struct LoadGroup {
  float praw;
  uint32_t code;
  uint64_t ow;
};
__device__ __forceinline__ LoadGroup load_group(const EdgeGeom& G, uint64_t e, uint32_t r) {
  const uint32_t kidx = (uint32_t)(e & ((1ull << G.kb) - 1));
  const uint32_t t1 = udiv_rcp(kidx, G.K2, G.rK2), kx = kidx - t1 * G.K2;
  const uint32_t kz = udiv_rcp(t1, G.K1, G.rK1), ky = t1 - kz * G.K1;
  const int ax = (kz & 1) ? 0 : ((ky & 1) ? 1 : 2);
  const int b0 = ax == 0 ? 1 : 0, b1 = ax == 2 ? 1 : 2;  // the two other axes
  // not an edge of the image (a broken invariant, reported where e is used as
  // a pivot): read in-range addresses only
  const bool edge = kz < G.K0 && ((kz & 1) + (ky & 1) + (kx & 1)) == 1;
  const uint32_t cz = edge ? kz >> 1 : 0, cy = edge ? ky >> 1 : 0, cx = edge ? kx >> 1 : 0;
  const uint32_t pax = sel3(ax, G.ps0, G.ps1, 1u);
  const uint32_t anchor = cz * G.ps0 + cy * G.ps1 + cx;
  const uint32_t slot = 3 * anchor + (uint32_t)ax;
  const uint32_t rq = r - 2;
  const bool rfar = r >= 2 && r < 10;
  const int bb = (rq & 4) ? b1 : b0;
  const int rsg = (rq & 2) ? 1 : -1;
  const uint32_t vb = sel3(bb, cz, cy, cx) + (uint32_t)rsg;  // wraps below 0
  const bool pix_ok = edge && (r < 2 || (rfar && vb < sel3(bb, G.n0, G.n1, G.n2)));
  const uint32_t pofs = ((r == 1 || (rfar && (rq & 1))) ? pax : 0u) +
                        (rfar ? (uint32_t)(rsg * (int32_t)sel3(bb, G.ps0, G.ps1, 1u)) : 0u);
  LoadGroup g;
  g.praw = G.img[pix_ok ? anchor + pofs : anchor];
  g.code = G.eapp[4 * anchor + (uint32_t)ax];
  g.ow = G.owner[slot];
  return g;
}

// Stores the column P ^ F ^ U ^ T as one arena list and records it for column
// c with pivot key pv: with a claim word, c is proposed for that pivot;
// without one (pv = YIELDED) c is appended to the next round's long list.
// In the asynchronous tail (O::kAsync) nothing is recorded: the caller claims
// the pivot.  Returns the list's arena offset, ~0 on failure.
template <class O>
__device__ __forceinline__ uint64_t store_column(const RedCtx& R, const WaveBufs& S, WState& W, uint32_t c,
                                                 uint64_t pv, uint64_t* claim_at, int lane) {
  uint64_t off;
  uint32_t len;
  if (W.nf == 0 && W.U.n == 0 && W.T.n == 0) {  // the column is P
    off = O::alloc(R, S, (uint64_t)W.np + 1, lane);
    if (off == ~0ull) return off;
    p_stage(W, R.arena + off + 1, lane);
    len = W.np;
  } else {
    if (!O::flush_p(R, S, W, lane)) return ~0ull;
    if (W.U.n && W.T.n && !O::push_front(R, S, W, lane)) return ~0ull;
    const Tail& G = W.T.n ? W.T : W.U;  // at most one of them is left with F
    const Tail& H = W.T.n ? W.U : W.T;
    off = O::alloc(R, S, (uint64_t)W.nf + G.n + H.n + 1, lane);
    if (off == ~0ull) return off;
    if (H.n) {
      len = O::merge_gg(S, G.v, G.n, H.v, H.n, R.arena + off + 1, lane);
    } else if (G.n) {
      len = O::merge_tail(S, G.v, G.n, fbuf(S, W.cur), W.nf, R.arena + off + 1, lane);
    } else {
      O::copy_out(S, R.arena + off + 1, fbuf(S, W.cur), W.nf, lane);
      len = W.nf;
    }
  }
  if (O::leader(lane)) {
    R.arena[off] = len;
    if (!O::kAsync) {
      const auto* K = cold(R);
      K->col_ptr[c] = off;
      K->piv[c] = pv;
      if (claim_at) {
        atomicMax(reinterpret_cast<unsigned long long*>(claim_at), claim_word(O::round(R), c));
      } else {
        const unsigned long long i = atomicAdd(K->yield_count, 1ull);
        K->yield_list[i] = c;
      }
    }
  }
  return off;
}

// Where a column reduction starts: its stored list, and optionally the owner
// word of one edge known better than a load of it could (hint_e = 0: none),
// whose list this workgroup wrote itself when hint_own is set.
struct ColStart {
  uint64_t off, hint_e, hint_ow;
  bool hint_own;
};
// How it ended (asynchronous tail): the pivot, the owner word seen for it (no
// owner, or an owner not to the left) and that owner word's address.
struct ColEnd {
  uint64_t e, ow;
  uint64_t* slot;
};

// Reduces column c for one round: until its pivot has no owner to its left,
// then stores it and proposes it for its pivot; or, after wave_yield additions,
// stores it unfinished for the next round, so that one long column does not
// hold back the columns of every other image at the round's end.  In a round
// of few columns (`few`: at most yield_few) there is nothing to run beside a
// long column, so it does not yield.
//
// Returns the stored list's arena offset, ~0 when the reduction stopped on an
// error (a flag is raised).
template <class O>
__device__ __forceinline__ uint64_t reduce_column(const RedCtx& R, const WaveBufs& S, WState& W, uint32_t c,
                                                  uint64_t off2, int lane, bool few, ColStart from,
                                                  ColEnd* end = nullptr) {
  const int im = (int)uni((uint32_t)skey_img(R.L, uni64(cold(R)->skeys[off2 + c])));  // every edge lies in this image
  ImgDesc d = cold(R)->imgs[im];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d.n[a] = (int32_t)uni((uint32_t)d.n[a]);
    d.K[a] = (int32_t)uni((uint32_t)d.K[a]);
  }
  d.pix_off = (int64_t)uni64((uint64_t)d.pix_off);
  const uint32_t K1 = (uint32_t)d.K[1], K2 = (uint32_t)d.K[2];
  // pixel and edge indices within the image fit 32 bits (an image has fewer
  // than 2^27 pixels: its Khalimsky index fits the key's index field)
  const uint32_t n0 = (uint32_t)d.n[0], n1 = (uint32_t)d.n[1], n2 = (uint32_t)d.n[2];
  const uint32_t ps0 = n1 * n2, ps1 = n2;
  const uint32_t ks0 = K1 * K2, ks1 = K2;
  const double rK1 = 1.0 / (double)K1, rK2 = 1.0 / (double)K2;
  const float* imgp = cold(R)->img + d.pix_off;
  const uint8_t* eappp = cold(R)->eapp + 4 * d.pix_off;
  const uint64_t* ownp = cold(R)->owner + 3 * d.pix_off;
  const uint64_t kpre = make_skey(R.L, 1, im, 0, 0);  // the dimension and image fields of an edge key
  const EdgeGeom G{R.L.kb, (uint32_t)d.K[0], K1, K2, rK1, rK2, n0, n1, n2, ps0, ps1, imgp, eappp, ownp};
  LoadGroup pf{0.0f, 0xFFu, NO_OWNER};  // the prefetched load groups and their three edges
  uint64_t pk0 = 0, pk1 = 0, pk2 = 0;
  {
    const uint64_t off = uni64(from.off);
    const uint32_t len = uni((uint32_t)R.arena[off]);
    const uint64_t* src = R.arena + off + 1;
    W.np = 0;
    W.cur = 0;
    tail_set(W.U, src, 0, lane);
    if (len <= PCAP) {  // into P
      p_load(W, src, len, lane);
      wait_vm();
      W.nf = 0;
      tail_set(W.T, src, 0, lane);
    } else if (len <= S.cap) {
      O::copy_in(S, S.F0, src, len, lane);
      W.nf = len;
      tail_set(W.T, src, 0, lane);
    } else {
      W.nf = 0;
      tail_set(W.T, src, len, lane);
    }
  }
  const uint32_t ylim = uni(few || !O::wave_yield(R) ? 0xFFFFFFFFu : O::wave_yield(R));
  uint64_t out_piv = YIELDED;   // what is stored when the loop ends: the pivot and its
  uint64_t* claim_at = nullptr;  // claim word, or YIELDED and none after wave_yield additions
  uint64_t out_ow = NO_OWNER;
  const uint64_t hint_e = uni64(from.hint_e), hint_ow = uni64(from.hint_ow);
  for (uint32_t it = 0;; ++it) {
    if (it >= RED_ITER_CAP) {
      if (lane == 0) raise_flag(cold(R)->st, &cold(R)->st->iter_cap);
      return ~0ull;
    }
    if ((it & 63) == 63 && O::aborted(R, S)) return ~0ull;
    if (it >= ylim) break;
    int where = 0;
    const uint64_t e = w_pivot(S, W, lane, &where);
    if (e == 0) {  // a zero column: impossible after clearing
      if (lane == 0) raise_flag(cold(R)->st, &cold(R)->st->internal);
      return ~0ull;
    }
    // the pivot edge: Khalimsky coordinates, axis, anchor pixel
    const uint32_t kidx = skey_kidx(R.L, e);
    const uint32_t t1 = udiv_rcp(kidx, K2, rK2), kx = kidx - t1 * K2;
    const uint32_t kz = udiv_rcp(t1, K1, rK1), ky = t1 - kz * K1;
    if ((e >> R.L.kb >> 32) != (kpre >> R.L.kb >> 32) || kz >= (uint32_t)d.K[0] ||
        ((kz & 1) + (ky & 1) + (kx & 1)) != 1) {  // not an edge of this image: a broken invariant
      if (lane == 0) raise_flag(cold(R)->st, &cold(R)->st->internal);
      return ~0ull;
    }
    const int ax = (kz & 1) ? 0 : ((ky & 1) ? 1 : 2);
    const int b1 = ax == 2 ? 1 : 2;  // the larger of the two other axes
    const uint32_t kax = sel3(ax, ks0, ks1, 1u);
    const uint32_t slot = 3 * ((kz >> 1) * ps0 + (ky >> 1) * ps1 + (kx >> 1)) + (uint32_t)ax;
    // the load group of e: prefetched with the previous apparent addition when
    // e is one of the three edges it brought in (lanes 16 g .. 16 g + 15 hold
    // edge g's), else loaded now (lanes 0 .. 15)
    const int hit = e == pk0 ? 0 : (e == pk1 ? 1 : (e == pk2 ? 2 : -1));
    uint32_t lb = 0;
    LoadGroup lg = pf;
    if (hit >= 0) lb = 16u * (uint32_t)hit;
    else lg = load_group(G, e, (uint32_t)lane);
    const uint32_t code = uni((uint32_t)__builtin_amdgcn_readlane((int)lg.code, (int)lb));
    const uint64_t ow = e == hint_e ? hint_ow : rdlane64(lg.ow, lb);
    const float pv = (lg.praw != lg.praw) ? INFINITY : canon(lg.praw);
    pk0 = pk1 = pk2 = 0;
    w_count(W.adds, 1, lane);
    if (code != 0xFF) {
      // apparent partner s: its boundary is e and three older edges
      const int pb = (int)(code >> 1);
      const int sg = (code & 1) ? 1 : -1;
      const uint32_t q = lb + 2 + ((pb == b1) ? 4 : 0) + (sg > 0 ? 2 : 0);
      const float v0 = rdlane_f(pv, lb), v1 = rdlane_f(pv, lb + 1);
      const float w0 = rdlane_f(pv, q), w1 = rdlane_f(pv, q + 1);
      const uint32_t kb = (uint32_t)((int)sel3(pb, ks0, ks1, 1u) * sg);
      const uint64_t kw = kpre | ((uint64_t)ord_of(fmaxf(w0, w1)) << R.L.kb) | (kidx + 2 * kb);
      const uint64_t ka0 = kpre | ((uint64_t)ord_of(fmaxf(v0, w0)) << R.L.kb) | (kidx - kax + kb);
      const uint64_t ka1 = kpre | ((uint64_t)ord_of(fmaxf(v1, w1)) << R.L.kb) | (kidx + kax + kb);
      if (kw >= e || ka0 >= e || ka1 >= e) {  // e must be the latest facet of s
        if (lane == 0) raise_flag(cold(R)->st, &cold(R)->st->internal);
        return ~0ull;
      }
      w_pop(W, where, lane);
      // the next pivot is often one of these three edges: start their loads
      // now, to arrive while they are inserted and the next pivot is found
      {
        const uint32_t g = (uint32_t)lane < 32 ? (uint32_t)lane >> 4 : 2u;
        pf = load_group(G, g == 0 ? kw : (g == 1 ? ka0 : ka1), (uint32_t)lane & 15u);
        pk0 = kw;
        pk1 = ka0;
        pk2 = ka1;
      }
      if (!O::insert3(R, S, W, kw, ka0, ka1, lane)) return ~0ull;
      continue;
    }
    const int32_t o = ow == NO_OWNER ? -1 : (int32_t)(ow >> 32);
    if (o >= 0 && (uint32_t)o < c) {  // add the column of o (its top key is e)
      const uint64_t* q = R.arena + (uint32_t)ow;
      // a list stored during the asynchronous tail, by a workgroup that may run
      // on another XCD: see its writes (the owner word was released after them)
      if (O::fresh(R, (uint32_t)ow) && !(from.hint_own && e == hint_e))
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint64_t head = q[lane];  // length word and the first 63 keys
      const uint32_t len = (uint32_t)rdlane64(head, 0);
      const uint32_t m = len - 1;     // keys below e
      w_pop(W, where, lane);
      if (m + W.np <= PCAP && m <= 63) {  // the loaded head holds keys 0..62
        if (lane >= 1 && (uint32_t)lane <= m) S.hx[lane - 1] = head;
        wsync();
        w_p_add(S, W, S.hx, m, lane);
      } else if (!O::owner_add(R, S, W, q + 1, m, lane)) {
        return ~0ull;
      }
      continue;
    }
    // an active column owns nothing; in the tail an owner word read with a
    // plain load may be stale, which the claim's compare-and-swap corrects
    if ((uint32_t)o == c && !O::kAsync) {
      if (lane == 0) raise_flag(cold(R)->st, &cold(R)->st->internal);
      return ~0ull;
    }
    // store P ^ F ^ U ^ T and propose c for e
    out_piv = e;
    out_ow = ow;
    claim_at = O::kAsync ? const_cast<uint64_t*>(ownp) + slot : &cold(R)->claim[3 * d.pix_off + slot];
    break;
  }
  const uint64_t off = store_column<O>(R, S, W, c, out_piv, claim_at, lane);
  if (end) {
    end->e = out_piv;
    end->ow = out_ow;
    end->slot = claim_at;
  }
  return off;
}

// Wave-mode round over the long-column list (and the short list when it has at
// most R.wave_short columns); columns are taken from a counter.
// R must stay the first parameter: the wave-mode helpers read some of its
// fields from the start of the kernel argument segment.
// The narrow configuration runs a round of at least R.narrow_min columns, the
// wide one a round of fewer (both are launched; the other returns at once).
template <class C>
__global__ __launch_bounds__(64 * WPB) void k_red_round_wave(RedCtx R, const uint32_t* __restrict__ list_s,
                                                             const unsigned long long* __restrict__ n_s,
                                                             const uint32_t* __restrict__ list_l,
                                                             const unsigned long long* __restrict__ n_l,
                                                             uint32_t front_cap) {
  extern __shared__ __align__(16) uint64_t lds_words[];
  if (aborted(R.st) || in_tail(R, n_s, 0)) return;
  const uint64_t nl = uni64(*n_l), ns0 = uni64(*n_s);
  const uint64_t ns = ns0 <= R.wave_short ? ns0 : 0;
  if (nl + ns <= R.group_max || (nl + ns >= R.narrow_min) != (C::XN == NarrowCfg::XN)) return;
  const bool few = nl + ns <= R.yield_few;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t* base = lds_words + (size_t)wv * wave_lds_words<C>(front_cap);
  WaveBufs S;
  S.cap = front_cap;
  S.F0 = base;
  S.F1 = base + S.cap;
  S.X = base + 2 * (size_t)S.cap;
  S.ps = S.X + C::XN;
  S.hx = S.X;
  S.po = nullptr;
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  WState W;
  W.adds = 0;
  W.merged = 0;
  for (;;) {
    unsigned long long li = 0;
    if (lane == 0) li = atomicAdd(R.work, 1ull);
    li = rdlane64(li, 0);
    if (li >= nl + ns || aborted(R.st)) break;
    const uint32_t c = uni(li < nl ? list_l[li] : list_s[li - nl]);
    reduce_column<WaveOps<C>>(R, S, W, c, off2, lane, few, ColStart{cold(R)->col_ptr[c], 0, 0, false});
    wsync();
  }
  if (lane == 0 && W.adds) {  // lane 0 holds the counts
    atomicAdd(&R.st->adds, W.adds);
    atomicAdd(&R.st->merged, W.merged);
  }
}

// ---- group mode: one workgroup of GNW wavefronts per column ---------------------------
//
// For rounds with few columns.  The first wavefront (the leader) reduces the
// column as in wave mode and alone holds P, the windows and the counts; the
// other wavefronts wait at a barrier and join it for the operations that carry
// the bulk of a long column's work: the merges of F, U and T, and the copies
// between LDS and the arena.  The leader describes each such operation in LDS
// and the whole workgroup runs it.  A merge advances in steps of GNW * 64 * P
// positions, each wavefront taking a contiguous part of the step (lane splits
// by merge path over the whole lists, restricted to what the step can reach);
// the wavefronts' output counts are combined through LDS before writing.
// Arena inputs stream through rings of four chunks of one step's size (the
// chunks before, at and after the step's start resident, the next one loading
// into registers).
constexpr int GNW = 8;              // wavefronts per group
constexpr int GP_LDS = 4;           // merge positions per lane per step: LDS lists
constexpr int GP_TAIL = 4;          // ... an arena list with an LDS list
constexpr int GP_GG = 2;            // ... two arena lists
constexpr uint32_t GXN = 4 * GNW * 64 * GP_TAIL;  // stage words: one ring of four chunks (two rings for GP_GG)
static_assert(2 * 4 * GNW * 64 * GP_GG == GXN, "the two rings of an arena-arena merge fill the stage");
constexpr uint32_t GPRIV = PCAP + 64 + PCAP;  // the leader's ps, hx, po

enum GOp : uint32_t { G_END = 0, G_MERGE_LDS, G_MERGE_TAIL, G_MERGE_TAIL_LDS, G_MERGE_GG, G_COPY_IN, G_COPY_OUT, G_FENCE };
// An operation for the whole group: LDS operands are word offsets from the
// start of the group's LDS, arena operands are addresses.
struct GDesc {
  uint32_t op, na, nb, pad;
  uint64_t a, b, out;
};
struct GroupShared {
  uint32_t cnt[GNW];   // output counts of the wavefronts in a merge step
  uint32_t end_a, end_b;
  GDesc desc;
};
__host__ __device__ __forceinline__ size_t group_lds_bytes(uint32_t cap) {
  return 8 * (2 * (size_t)cap + GXN + GPRIV) + sizeof(GroupShared);
}
// the largest front list that fits the LDS of a workgroup with the rest
constexpr uint32_t FRONT_CAP_GROUP_MAX =
    (uint32_t)(((160 * 1024 - sizeof(GroupShared)) / 8 - GXN - GPRIV) / 2) & ~63u;
static_assert(FRONT_CAP_GROUP_MAX >= FRONT_CAP_MIN, "group mode LDS leaves no room for the front list");
static_assert(8 * (2 * FRONT_CAP_GROUP_MAX + GXN + GPRIV) + sizeof(GroupShared) <= 160 * 1024,
              "group mode LDS exceeds a workgroup's share");

__device__ __forceinline__ GroupShared* gshared(const WaveBufs& S) {
  return reinterpret_cast<GroupShared*>(S.X + GXN + GPRIV);
}

// Merge-path split at position d, knowing that the split at d0 <= d took ia0
// keys of A: the search only reads A in [ia0, ia0 + d - d0) and B within one
// step of its own start.
template <class AA, class BB>
__device__ __forceinline__ uint32_t g_split(const AA& A, uint32_t na, const BB& B, uint32_t nb, uint32_t d,
                                            uint32_t d0, uint32_t ia0) {
  uint32_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  lo = lo > ia0 ? lo : ia0;
  hi = hi < ia0 + (d - d0) ? hi : ia0 + (d - d0);
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if (A[m] <= B[d - m - 1]) lo = m + 1;
    else hi = m;
  }
  return lo;
}

// A sorted arena list streamed through a ring of four chunks of CH keys; the
// workgroup loads a chunk with P keys per thread.
template <int P>
struct GRing {
  static constexpr uint32_t CH = GNW * 64 * P;
  lds64* slots;
  const glb64* src;
  uint32_t n, nch, next;
  uint64_t pre[P];
  __device__ __forceinline__ uint64_t operator[](uint32_t i) const { return slots[i & (4 * CH - 1)]; }
  __device__ __forceinline__ void load(uint32_t c) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const uint32_t i = c * CH + (uint32_t)j * (GNW * 64) + threadIdx.x;
      pre[j] = (c < nch && i < n) ? src[i] : 0ull;
    }
  }
  __device__ __forceinline__ void store(uint32_t c) {
#pragma unroll
    for (int j = 0; j < P; ++j) slots[(c % 4) * CH + (uint32_t)j * (GNW * 64) + threadIdx.x] = pre[j];
  }
  __device__ __forceinline__ void init(uint64_t* sl, const uint64_t* s, uint32_t len) {
    slots = to_lds(sl);
    src = to_glb(s);
    n = len;
    nch = (len + CH - 1) / CH;
    load(0);
    store(0);
    load(1);
    store(1);
    next = 2;
    load(2);
  }
  // Makes the chunks up to the one after the chunk of key i resident (the
  // slot it takes held a chunk at least three below).
  __device__ __forceinline__ void advance(uint32_t i) {
    if (next < nch && next <= i / CH + 1) {
      store(next);
      ++next;
      load(next);
    }
  }
};
struct GLds {
  const lds64* p;
  __device__ __forceinline__ uint64_t operator[](uint32_t i) const { return p[i]; }
};
using lds_gs = __attribute__((address_space(3))) GroupShared;

// out = A XOR B by the whole workgroup, in steps of GNW * 64 * P positions;
// pre(ia, ib) runs at the start of each step (the keys of A and B consumed so
// far) to make what the step reads resident.  Returns the number written.
template <int P, class AA, class BB, class O, class Pre>
__device__ __forceinline__ uint32_t g_merge(const AA& A, uint32_t na, const BB& B, uint32_t nb, O* out, lds_gs* G,
                                            int lane, Pre pre) {
  constexpr uint32_t D = GNW * 64 * P;
  const uint32_t wv = threadIdx.x >> 6;
  const uint32_t total = na + nb;
  uint32_t d0 = 0, ia0 = 0, ib0 = 0, o = 0;
  while (d0 < total) {
    pre(ia0, ib0);
    __syncthreads();
    const uint32_t d1 = total - d0 < D ? total : d0 + D;
    const uint32_t mine = d0 + (wv * 64 + (uint32_t)lane + 1) * P;
    const uint32_t dend = mine < d1 ? mine : d1;
    const uint32_t ie = g_split(A, na, B, nb, dend, d0, ia0);
    uint32_t je = dend - ie;
    if (ie > 0 && je < nb && A[ie - 1] == B[je]) ++je;
    uint32_t is = __shfl_up(ie, 1, 64), js = __shfl_up(je, 1, 64);
    if (lane == 0) {
      if (wv == 0) {
        is = ia0;
        js = ib0;
      } else {  // where the previous wavefront's last lane ends
        const uint32_t ws = d0 + wv * 64 * P;
        const uint32_t ds = ws < d1 ? ws : d1;
        is = g_split(A, na, B, nb, ds, d0, ia0);
        js = ds - is;
        if (is > 0 && js < nb && A[is - 1] == B[js]) ++js;
      }
    }
    uint32_t i = is, j = js;
    uint64_t a = i < ie ? A[i] : KEY_INF;
    uint64_t b = j < je ? B[j] : KEY_INF;
    uint64_t buf[P + 1];
    uint32_t keep = 0;
#pragma unroll
    for (int t = 0; t <= P; ++t) {
      buf[t] = 0;
      if (a < b) {
        buf[t] = a;
        keep |= 1u << t;
        ++i;
        a = i < ie ? A[i] : KEY_INF;
      } else if (b < a) {
        buf[t] = b;
        keep |= 1u << t;
        ++j;
        b = j < je ? B[j] : KEY_INF;
      } else if (a != KEY_INF) {
        ++i;
        ++j;
        a = i < ie ? A[i] : KEY_INF;
        b = j < je ? B[j] : KEY_INF;
      }
    }
    uint32_t wtot;
    uint32_t pos = w_excl_small<(P < 8 ? 3 : (P < 16 ? 4 : 5))>((uint32_t)__popc(keep), &wtot);
    if (lane == 0) G->cnt[wv] = wtot;
    if (wv == GNW - 1 && lane == 63) {
      G->end_a = ie;
      G->end_b = je;
    }
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (uint32_t w = 0; w < (uint32_t)GNW; ++w) {
      const uint32_t cw = G->cnt[w];
      before += w < wv ? cw : 0u;
      sum += cw;
    }
    pos += o + before;
#pragma unroll
    for (int t = 0; t <= P; ++t)
      if (keep & (1u << t)) out[pos++] = buf[t];
    o += sum;
    ia0 = G->end_a;
    ib0 = G->end_b;
    d0 = d1;
  }
  __syncthreads();
  return uni(o);
}

// Runs operation d with the whole workgroup; returns the keys written.
__device__ __noinline__ uint32_t g_run(const WaveBufs& S, uint32_t op, uint32_t na, uint32_t nb, uint64_t a,
                                       uint64_t b, uint64_t out, int lane) {
  lds_gs* G = (lds_gs*)gshared(S);
  lds64* L = to_lds(S.F0);  // the start of the group's LDS
  if (op == G_MERGE_LDS) {
    return g_merge<GP_LDS>(GLds{L + a}, na, GLds{L + b}, nb, L + out, G, lane, [](uint32_t, uint32_t) {});
  }
  if (op == G_MERGE_TAIL || op == G_MERGE_TAIL_LDS) {  // the output in the arena, or in LDS
    GRing<GP_TAIL> ra;
    ra.init(S.X, reinterpret_cast<const uint64_t*>(a), na);
    auto adv = [&](uint32_t ia, uint32_t) { ra.advance(ia); };
    if (op == G_MERGE_TAIL)
      return g_merge<GP_TAIL>(ra, na, GLds{L + b}, nb, to_glb(reinterpret_cast<uint64_t*>(out)), G, lane, adv);
    return g_merge<GP_TAIL>(ra, na, GLds{L + b}, nb, L + out, G, lane, adv);
  }
  if (op == G_MERGE_GG) {
    GRing<GP_GG> ra, rb;
    ra.init(S.X, reinterpret_cast<const uint64_t*>(a), na);
    rb.init(S.X + GXN / 2, reinterpret_cast<const uint64_t*>(b), nb);
    return g_merge<GP_GG>(ra, na, rb, nb, to_glb(reinterpret_cast<uint64_t*>(out)), G, lane,
                          [&](uint32_t ia, uint32_t ib) {
                            ra.advance(ia);
                            rb.advance(ib);
                          });
  }
  if (op == G_FENCE) {  // every wavefront's global stores have reached the L2 (vmcnt(0))
    __builtin_amdgcn_s_waitcnt(0xF70);
    __syncthreads();
    return 0;
  }
  if (op == G_COPY_IN) {
    const glb64* src = to_glb(reinterpret_cast<const uint64_t*>(a));
    for (uint32_t i = threadIdx.x; i < na; i += GNW * 64) L[out + i] = src[i];
  } else {  // G_COPY_OUT
    glb64* dst = to_glb(reinterpret_cast<uint64_t*>(out));
    for (uint32_t i = threadIdx.x; i < na; i += GNW * 64) dst[i] = L[a + i];
  }
  __syncthreads();
  return na;
}

// The leader posts an operation and runs it with the other wavefronts.
__device__ __forceinline__ uint32_t g_issue(const WaveBufs& S, uint32_t op, uint32_t na, uint32_t nb, uint64_t a,
                                            uint64_t b, uint64_t out, int lane) {
  GroupShared* G = gshared(S);
  if (lane == 0) {
    G->desc.op = op;
    G->desc.na = na;
    G->desc.nb = nb;
    G->desc.a = a;
    G->desc.b = b;
    G->desc.out = out;
  }
  __syncthreads();
  return uni(g_run(S, op, na, nb, a, b, out, lane));
}
__device__ __forceinline__ uint64_t loff(const WaveBufs& S, const uint64_t* p) { return (uint64_t)(p - S.F0); }
__device__ __forceinline__ uint64_t gaddr(const uint64_t* p) { return (uint64_t)(uintptr_t)p; }

// T ^= U (U becomes empty).
__device__ __forceinline__ bool g_fold_mid(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
  if (W.U.n == 0) return true;
  if (W.T.n == 0) {
    W.T = W.U;
  } else {
    const uint64_t off = w_alloc(R, (uint64_t)W.T.n + W.U.n, lane);
    if (off == ~0ull) return false;
    const uint32_t len = g_issue(S, G_MERGE_GG, W.T.n, W.U.n, gaddr(W.T.v), gaddr(W.U.v), gaddr(R.arena + off), lane);
    w_count(W.merged, W.T.n + W.U.n, lane);
    tail_set(W.T, R.arena + off, len, lane);
  }
  W.U.n = 0;
  return true;
}

// U ^= F (F becomes empty), folding U into T first if U would outgrow mid_cap.
__device__ __forceinline__ bool g_push_front(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
  if (W.nf == 0) return true;
  if (W.U.n + W.nf > cold(R)->mid_cap && !g_fold_mid(R, S, W, lane)) return false;
  const uint64_t off = w_alloc(R, (uint64_t)W.U.n + W.nf, lane);
  if (off == ~0ull) return false;
  const uint32_t len = g_issue(S, G_MERGE_TAIL, W.U.n, W.nf, gaddr(W.U.v), loff(S, fbuf(S, W.cur)),
                               gaddr(R.arena + off), lane);
  w_count(W.merged, W.U.n + W.nf, lane);
  W.nf = 0;
  tail_set(W.U, R.arena + off, len, lane);
  return true;
}

// F ^= X[0..m) (X in LDS), pushing F into U first if the result might not fit.
__device__ __forceinline__ bool g_front_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* X,
                                            uint32_t m, int lane) {
  if (W.nf + m > S.cap && !g_push_front(R, S, W, lane)) return false;
  w_count(W.merged, W.nf + m, lane);
  W.nf = g_issue(S, G_MERGE_LDS, W.nf, m, loff(S, fbuf(S, W.cur)), loff(S, X), loff(S, fbuf(S, W.cur ^ 1)), lane);
  W.cur ^= 1;
  return true;
}

// Adds a sorted arena list Q[0..m) (an owner column): as w_owner_add.
__device__ __forceinline__ bool g_owner_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* Q,
                                            uint32_t m, int lane) {
  if (2 * m > S.cap) {
    if (W.U.n + m > cold(R)->mid_cap && !g_fold_mid(R, S, W, lane)) return false;
    if (W.U.n == 0) {
      tail_set(W.U, Q, m, lane);
      return true;
    }
    const uint64_t off = w_alloc(R, (uint64_t)W.U.n + m, lane);
    if (off == ~0ull) return false;
    const uint32_t len = g_issue(S, G_MERGE_GG, W.U.n, m, gaddr(W.U.v), gaddr(Q), gaddr(R.arena + off), lane);
    w_count(W.merged, W.U.n + m, lane);
    tail_set(W.U, R.arena + off, len, lane);
    return true;
  }
  if (W.nf + m > S.cap && !g_push_front(R, S, W, lane)) return false;
  w_count(W.merged, W.nf + m, lane);
  W.nf = g_issue(S, G_MERGE_TAIL_LDS, m, W.nf, gaddr(Q), loff(S, fbuf(S, W.cur)), loff(S, fbuf(S, W.cur ^ 1)), lane);
  W.cur ^= 1;
  return true;
}

// F ^= P (P becomes empty).
__device__ __forceinline__ bool g_flush_p(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
  if (W.np == 0) return true;
  p_stage(W, S.ps, lane);
  const uint32_t np = W.np;
  W.np = 0;
  return g_front_add(R, S, W, S.ps, np, lane);
}

__device__ __forceinline__ bool g_insert3(const RedCtx& R, const WaveBufs& S, WState& W, uint64_t k0, uint64_t k1,
                                          uint64_t k2, int lane) {
  if (W.np > PCAP - 3 && !g_flush_p(R, S, W, lane)) return false;
  p_insert3(S, W, k0, k1, k2, lane);
  return true;
}

// The leader's side of the column steps.
struct GroupOps {
  static constexpr bool kAsync = false;
  __device__ static bool fresh(const RedCtx&, uint32_t) { return false; }
  __device__ static bool leader(int lane) { return lane == 0; }
  __device__ static uint32_t round(const RedCtx& R) { return cold(R)->round; }
  __device__ static uint32_t wave_yield(const RedCtx& R) { return cold(R)->wave_yield; }
  __device__ static bool aborted(const RedCtx& R, const WaveBufs&) { return cr::aborted(cold(R)->st); }
  __device__ static uint64_t alloc(const RedCtx& R, const WaveBufs&, uint64_t n, int lane) { return w_alloc(R, n, lane); }
  __device__ static bool insert3(const RedCtx& R, const WaveBufs& S, WState& W, uint64_t k0, uint64_t k1, uint64_t k2,
                                 int lane) {
    return g_insert3(R, S, W, k0, k1, k2, lane);
  }
  __device__ static bool flush_p(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
    return g_flush_p(R, S, W, lane);
  }
  __device__ static bool push_front(const RedCtx& R, const WaveBufs& S, WState& W, int lane) {
    return g_push_front(R, S, W, lane);
  }
  __device__ static bool front_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* X, uint32_t m,
                                   int lane) {
    return g_front_add(R, S, W, X, m, lane);
  }
  __device__ static uint32_t merge_tail(const WaveBufs& S, const uint64_t* T, uint32_t nt, const uint64_t* F,
                                        uint32_t nf, uint64_t* out, int lane) {
    return g_issue(S, G_MERGE_TAIL, nt, nf, gaddr(T), loff(S, F), gaddr(out), lane);
  }
  __device__ static uint32_t merge_gg(const WaveBufs& S, const uint64_t* A, uint32_t na, const uint64_t* B,
                                      uint32_t nb, uint64_t* out, int lane) {
    return g_issue(S, G_MERGE_GG, na, nb, gaddr(A), gaddr(B), gaddr(out), lane);
  }
  __device__ static void copy_in(const WaveBufs& S, uint64_t* dst, const uint64_t* src, uint32_t n, int lane) {
    g_issue(S, G_COPY_IN, n, 0, gaddr(src), 0, loff(S, dst), lane);
  }
  __device__ static void copy_out(const WaveBufs& S, uint64_t* dst, const uint64_t* src, uint32_t n, int lane) {
    g_issue(S, G_COPY_OUT, n, 0, loff(S, src), 0, gaddr(dst), lane);
  }
  __device__ static bool owner_add(const RedCtx& R, const WaveBufs& S, WState& W, const uint64_t* Q, uint32_t m,
                                   int lane) {
    return g_owner_add(R, S, W, Q, m, lane);
  }
};

// Group-mode round over the same lists as the wave-mode round, when they hold
// at most R.group_max columns (the wave-mode kernels return at once then).
// R must stay the first parameter (see cold()).
__global__ __launch_bounds__(64 * GNW) void k_red_round_group(RedCtx R, const uint32_t* __restrict__ list_s,
                                                             const unsigned long long* __restrict__ n_s,
                                                             const uint32_t* __restrict__ list_l,
                                                             const unsigned long long* __restrict__ n_l,
                                                             uint32_t front_cap) {
  extern __shared__ __align__(16) uint64_t lds_words[];
  if (in_tail(R, n_s, 0)) return;
  const uint64_t nl = uni64(*n_l), ns0 = uni64(*n_s);
  const uint64_t ns = ns0 <= R.wave_short ? ns0 : 0;
  if (nl + ns == 0 || nl + ns > R.group_max) return;
  const bool few = nl + ns <= R.yield_few;
  const int lane = threadIdx.x & 63;
  WaveBufs S;
  S.cap = front_cap;
  S.F0 = lds_words;
  S.F1 = S.F0 + S.cap;
  S.X = S.F1 + S.cap;
  S.ps = S.X + GXN;
  S.hx = S.ps + PCAP;
  S.po = S.hx + 64;
  GroupShared* G = gshared(S);
  if (threadIdx.x >= 64) {  // helpers: run what the leader posts until it posts the end
    for (;;) {
      __syncthreads();
      const uint32_t op = uni(G->desc.op);
      if (op == G_END) return;
      g_run(S, op, uni(G->desc.na), uni(G->desc.nb), uni64(G->desc.a), uni64(G->desc.b), uni64(G->desc.out), lane);
    }
  }
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  WState W;
  W.adds = 0;
  W.merged = 0;
  for (;;) {
    unsigned long long li = 0;
    if (lane == 0) li = atomicAdd(R.work, 1ull);
    li = rdlane64(li, 0);
    if (li >= nl + ns || aborted(R.st)) break;
    const uint32_t c = uni(li < nl ? list_l[li] : list_s[li - nl]);
    reduce_column<GroupOps>(R, S, W, c, off2, lane, few, ColStart{cold(R)->col_ptr[c], 0, 0, false});
    wsync();
  }
  if (lane == 0) G->desc.op = G_END;
  __syncthreads();
  if (lane == 0 && W.adds) {
    atomicAdd(&R.st->adds, W.adds);
    atomicAdd(&R.st->merged, W.merged);
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
// wave-mode list).  Yielded columns were already listed.
// It also clears the counts the round after next will fill (nobody reads them
// during this round) and the wave-mode column counter, so that no separate
// launch is needed for them.
// A workgroup collects what it appends in LDS and reserves room in a list with
// one atomic per COMMIT_BUF entries: one atomic per wavefront on the two shared
// counts serialised the first round's commit (~1.2 ms of 6.2M columns).
constexpr int COMMIT_TPB = 256;    // threads per workgroup of the commit
constexpr int COMMIT_BUF = 2048;   // entries of each LDS list buffer
__global__ __launch_bounds__(COMMIT_TPB) void k_red_commit(RedCtx R, const uint32_t* __restrict__ list_t,
                                                          const unsigned long long* __restrict__ n_t,
                                                          const uint32_t* __restrict__ list_b,
                                                          const unsigned long long* __restrict__ n_b, int first,
                                                          uint32_t* next_t, uint32_t* next_b,
                                                          unsigned long long* __restrict__ n_next,
                                                          unsigned long long* __restrict__ n_clear) {
  __shared__ uint32_t buf[2][COMMIT_BUF];
  __shared__ uint32_t cnt[2];
  __shared__ unsigned long long base[2];
  __shared__ uint32_t stop;
  // one reading of the abort flag for the whole workgroup (it has barriers)
  if (threadIdx.x == 0) stop = aborted(R.st) ? 1u : 0u;
  __syncthreads();
  if (stop) return;
  if (in_tail(R, n_t, first)) {  // nothing proposed; the counts stay for the tail
    if (blockIdx.x == 0 && threadIdx.x == 0 && R.st->tail_round == 0) {
      R.st->tail_round = R.round + 1;
      *R.async_base = *R.arena_top;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *R.async_base = *R.arena_top;  // the tail's, should it start after this round
    n_clear[0] = 0;
    n_clear[1] = 0;
    R.work[0] = 0;
  }
  const bool sp = first && R.spatial && *R.n_spatial;  // then the spatial order is listed
  const uint64_t nt = first ? (sp ? *R.n_spatial : R.dim_count[2]) : *n_t;
  const uint64_t nb = first ? 0 : *n_b;
  if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * COMMIT_TPB;
  const uint64_t nr = (nt + nb + COMMIT_TPB - 1) / COMMIT_TPB * COMMIT_TPB;  // the same passes for a whole workgroup
  uint32_t* next[2] = {next_t, next_b};
  for (uint64_t i0 = (uint64_t)blockIdx.x * COMMIT_TPB; i0 < nr; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    if (i < nt + nb) {
      uint32_t c;
      bool skip = false;
      if (i < nt) {
        const uint64_t sk = sp ? R.spatial[i] : 0;
        c = first ? (sp ? (uint32_t)(sk >> 32) : (uint32_t)i) : list_t[i];
        skip = first && (sp ? spatial_none(R, sk) : R.cleared[c] != 0);
      } else {
        c = list_b[i - nt];
      }
      const uint64_t e = skip ? YIELDED : R.piv[c];
      if (e != YIELDED) {
        const int64_t slot = pivot_slot(R, e);
        bool push = true;
        uint32_t again = c;
        if (R.claim[slot] == claim_word(R.round, c)) {
          const uint64_t old = R.owner[slot];
          R.owner[slot] = ((uint64_t)c << 32) | R.col_ptr[c];
          push = old != NO_OWNER;
          again = (uint32_t)(old >> 32);
        }
        if (push) {
          const int b = R.arena[R.col_ptr[again]] > R.long_len ? 1 : 0;
          buf[b][atomicAdd(&cnt[b], 1u)] = again;
        }
      }
    }
    __syncthreads();
    // empty a buffer that the next pass could overflow, and both after the last
    const bool last = i0 + stride >= nr;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint32_t k = cnt[b];
      if (k + COMMIT_TPB > (uint32_t)COMMIT_BUF || (last && k)) {
        if (threadIdx.x == 0) base[b] = atomicAdd(&n_next[b], (unsigned long long)k);
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < k; j += COMMIT_TPB) next[b][base[b] + j] = buf[b][j];
        __syncthreads();
        if (threadIdx.x == 0) cnt[b] = 0;
        __syncthreads();
      }
    }
  }
}

// ---- the asynchronous tail -------------------------------------------------------
//
// In rounds of few columns, every round waits for its longest column, and a
// column that lost a claim waits for the next round.  The tail reduces the
// columns still listed without rounds: each workgroup (eight wavefronts, as in
// group mode) takes a listed column and reduces it to its end -- adding, while
// the pivot is owned by a column to its left, that column's stored list -- and
// then claims the pivot's owner word with a compare-and-swap:
//   * the word was free: the column owns the pivot;
//   * it held a column to the right: the column owns it, and the displaced one
//     (parked as an owner until then, so active nowhere else) is reduced next
//     by the same workgroup, starting with the new owner's list;
//   * it changed meanwhile to a column to the left: the column adds that one
//     and goes on.
// An owner word only ever names a column holding that pivot, and its list (a
// sum of columns no further right, immutable) is a valid addition for every
// column to the right of it; a claim fails only when another one succeeded.  So
// the tail ends in a reduced matrix with the pivots of the sequential
// reduction, in any order of events.  Owner words are read with plain loads
// while reducing: a stale one costs at most a failed claim, whose returned word
// is then used instead.  A list stored during the tail reaches the device's
// L2 (every wavefront waits for its stores) and is written back from there
// (release) before its owner word is swapped in, and a reader acquires before
// reading it.
__shared__ uint32_t async_base_lds;

struct AsyncOps : GroupOps {
  static constexpr bool kAsync = true;
  __device__ static uint32_t wave_yield(const RedCtx&) { return 0u; }
  __device__ static bool fresh(const RedCtx&, uint32_t off) { return off >= async_base_lds; }
};

// R must stay the first parameter (see cold()).
__global__ __launch_bounds__(64 * GNW) void k_red_async(RedCtx R, const uint32_t* __restrict__ l0,
                                                       const uint32_t* __restrict__ l1,
                                                       const uint32_t* __restrict__ l2,
                                                       const uint32_t* __restrict__ l3,
                                                       const unsigned long long* __restrict__ counts,
                                                       uint32_t round_end, uint32_t front_cap) {
  extern __shared__ __align__(16) uint64_t lds_words[];
  // what every thread reads before the split into leader and helpers must be
  // the same for all of them: words that no kernel running now writes
  const uint32_t tr = R.st->tail_round;
  const uint32_t r = tr ? tr - 1 : round_end;  // the round whose lists are left
  const unsigned long long* ct = counts + 2 * (r % 3);
  const uint64_t ns = uni64(ct[0]), nl = uni64(ct[1]);
  if (ns + nl == 0) return;
  const uint32_t* list_s = (r & 1) ? l2 : l0;
  const uint32_t* list_l = (r & 1) ? l3 : l1;
  const int lane = threadIdx.x & 63;
  WaveBufs S;
  S.cap = front_cap;
  S.F0 = lds_words;
  S.F1 = S.F0 + S.cap;
  S.X = S.F1 + S.cap;
  S.ps = S.X + GXN;
  S.hx = S.ps + PCAP;
  S.po = S.hx + 64;
  GroupShared* G = gshared(S);
  if (threadIdx.x >= 64) {  // helpers, as in group mode
    for (;;) {
      __syncthreads();
      const uint32_t op = uni(G->desc.op);
      if (op == G_END) return;
      g_run(S, op, uni(G->desc.na), uni(G->desc.nb), uni64(G->desc.a), uni64(G->desc.b), uni64(G->desc.out), lane);
    }
  }
  if (lane == 0) async_base_lds = (uint32_t)*R.async_base;
  wsync();
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  WState W;
  W.adds = 0;
  W.merged = 0;
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  uint32_t c = NONE;
  ColStart from{0, 0, 0, false};
  for (;;) {
    if (c == NONE) {  // the next listed column
      unsigned long long li = 0;
      if (lane == 0) li = atomicAdd(R.work, 1ull);
      li = rdlane64(li, 0);
      if (li >= nl + ns || aborted(R.st)) break;
      c = uni(li < nl ? list_l[li] : list_s[li - nl]);
      from = ColStart{uni64(R.col_ptr[c]), 0, 0, false};
    }
    ColEnd end{0, 0, nullptr};
    const uint64_t off = reduce_column<AsyncOps>(R, S, W, c, off2, lane, true, from, &end);
    if (off == ~0ull) break;  // a raised flag: the call reports it
    if (end.slot == nullptr) {  // cannot happen: the tail's columns do not yield
      if (lane == 0) raise_flag(R.st, &R.st->internal);
      break;
    }
    g_issue(S, G_FENCE, 0, 0, 0, 0, 0, lane);
    const uint64_t mine = ((uint64_t)c << 32) | off;
    uint64_t old = 0;
    uint32_t lost = 0;
    if (lane == 0) {
      __hip_atomic_store(&R.piv[c], end.e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&R.col_ptr[c], off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint64_t seen = end.ow;
      for (;;) {
        uint64_t cur = seen;
        // release: the list (and piv, col_ptr) before the word; acquire where a
        // list named by the returned word is read
        if (__hip_atomic_compare_exchange_strong(end.slot, &cur, mine, __ATOMIC_RELEASE, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
          old = seen;
          break;
        }
        if (cur != NO_OWNER && (uint32_t)(cur >> 32) < c) {  // a column to the left got there first
          old = cur;
          lost = 1;
          break;
        }
        seen = cur;
      }
    }
    old = uni64(rdlane64(old, 0));
    lost = uni((uint32_t)__builtin_amdgcn_readlane((int)lost, 0));
    if (lost) {  // add that column (the pivot's word is known) and go on
      from = ColStart{off, end.e, old, false};
    } else if (old != NO_OWNER) {  // reduce the displaced column next, from its stored list
      if ((uint32_t)old >= async_base_lds) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t j = (uint32_t)(old >> 32);
      from = ColStart{(uint32_t)old, end.e, mine, true};
      c = j;
    } else {
      c = NONE;
    }
  }
  if (lane == 0) G->desc.op = G_END;
  __syncthreads();
  if (lane == 0 && W.adds) {
    atomicAdd(&R.st->adds, W.adds);
    atomicAdd(&R.st->merged, W.merged);
  }
}

// Degree-1 rows of a volume: column c pairs its final pivot edge (birth) with
// its square (death).
__global__ void k_h1_emit(RedCtx R, EmitCtx E) {
  if (aborted_block(R.st)) return;
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  const uint64_t n2 = R.dim_count[2];
  emit_tiled(E, n2, [&](uint64_t c, int* im, uint64_t* ck) {
    if (R.cleared[c]) return false;
    const uint64_t e = R.piv[c];
    const ImgDesc d = R.imgs[skey_img(R.L, e)];
    int ec[3];
    kidx_coords(d, skey_kidx(R.L, e), ec);
    const uint64_t ow = R.owner[edge_slot(d, ec)];
    if (ow == NO_OWNER || (uint32_t)(ow >> 32) != (uint32_t)c) {
      raise_flag(R.st, &R.st->internal);
      return false;
    }
    return pair_row(E, e, R.skeys[off2 + c], false, im, ck);
  });
}

RedCtx make_redctx(const float* img, const ImgDesc* imgs, Layout L, const uint64_t* skeys,
                   const unsigned long long* dim_count, const uint8_t* cleared, const uint8_t* eapp,
                   uint64_t* owner, uint64_t* claim,
                   uint64_t* piv, uint64_t* col_ptr, uint64_t* arena, uint64_t arena_cap,
                   unsigned long long* arena_top, unsigned long long* work, Status* st) {
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
  R.work = work;
  R.st = st;
  R.long_len = THREAD_CAP;
  R.yield_iters = 1024;
  R.wave_short = 4096;
  R.front_cap = 1024;
  R.mid_cap = 8192;
  R.narrow_min = 8192;
  R.narrow_cap = 256;
  R.group_max = 1024;
  R.group_cap = 2048;
  R.wave_yield = 0;
  R.yield_few = 2;
  R.yield_list = nullptr;
  R.yield_count = nullptr;
  R.round = 0;
  R.async_max = 0;
  R.async_base = nullptr;
  R.spatial = nullptr;
  R.n_spatial = nullptr;
  return R;
}

// Dynamic LDS bytes of a wave-mode workgroup, and the grid: as many
// workgroups as fit the CUs at once (at most eight per CU).
template <class C>
static size_t wave_setup(uint32_t front_cap, int ncu, int* grid) {
  const size_t lds = WPB * 8 * wave_lds_words<C>(front_cap);
  static size_t lds_set = 0;
  if (lds_set < lds) {
    (void)hipFuncSetAttribute((const void*)k_red_round_wave<C>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    lds_set = lds;
  }
  const int fit = (int)(160 * 1024 / lds);
  *grid = ncu * (fit < 1 ? 1 : (fit > 8 ? 8 : fit));
  return lds;
}

void launch_h1_rounds(int grid, const RedCtx& R, uint32_t* lists[4], unsigned long long* counts, int round0,
                      int nrounds, int yield_rounds, hipStream_t s) {
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int wgrid = 0, ngrid = 0;
  const size_t lds = wave_setup<WideCfg>(R.front_cap, ncu, &wgrid);
  const size_t nlds = wave_setup<NarrowCfg>(R.narrow_cap, ncu, &ngrid);
  const uint32_t gcap = R.group_cap < FRONT_CAP_GROUP_MAX ? R.group_cap : FRONT_CAP_GROUP_MAX;
  const size_t glds = group_lds_bytes(gcap);
  static size_t glds_set = 0;
  if (glds_set < glds) {
    (void)hipFuncSetAttribute((const void*)k_red_round_group, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
    glds_set = glds;
  }
  for (int r = round0; r < round0 + nrounds; ++r) {
    const int cur = r & 1, nxt = (r + 1) & 1;  // list pairs alternate; count pairs rotate by three
    const int first = r == 0;
    // lists[2*k + 0] short (thread mode), lists[2*k + 1] long (wave mode); counts likewise
    uint32_t* lt = lists[2 * cur];
    uint32_t* lb = lists[2 * cur + 1];
    unsigned long long* ct = counts + 2 * (r % 3);
    unsigned long long* cnx = counts + 2 * ((r + 1) % 3);
    unsigned long long* cclr = counts + 2 * ((r + 2) % 3);
    RedCtx Rr = R;  // this round's number; columns that yield go to its next long list
    Rr.round = (uint32_t)r;
    Rr.yield_list = lists[2 * nxt + 1];
    Rr.yield_count = cnx + 1;
    if (r >= yield_rounds) Rr.wave_yield = 0;
    if (first)
      k_red_round<THREAD_CAP_FIRST><<<grid, 256, 0, s>>>(Rr, lt, ct, first, lists[2 * nxt], cnx, lists[2 * nxt + 1],
                                                         cnx + 1);
    else
      k_red_round<THREAD_CAP><<<grid, 256, 0, s>>>(Rr, lt, ct, first, lists[2 * nxt], cnx, lists[2 * nxt + 1], cnx + 1);
    if (!first) {
      k_red_round_wave<NarrowCfg><<<ngrid, 64 * WPB, nlds, s>>>(Rr, lt, ct, lb, ct + 1, R.narrow_cap);
      k_red_round_wave<WideCfg><<<wgrid, 64 * WPB, lds, s>>>(Rr, lt, ct, lb, ct + 1, R.front_cap);
      k_red_round_group<<<ncu, 64 * GNW, glds, s>>>(Rr, lt, ct, lb, ct + 1, gcap);
    }
    k_red_commit<<<grid, COMMIT_TPB, 0, s>>>(Rr, lt, ct, lb, ct + 1, first, lists[2 * nxt], lists[2 * nxt + 1], cnx,
                                             cclr);
  }
}

void launch_h1_async(const RedCtx& R, uint32_t* lists[4], unsigned long long* counts, int round_end, hipStream_t s) {
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t gcap = R.group_cap < FRONT_CAP_GROUP_MAX ? R.group_cap : FRONT_CAP_GROUP_MAX;
  const size_t glds = group_lds_bytes(gcap);
  static size_t glds_set = 0;
  if (glds_set < glds) {
    (void)hipFuncSetAttribute((const void*)k_red_async, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
    glds_set = glds;
  }
  k_red_async<<<ncu, 64 * GNW, glds, s>>>(R, lists[0], lists[1], lists[2], lists[3], counts, (uint32_t)round_end,
                                          gcap);
}

// The first round's spatial order: threads that reduce squares next to each
// other in the grid read the same cache lines of pixels, partner codes and
// owner words, where in rank order (by value) they read scattered ones.
// One key per column, in place (no compaction: a shared counter would serialise
// the wavefronts); a cleared column gets the all-ones field, which no square
// has (a Khalimsky index is below 2^kb - 1), so it sorts last and is skipped.
__global__ void k_red_spatial_keys(RedCtx R, uint64_t* __restrict__ out, uint64_t cap,
                                   unsigned long long* __restrict__ n_out) {
  if (aborted(R.st)) return;
  const uint64_t off2 = R.dim_count[0] + R.dim_count[1];
  const uint64_t n2 = R.dim_count[2];
  const bool fits = n2 <= cap && R.L.ib + R.L.kb <= 32;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = fits ? n2 : 0;
  if (!fits) return;
  const uint64_t none = (1ull << (R.L.ib + R.L.kb)) - 1;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n2; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t f = none;
    if (!R.cleared[i]) {
      const uint64_t k = R.skeys[off2 + i];
      f = ((uint64_t)skey_img(R.L, k) << R.L.kb) | skey_kidx(R.L, k);
    }
    out[i] = (i << 32) | f;
  }
}


void launch_h1_spatial_keys(int grid, const RedCtx& R, uint64_t* out, uint64_t cap, unsigned long long* n_out,
                            hipStream_t s) {
  k_red_spatial_keys<<<grid, 256, 0, s>>>(R, out, cap, n_out);
}

void launch_h1_emit(int grid, const RedCtx& R, const EmitCtx& E, hipStream_t s) {
  k_h1_emit<<<grid, 256, 0, s>>>(R, E);
}

}  // namespace cr
