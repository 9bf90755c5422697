// LSD radix sort of 64-bit keys (key only), 8-bit digits.
//
// The number of keys lives in device memory, so the sort can be enqueued before
// the count is known (and captured in a graph).  Per digit position, over
// tiles of 2048 keys, with the per-tile digit counts stored tile-major (one
// contiguous row of 256 counts per tile, so every kernel reads and writes them
// in whole rows):
//   count      -- per tile, the number of keys of each digit;
//   scan_block -- per block of SBT tiles and digit, the counts become the
//                 number of keys of that digit in the block's earlier tiles,
//                 and the block's totals are recorded;
//   scan_top   -- one workgroup: the block totals become the keys of each
//                 digit in the earlier blocks, and the digit totals the start
//                 of every digit's bucket;
//   scatter    -- each tile is ranked by digit with wavefront ballots (stable:
//                 wavefront, step, then lane order), sorted by digit in LDS
//                 and written out in runs of equal digits, so the stores are
//                 contiguous.
#include "cr_internal.h"

namespace cr {

constexpr int ST = 256;               // threads of a pass workgroup
constexpr int SKEYS = 8;              // keys per thread per tile (2048-key tiles: the scatter's
                                      // LDS lets seven workgroups share a CU; 4096-key tiles: 1.15 ->
                                      // 1.04 ms per 256^3 cell sort)
constexpr int STILE = ST * SKEYS;     // keys per tile
constexpr int SWAVES = ST / 64;
constexpr int SGRID = 2048;           // persistent workgroups of a scatter pass
constexpr int CGRID = 2048;           // ... of a count pass (small LDS: eight per CU)
constexpr int SBT = 64;               // tiles per block of the count scan

__device__ __forceinline__ uint64_t n_keys(const unsigned long long* n_ptr, uint64_t cap) {
  return *n_ptr < cap ? *n_ptr : cap;
}

// Ranks the keys of one tile by digit: wavefront w takes keys
// [w*SKEYS*64, (w+1)*SKEYS*64) of the tile, 64 per step; rank[j] = number of earlier keys of the same digit
// among this wavefront's keys; S.cnt[w][d] ends as the wavefront's count of d.
struct SortLds {
  uint64_t sk[STILE];         // the tile, sorted by digit
  uint32_t cnt[SWAVES][256];  // per-wavefront digit counts, then their exclusive offsets
  uint32_t tdig[256];         // exclusive start of each digit in the sorted tile
  uint32_t gpos[256];         // global position of the tile's first key of each digit
  uint32_t wsum[SWAVES];
};

__device__ __forceinline__ void rank_tile(SortLds& S, const uint64_t* __restrict__ in, uint64_t t0, uint32_t tcount,
                                          int shift, uint64_t key[SKEYS], uint32_t rank[SKEYS]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
  for (int j = 0; j < SKEYS; ++j) {
    const uint32_t li = (uint32_t)(w * (SKEYS * 64) + j * 64 + lane);
    key[j] = li < tcount ? in[t0 + li] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < SKEYS; ++j) {
    const uint32_t li = (uint32_t)(w * (SKEYS * 64) + j * 64 + lane);
    const bool valid = li < tcount;
    const uint32_t dig = (uint32_t)(key[j] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (dig >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t r = (uint32_t)__popcll(peers & lt);
    const uint32_t base = valid ? S.cnt[w][dig] : 0u;
    rank[j] = base + r;
    if (valid && r == 0) S.cnt[w][dig] = base + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
}

// Per tile and digit: the number of keys, counts[tile * 256 + d].
// Its LDS is the per-wavefront counts only (4 KiB, not the scatter's tile), so
// that more workgroups share a CU and more loads are in flight.
__global__ __launch_bounds__(ST) void k_sort_count(const uint64_t* __restrict__ in,
                                                   const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                   int shift, uint32_t* __restrict__ counts) {
  struct CountLds {
    uint32_t cnt[SWAVES][256];
  };
  __shared__ CountLds S;
  const int tid = threadIdx.x;
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t ntiles = (n + STILE - 1) / STILE;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int i = 0; i < SWAVES; ++i) S.cnt[i][tid] = 0;
    __syncthreads();
    const uint64_t t0 = tile * STILE;
    const uint32_t tcount = (uint32_t)(n - t0 < (uint64_t)STILE ? n - t0 : (uint64_t)STILE);
    {  // only the histogram: one LDS add per key into the wavefront's counts
      const int lane = tid & 63, w = tid >> 6;
      uint32_t dig[SKEYS];
#pragma unroll
      for (int j = 0; j < SKEYS; ++j) {
        const uint32_t li = (uint32_t)(w * (SKEYS * 64) + j * 64 + lane);
        dig[j] = li < tcount ? (uint32_t)(in[t0 + li] >> shift) & 255u : 256u;
      }
#pragma unroll
      for (int j = 0; j < SKEYS; ++j)
        if (dig[j] < 256u) atomicAdd(&S.cnt[w][dig[j]], 1u);
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int i = 0; i < SWAVES; ++i) tot += S.cnt[i][tid];
    counts[tile * 256 + (uint64_t)tid] = tot;
    __syncthreads();
  }
}

// Per block b of SBT tiles (one workgroup each, thread d for digit d):
// counts[t * 256 + d] becomes the number of keys of digit d in the block's
// tiles before t, and bsum[b * 256 + d] the block's total of digit d.
__global__ __launch_bounds__(256) void k_sort_scan_block(uint32_t* __restrict__ counts,
                                                         const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                         uint32_t* __restrict__ bsum) {
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t ntiles = (n + STILE - 1) / STILE;
  const uint64_t t0 = (uint64_t)blockIdx.x * SBT;
  if (t0 >= ntiles) return;
  const uint64_t t1 = t0 + SBT < ntiles ? t0 + SBT : ntiles;
  const uint32_t nt = (uint32_t)(t1 - t0);
  uint32_t* c = counts + t0 * 256 + threadIdx.x;
  uint32_t v[SBT];  // all loads first, so that they are in flight together
#pragma unroll
  for (int i = 0; i < SBT; ++i) v[i] = (uint32_t)i < nt ? c[(uint64_t)i * 256] : 0u;
  uint32_t run = 0;
#pragma unroll
  for (int i = 0; i < SBT; ++i) {
    if ((uint32_t)i < nt) c[(uint64_t)i * 256] = run;
    run += v[i];
  }
  bsum[(uint64_t)blockIdx.x * 256 + threadIdx.x] = run;
}

// One workgroup, thread d for digit d: bsum[b * 256 + d] becomes the number of
// keys of digit d in the blocks before b, and bucket[d] the start of digit d's
// bucket (the keys of all smaller digits).
__global__ __launch_bounds__(256) void k_sort_scan_top(uint32_t* __restrict__ bsum,
                                                       const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                       uint32_t* __restrict__ bucket) {
  __shared__ uint32_t wsum[4];
  const int d = threadIdx.x, lane = d & 63, w = d >> 6;
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t nblocks = ((n + STILE - 1) / STILE + SBT - 1) / SBT;
  constexpr int BATCH = 16;  // loads in flight together
  uint32_t run = 0;
  for (uint64_t b0 = 0; b0 < nblocks; b0 += BATCH) {
    uint32_t v[BATCH];
#pragma unroll
    for (int i = 0; i < BATCH; ++i) v[i] = b0 + i < nblocks ? bsum[(b0 + i) * 256 + d] : 0u;
#pragma unroll
    for (int i = 0; i < BATCH; ++i) {
      if (b0 + i < nblocks) bsum[(b0 + i) * 256 + d] = run;
      run += v[i];
    }
  }
  uint32_t incl = run;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t up = __shfl_up(incl, off, 64);
    if (lane >= off) incl += up;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int i = 0; i < w; ++i) before += wsum[i];
  bucket[d] = before + incl - run;
}

// One pass: each tile is ranked again, sorted by digit in LDS and written out
// in runs of equal digits at the positions from k_sort_scan_tiles.
__global__ __launch_bounds__(ST) void k_sort_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                     const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                     int shift, const uint32_t* __restrict__ pos,
                                                     const uint32_t* __restrict__ bsum,
                                                     const uint32_t* __restrict__ bucket) {
  __shared__ SortLds S;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t ntiles = (n + STILE - 1) / STILE;
  const uint32_t start = bucket[tid];  // digit tid's bucket
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int i = 0; i < SWAVES; ++i) S.cnt[i][tid] = 0;
    __syncthreads();
    const uint64_t t0 = tile * STILE;
    const uint32_t tcount = (uint32_t)(n - t0 < (uint64_t)STILE ? n - t0 : (uint64_t)STILE);
    uint64_t key[SKEYS];
    uint32_t rank[SKEYS];
    rank_tile(S, in, t0, tcount, shift, key, rank);
    __syncthreads();
    // per digit: wavefront offsets, tile total, tile-wide exclusive start
    const int d = tid;
    uint32_t tot = 0;
    for (int i = 0; i < SWAVES; ++i) {
      const uint32_t c = S.cnt[i][d];
      S.cnt[i][d] = tot;
      tot += c;
    }
    uint32_t incl = tot;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t up = __shfl_up(incl, off, 64);
      if (lane >= off) incl += up;
    }
    if (lane == 63) S.wsum[w] = incl;
    S.gpos[d] = start + bsum[(tile / SBT) * 256 + (uint64_t)d] + pos[tile * 256 + (uint64_t)d];
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += S.wsum[i];
    S.tdig[d] = before + incl - tot;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SKEYS; ++j) {
      const uint32_t li = (uint32_t)(w * (SKEYS * 64) + j * 64 + lane);
      if (li < tcount) {
        const uint32_t dig = (uint32_t)(key[j] >> shift) & 255u;
        S.sk[S.tdig[dig] + S.cnt[w][dig] + rank[j]] = key[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < SKEYS; ++m) {
      const uint32_t i = (uint32_t)(tid + m * ST);
      if (i < tcount) {
        const uint64_t k = S.sk[i];
        const uint32_t dig = (uint32_t)(k >> shift) & 255u;
        out[(uint64_t)S.gpos[dig] + (i - S.tdig[dig])] = k;
      }
    }
    __syncthreads();
  }
}

// Scratch of launch_sort: per-tile counts and per-block totals.
size_t sort_scratch_bytes(uint64_t cap) {
  const uint64_t tiles = (cap + STILE - 1) / STILE + 1;
  const uint64_t blocks = (tiles + SBT - 1) / SBT + 1;
  return 4ull * 256 + 4ull * 256 * blocks + 4ull * tiles * 256 + 256;
}

// Sorts keys[0..min(*n, cap)) ascending on bits [0, bits); tmp is scratch of the same
// size.  Returns the buffer (keys or tmp) that holds the result.
uint64_t* launch_sort(uint64_t* keys, uint64_t* tmp, const unsigned long long* n_ptr, uint64_t cap, int bits,
                      void* scratch, hipStream_t stream) {
  const int passes = (bits + 7) / 8;
  const uint64_t max_tiles = (cap + STILE - 1) / STILE;
  const uint64_t max_blocks = (max_tiles + SBT - 1) / SBT;
  uint32_t* bucket = static_cast<uint32_t*>(scratch);
  uint32_t* bsum = bucket + 256;
  uint32_t* counts = bsum + 256 * (max_blocks + 1);
  const int grid = (int)(max_tiles < (uint64_t)SGRID ? (max_tiles ? max_tiles : 1) : (uint64_t)SGRID);
  const int cgrid = (int)(max_tiles < (uint64_t)CGRID ? (max_tiles ? max_tiles : 1) : (uint64_t)CGRID);
  const int bgrid = (int)(max_blocks ? max_blocks : 1);
  uint64_t* a = keys;
  uint64_t* b = tmp;
  for (int p = 0; p < passes; ++p) {
    k_sort_count<<<cgrid, ST, 0, stream>>>(a, n_ptr, cap, 8 * p, counts);
    k_sort_scan_block<<<bgrid, 256, 0, stream>>>(counts, n_ptr, cap, bsum);
    k_sort_scan_top<<<1, 256, 0, stream>>>(bsum, n_ptr, cap, bucket);
    k_sort_scatter<<<grid, ST, 0, stream>>>(a, b, n_ptr, cap, 8 * p, counts, bsum, bucket);
    uint64_t* t = a;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace cr
