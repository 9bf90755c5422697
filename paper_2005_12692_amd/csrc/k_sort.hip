// LSD radix sort of 64-bit keys (key only), 8-bit digits.
//
// The number of keys lives in device memory, so the sort can be enqueued before
// the count is known (and captured in a graph).  Per digit position, over
// tiles of 4096 keys:
//   count      -- per tile and digit, the number of keys;
//   scan_tiles -- per digit, those counts become the position of each tile's
//                 first key of that digit among the keys of that digit, and the
//                 digit's total is recorded;
//   scatter    -- each workgroup first turns the 256 totals into the start of
//                 every digit's bucket (a scan of 256 values), then ranks each
//                 tile by digit with wavefront ballots (stable: wavefront, step,
//                 then lane order), sorts it by digit in LDS and writes it out
//                 in runs of equal digits, so the stores are contiguous.
#include "cr_internal.h"

namespace cr {

constexpr int ST = 256;               // threads of a pass workgroup
constexpr int SKEYS = 16;             // keys per thread per tile
constexpr int STILE = ST * SKEYS;     // keys per tile
constexpr int SWAVES = ST / 64;
constexpr int SGRID = 1024;           // persistent workgroups of a pass

__device__ __forceinline__ uint64_t n_keys(const unsigned long long* n_ptr, uint64_t cap) {
  return *n_ptr < cap ? *n_ptr : cap;
}

// Ranks the keys of one tile by digit: wavefront w takes keys [w*1024, (w+1)*1024)
// of the tile, 64 per step; rank[j] = number of earlier keys of the same digit
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

// Per tile and digit: the number of keys, stored digit-major: counts[d * ntiles + tile].
__global__ __launch_bounds__(ST) void k_sort_count(const uint64_t* __restrict__ in,
                                                   const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                   int shift, uint32_t* __restrict__ counts) {
  __shared__ SortLds S;
  const int tid = threadIdx.x;
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t ntiles = (n + STILE - 1) / STILE;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int i = 0; i < SWAVES; ++i) S.cnt[i][tid] = 0;
    __syncthreads();
    const uint64_t t0 = tile * STILE;
    const uint32_t tcount = (uint32_t)(n - t0 < (uint64_t)STILE ? n - t0 : (uint64_t)STILE);
    uint64_t key[SKEYS];
    uint32_t rank[SKEYS];
    rank_tile(S, in, t0, tcount, shift, key, rank);
    __syncthreads();
    uint32_t tot = 0;
    for (int i = 0; i < SWAVES; ++i) tot += S.cnt[i][tid];
    counts[(uint64_t)tid * ntiles + tile] = tot;
    __syncthreads();
  }
}

// Per digit d (one workgroup each): counts[d * ntiles + t] becomes the number
// of keys of digit d in the tiles before t, and tot[d] the digit's total.
__global__ __launch_bounds__(256) void k_sort_scan_tiles(uint32_t* __restrict__ counts,
                                                         const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                         uint32_t* __restrict__ tot) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t carry_s;
  const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t ntiles = (n + STILE - 1) / STILE;
  uint32_t* col = counts + (uint64_t)d * ntiles;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  constexpr int PER = 8;
  for (uint64_t base = 0; base < ntiles; base += 256 * PER) {
    uint32_t v[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint64_t i = base + (uint64_t)tid * PER + k;
      v[k] = i < ntiles ? col[i] : 0u;
      sum += v[k];
    }
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t up = __shfl_up(incl, off, 64);
      if (lane >= off) incl += up;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t run = carry_s + incl - sum;
    for (int i = 0; i < w; ++i) run += wsum[i];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint64_t i = base + (uint64_t)tid * PER + k;
      if (i < ntiles) col[i] = run;
      run += v[k];
    }
    __syncthreads();
    if (tid == 255) carry_s = run;
    __syncthreads();
  }
  if (tid == 0) tot[d] = carry_s;
}

// One pass: each tile is ranked again, sorted by digit in LDS and written out
// in runs of equal digits at the positions from k_sort_scan_tiles.
__global__ __launch_bounds__(ST) void k_sort_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                     const unsigned long long* __restrict__ n_ptr, uint64_t cap,
                                                     int shift, const uint32_t* __restrict__ pos,
                                                     const uint32_t* __restrict__ tot) {
  __shared__ SortLds S;
  __shared__ uint32_t bucket[256];  // start of each digit's bucket
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t n = n_keys(n_ptr, cap);
  const uint64_t ntiles = (n + STILE - 1) / STILE;
  {
    const uint32_t t = tot[tid];
    uint32_t incl = t;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t up = __shfl_up(incl, off, 64);
      if (lane >= off) incl += up;
    }
    if (lane == 63) S.wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += S.wsum[i];
    bucket[tid] = before + incl - t;
    __syncthreads();
  }
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
    S.gpos[d] = bucket[d] + pos[(uint64_t)d * ntiles + tile];
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

// Scratch of launch_sort: per-tile counts and the digit totals.
size_t sort_scratch_bytes(uint64_t cap) {
  const uint64_t tiles = (cap + STILE - 1) / STILE + 1;
  return 4ull * 256 + 4ull * tiles * 256 + 256;
}

// Sorts keys[0..min(*n, cap)) ascending on bits [0, bits); tmp is scratch of the same
// size.  Returns the buffer (keys or tmp) that holds the result.
uint64_t* launch_sort(uint64_t* keys, uint64_t* tmp, const unsigned long long* n_ptr, uint64_t cap, int bits,
                      void* scratch, hipStream_t stream) {
  const int passes = (bits + 7) / 8;
  uint32_t* tot = static_cast<uint32_t*>(scratch);
  uint32_t* counts = tot + 256;
  const uint64_t max_tiles = (cap + STILE - 1) / STILE;
  const int grid = (int)(max_tiles < (uint64_t)SGRID ? (max_tiles ? max_tiles : 1) : (uint64_t)SGRID);
  uint64_t* a = keys;
  uint64_t* b = tmp;
  for (int p = 0; p < passes; ++p) {
    k_sort_count<<<grid, ST, 0, stream>>>(a, n_ptr, cap, 8 * p, counts);
    k_sort_scan_tiles<<<256, 256, 0, stream>>>(counts, n_ptr, cap, tot);
    k_sort_scatter<<<grid, ST, 0, stream>>>(a, b, n_ptr, cap, 8 * p, counts, tot);
    uint64_t* t = a;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace cr
