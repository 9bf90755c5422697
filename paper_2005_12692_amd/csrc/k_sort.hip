// LSD radix sort of 64-bit keys (key only), 8-bit digits.
//
// The number of keys lives in device memory, so the sort can be enqueued before
// the count is known (and captured in a graph).  The grid is fixed: SORT_G
// workgroups each own one contiguous chunk of ceil(n / SORT_G) keys.  One pass:
//   hist    -- per-chunk digit histogram in LDS, written digit-major;
//   scan    -- one workgroup turns the SORT_G x 256 counts into exclusive offsets;
//   scatter -- each chunk is walked in rounds of 256 keys in input order; wave64
//              ballots over the 8 digit bits give every key its rank among the
//              equal digits of its wavefront, LDS counters chain the wavefronts,
//              so the pass is stable and the sort is correct.
#include "cr_internal.h"

namespace cr {

constexpr int SORT_G = 1024;
constexpr int SORT_T = 256;

__global__ __launch_bounds__(SORT_T) void k_sort_hist(const uint64_t* __restrict__ keys,
                                                      const unsigned long long* __restrict__ n_ptr,
                                                      uint64_t cap, int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x, b = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint64_t n = *n_ptr < cap ? *n_ptr : cap;
  const uint64_t chunk = (n + SORT_G - 1) / SORT_G;
  const uint64_t lo = (uint64_t)b * chunk;
  const uint64_t hi = lo + chunk < n ? lo + chunk : n;
  for (uint64_t i = lo + tid; i < hi; i += SORT_T) atomicAdd(&h[(keys[i] >> shift) & 255], 1u);
  __syncthreads();
  hist[tid * SORT_G + b] = h[tid];
}

// Exclusive scan of SORT_G*256 counts, in place, by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist) {
  constexpr int TOTAL = SORT_G * 256;
  constexpr int PER = TOTAL / 1024;
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  uint32_t* seg = hist + (size_t)tid * PER;
  uint32_t s = 0;
  for (int i = 0; i < PER; ++i) s += seg[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = part[tid] - s;
  for (int i = 0; i < PER; ++i) {
    uint32_t c = seg[i];
    seg[i] = run;
    run += c;
  }
}

__global__ __launch_bounds__(SORT_T) void k_sort_scatter(const uint64_t* __restrict__ in,
                                                         uint64_t* __restrict__ out,
                                                         const unsigned long long* __restrict__ n_ptr,
                                                         uint64_t cap, int shift, const uint32_t* __restrict__ hist) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[SORT_T / 64][256];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  base[tid] = hist[tid * SORT_G + b];
  const uint64_t n = *n_ptr < cap ? *n_ptr : cap;
  const uint64_t chunk = (n + SORT_G - 1) / SORT_G;
  const uint64_t lo = (uint64_t)b * chunk;
  const uint64_t hi = lo + chunk < n ? lo + chunk : n;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint64_t start = lo; start < hi; start += SORT_T) {
    const uint64_t i = start + tid;
    const bool valid = i < hi;
    const uint64_t key = valid ? in[i] : 0;
    const uint32_t dig = (uint32_t)(key >> shift) & 255;
    for (int w = 0; w < SORT_T / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (dig >> bit) & 1;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][dig] = __popcll(peers);
    __syncthreads();
    {  // per digit: chain the wavefronts, advance the running base
      uint32_t run = base[tid];
      for (int w = 0; w < SORT_T / 64; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) out[wcnt[wave][dig] + rank] = key;
    __syncthreads();
  }
}

// Sorts keys[0..min(*n, cap)) ascending on bits [0, bits); tmp is scratch of the same
// size.  Returns the buffer (keys or tmp) that holds the result.
uint64_t* launch_sort(uint64_t* keys, uint64_t* tmp, const unsigned long long* n_ptr, uint64_t cap, int bits,
                      uint32_t* hist, hipStream_t stream) {
  const int passes = (bits + 7) / 8;
  uint64_t* a = keys;
  uint64_t* b = tmp;
  for (int p = 0; p < passes; ++p) {
    k_sort_hist<<<SORT_G, SORT_T, 0, stream>>>(a, n_ptr, cap, 8 * p, hist);
    k_sort_scan<<<1, 1024, 0, stream>>>(hist);
    k_sort_scatter<<<SORT_G, SORT_T, 0, stream>>>(a, b, n_ptr, cap, 8 * p, hist);
    uint64_t* t = a;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace cr
