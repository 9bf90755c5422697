// Host layer of libcr: argument checks, scratch planning, stage sequencing.
// Every stage is a HIP kernel enqueued on the caller's stream; the host only
// validates arguments, lays out scratch memory and reads back counts.
#include <string>
#include <vector>
#include <cstring>
#include <algorithm>
#include <cstdlib>
#include <cstddef>
#include <cstdio>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>

#include "cr.h"
#include "cr_reduce.h"

namespace cr {
// launchers defined in the kernel translation units
void launch_apparent(int ndim, int variant, int ntiles, const float* img, const ImgDesc* imgs, const int4* tiles,
                     Layout L, uint64_t* surv, uint64_t surv_cap, unsigned long long* surv_count,
                     int32_t* vlink, int32_t* tlink, uint8_t* eapp, uint32_t* img_status, Status* st,
                     hipStream_t stream);
void launch_dim_bounds(const uint64_t* keys, const unsigned long long* n_ptr, uint64_t cap, Layout L,
                       unsigned long long* dim_count, hipStream_t s);
uint64_t* launch_sort(uint64_t* keys, uint64_t* tmp, const unsigned long long* n_ptr, uint64_t cap, int bits,
                      void* scratch, hipStream_t stream);
size_t sort_scratch_bytes(uint64_t cap);
void launch_h0(int grid, const uint64_t* skeys, const unsigned long long* dim_count, const ImgDesc* imgs,
               Layout L, int32_t* vlink, uint64_t* T, uint8_t* neg, const EmitCtx& E, Status* st,
               hipStream_t s);
void launch_dual(int grid, int top, const uint64_t* skeys, const unsigned long long* dim_count,
                 const ImgDesc* imgs, Layout L, int32_t* tlink, const uint8_t* neg, uint8_t* mark, int emit,
                 uint64_t* T, const EmitCtx& E, Status* st, hipStream_t s);
struct RedCtx;
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_gather(int grid, const uint64_t* cand, const unsigned long long* n_ptr, uint64_t cap,
                   const float* img, const ImgDesc* imgs, Layout L, int32_t* dim, float* birth, float* death,
                   int64_t* bpix, int64_t* dpix, hipStream_t s);
void launch_img_offsets(const uint32_t* cnt, const uint32_t* img_status, const Status* st, int64_t capacity,
                        int nimg, int64_t* offsets, int32_t* status, hipStream_t s);
void launch_backward(const int64_t* bpix, const int64_t* dpix, const float* gb, const float* gd, int64_t n,
                     float* grad, int64_t n_pixels, uint32_t* bad, hipStream_t s);
void launch_lifetime(const int32_t* dim, const float* birth, const float* death, const int64_t* loc, int64_t n,
                     float* out, int64_t n_pixels, int skip_missing, uint32_t* bad, hipStream_t s);
void launch_pixel_coords(const int64_t* pixel, int64_t n, int64_t base, const int64_t ext[3], int32_t* xyz,
                         uint32_t* bad, hipStream_t s);
bool stencil_tile(int ndim, int variant, int ext[3]);
void stencil_tile_row1(int ext[3]);
constexpr int ROW1_VARIANT = 3;  // the stencil's one-row layout (see launch_apparent)

}  // namespace cr

using namespace cr;

// Scratch of cr_persistence_batched_noalloc, in static device memory: every GPU
// the library runs on holds its own copy of the array from the load of the code
// object until the process ends.  In host code this name is only a stand-in for
// the symbol: the device address comes from hipGetSymbolAddress (noalloc_setup)
// and is the one passed to kernels and copies.
static __device__ __align__(256) char noalloc_scratch[CR_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err = "no error";

cr_status fail(cr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(CR_ERR_HIP, std::string(#expr " failed: ") + hipGetErrorString(e_));       \
  } while (0)

// A non-negative integer from the environment, or `def` when unset.
uint64_t env_u64(const char* name, uint64_t def) {
  const char* v = getenv(name);
  return (v && *v) ? (uint64_t)strtoull(v, nullptr, 10) : def;
}

int bits_for(uint64_t x) {  // smallest b with x < 2^b
  int b = 0;
  while (b < 64 && (x >> b) != 0) ++b;
  return b;
}

constexpr int RGRID = 512;            // workgroups of the thread-mode reduction (256 threads each)
constexpr int N_TILE_VARIANTS = 3;    // stencil tile shapes (see stencil_tile)

// Default launch parameters (cr_tuning) per ndim.
cr_tuning default_tuning(int ndim) {
  cr_tuning t;
  t.tile = 0;
  t.grid = 2048;
  t.long_len = 32;
  t.yield_iters = 1024;
  // with the asynchronous tail taking the last, latency-bound part of degree 1,
  // shorter rounds pay before it: the 256^3 volume 58.7 ms per step with
  // (wave_yield, wave_short) = (128, 4096), 55.0 with (64, 16384), 54.3 with
  // (48, 65536); the 32-volume batch 44.4, 45.0, 46.6 ms
  t.wave_short = 16384;
  t.front_cap = 1024;
  t.wave_yield = 64;
  t.group_max = 0;   // automatic (by the number of images)
  t.narrow_min = 0;
  (void)ndim;
  return t;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Problem {
  int nimg = 0, ndim = 0, maxdim = 0;
  std::vector<ImgDesc> imgs;
  std::vector<int4> tiles;
  uint64_t P = 0, N = 0;  // totals over the batch
  int tile = 0;           // stencil tile variant of the call (ROW1_VARIANT: every image one row)
  Layout L{};
};

struct Plan {
  size_t status, counters, img_status, img_pairs, imgs, tiles, surv_a, surv_b, hist, vlink, tlink, T, neg,
      owner, claim, piv, colptr, arena, cleared, list[4], eapp, total;
  uint64_t surv_cap, e_cap, arena_cap;
  size_t T0 = 0;  // degree 0's own merge structure when it runs beside degree 2 and the reduction (0: none)
};

}  // namespace

struct cr_context {
  int device = 0;
  cr_alloc_fn alloc = nullptr;
  cr_free_fn free_fn = nullptr;
  void* user = nullptr;
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  char* host_stage = nullptr;
  size_t host_stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
  hipEvent_t round_ev[2] = {};   // the reduction's list counts of a batch of rounds have landed
  hipStream_t side = nullptr;    // degree 0 of a volume runs here beside degree 2 and the reduction
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  uint64_t arena_entries = 1ull << 28;  // column arena of the next call (grown on overflow)
  Plan plan{};
  Problem prob{};
  cr_stats stats{};
  bool last_batched_valid = false;
  uint32_t* bwd_flag = nullptr;  // device word for the backward index check
  bool sync_allowed = false;     // the plain call may synchronise between reduction rounds
  int rounds = 0;
  int reruns = 0;                // plain calls rerun with a larger column arena (since creation)
  char* noalloc = nullptr;       // device address of this device's noalloc_scratch
  bool last_noalloc = false;     // the last batched call ran on noalloc_scratch
  // stage timing (CR_FLAG_STAGE_TIMES)
  hipEvent_t ev[8] = {};
  bool ev_ready = false;
  bool timing = false;
  float stage_ms[6] = {};
  cr_tuning tune[4] = {};        // launch parameters per ndim (2, 3)
  bool tune_set[4] = {};         // cr_set_tuning was called for this ndim (the tuning cache is not used)
  bool in_autotune = false;      // the autotuner's own calls (the tuning cache is not used)
  bool cache_loaded = false;     // CR_TUNE_CACHE has been read
  std::map<std::string, cr_tuning> cache;  // its entries
  std::string arch;              // gcn arch name of the device (tuning cache key)
};

namespace {

// Column arena (64-bit entries) of a batched call, which cannot rerun: the
// context's size (grown when a batched call is found to have overflowed it),
// at least ARENA_PER_PIXEL entries per pixel of the batch (a 256^3 volume of
// blobs and noise uses ~12.8), or CR_ARENA_ENTRIES when that is set.
constexpr uint64_t ARENA_PER_PIXEL = 16;
constexpr uint64_t ARENA_DEFAULT = 1ull << 28;
uint64_t batch_arena(const cr_context* ctx, const Problem& pb) {
  const uint64_t env = env_u64("CR_ARENA_ENTRIES", 0);
  if (env) return env;
  const uint64_t have = ctx ? ctx->arena_entries : ARENA_DEFAULT;
  return std::max(have, std::min<uint64_t>(ARENA_MAX, ARENA_PER_PIXEL * pb.P));
}

// After a batched call (or graph replay) whose column arena of `cap` entries
// overflowed, with `top` entries asked for before it stopped (a lower bound of
// the need): the context's later batched calls and graphs get a larger arena.
void grow_arena(cr_context* ctx, uint64_t cap, uint64_t top) {
  const uint64_t want = std::max<uint64_t>(cap * 4, top * 2);
  ctx->arena_entries = std::max<uint64_t>(ctx->arena_entries, std::min<uint64_t>(want, ARENA_MAX));
}

// Device address of noalloc_scratch on each device, looked up once per device
// with that device current (each GPU holds its own copy at its own address).
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

cr_status noalloc_setup(int device, char** out) {
  *out = nullptr;
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(CR_ERR_INVALID_ARGUMENT, "device index too large");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !ptr)
      return fail(CR_ERR_HIP, std::string("hipGetSymbolAddress(noalloc_scratch) failed: ") + hipGetErrorString(e));
    g_noalloc_ptr[device] = static_cast<char*>(ptr);
  }
  *out = g_noalloc_ptr[device];
  return CR_OK;
}

// Column arena of a batched call on noalloc_scratch: ARENA_PER_PIXEL entries per
// pixel (at least 2^16), or CR_ARENA_ENTRIES when that is set.
uint64_t noalloc_arena(const Problem& pb) {
  const uint64_t env = env_u64("CR_ARENA_ENTRIES", 0);
  return env ? env : std::max<uint64_t>(1ull << 16, ARENA_PER_PIXEL * pb.P);
}

// counters block: surv_count, dim_count[4], cand_count, arena_top, lists[4], wave work counter,
// arena offset at the start of the asynchronous tail, columns in the first round's spatial order
enum { C_SURV = 0, C_DIM = 1, C_CAND = 5, C_ARENA = 6, C_LIST = 7 /* six words */, C_WORK = 13, C_BASE = 14, C_SPATIAL = 15,
       C_WORDS = 16 };

// A 1D signal lies on one line of the grid (Sec. 2): it runs as a 1 x n image,
// with the 2D launch parameters.
int grid_ndim(int ndim) { return ndim == 1 ? 2 : ndim; }

cr_status build_problem(Problem& pb, int nimg, const int64_t* pixel_offsets, const int64_t* shapes, int ndim,
                        int maxdim, int tile_variant) {
  if (nimg < 1) return fail(CR_ERR_INVALID_ARGUMENT, "n_images must be >= 1");
  if (ndim < 1 || ndim > 3) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  if (maxdim < 0) return fail(CR_ERR_INVALID_ARGUMENT, "maxdim must be >= 0");
  if (!shapes) return fail(CR_ERR_INVALID_ARGUMENT, "shape is NULL");
  pb.nimg = nimg;
  pb.ndim = grid_ndim(ndim);
  pb.maxdim = std::min(maxdim, ndim - 1);
  pb.imgs.resize(nimg);
  pb.tiles.clear();
  pb.P = 0;
  pb.N = 0;
  uint64_t maxN = 1, maxP = 1;
  int tile[3];
  if (!stencil_tile(pb.ndim, tile_variant, tile)) return fail(CR_ERR_INVALID_ARGUMENT, "bad stencil tile variant");
  // images of one row (1D signals) take the one-row layout: a workgroup's
  // wavefronts lie side by side along the row, not on rows outside the image
  bool row1 = pb.ndim == 2;
  for (int i = 0; i < nimg && row1; ++i) row1 = ndim == 1 || shapes[(int64_t)i * ndim] == 1;
  pb.tile = row1 ? ROW1_VARIANT : tile_variant;
  if (row1) stencil_tile_row1(tile);
  for (int i = 0; i < nimg; ++i) {
    int64_t n[3] = {1, 1, 1};
    for (int a = 0; a < ndim; ++a) {
      const int64_t s = shapes[(int64_t)i * ndim + a];
      if (s < 1) return fail(CR_ERR_INVALID_ARGUMENT, "every extent must be >= 1");
      if (s > (1 << 29)) return fail(CR_ERR_TOO_LARGE, "extent too large");
      n[3 - ndim + a] = s;
    }
    ImgDesc& d = pb.imgs[i];
    uint64_t P = 1, N = 1;
    for (int a = 0; a < 3; ++a) {
      d.n[a] = (int32_t)n[a];
      d.K[a] = (int32_t)(2 * n[a] - 1);
      P *= (uint64_t)n[a];
      N *= (uint64_t)(2 * n[a] - 1);
    }
    if (N > (1ull << 30)) return fail(CR_ERR_TOO_LARGE, "an image has more than 2^30 cells");
    d.pix_off = (int64_t)pb.P;
    if (pixel_offsets) {
      if (pixel_offsets[i] != (int64_t)pb.P || pixel_offsets[i + 1] != (int64_t)(pb.P + P))
        return fail(CR_ERR_INVALID_ARGUMENT, "pixel_offsets do not match the shapes");
    }
    pb.P += P;
    pb.N += N;
    maxN = std::max(maxN, N);
    maxP = std::max(maxP, P);
    for (int64_t z = 0; z < n[0]; z += tile[0])
      for (int64_t y = 0; y < n[1]; y += tile[1])
        for (int64_t x = 0; x < n[2]; x += tile[2]) pb.tiles.push_back(make_int4(i, (int)z, (int)y, (int)x));
  }
  if (pb.P >= (1ull << 31) - 2) return fail(CR_ERR_TOO_LARGE, "more than 2^31 pixels in one call");
  if (pb.N >= (1ull << 32)) return fail(CR_ERR_TOO_LARGE, "more than 2^32 cells in one call");
  Layout& L = pb.L;
  L.kb = std::max(1, bits_for(maxN - 1));
  L.ib = nimg > 1 ? bits_for((uint64_t)nimg - 1) : 0;
  L.pb = bits_for(maxP);
  L.nimg = nimg;
  L.ndim = ndim;
  if (2 + L.ib + 32 + L.kb > 64 || L.ib + 2 + 2 * L.pb > 64)
    return fail(CR_ERR_TOO_LARGE, "batch too large for the 64-bit key layout; split it");
  return CR_OK;
}

Plan make_plan(const Problem& pb, uint64_t arena_entries, bool side_h0 = false) {
  Plan p{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  p.surv_cap = pb.N;
  p.e_cap = 3 * pb.P + 64;
  const bool vol = pb.ndim == 3 && pb.maxdim >= 1;
  p.arena_cap = vol ? std::min<uint64_t>(arena_entries, ARENA_MAX) : 0;
  p.status = take(sizeof(Status));
  p.counters = take(C_WORDS * 8);
  p.img_status = take(4 * (size_t)pb.nimg);
  p.img_pairs = take(4 * (size_t)(pb.nimg + 1));
  p.imgs = take(sizeof(ImgDesc) * pb.nimg);
  p.tiles = take(sizeof(int4) * pb.tiles.size());
  p.surv_a = take(8 * p.surv_cap);
  p.surv_b = take(8 * p.surv_cap);
  p.hist = take(sort_scratch_bytes(p.surv_cap));
  p.vlink = take(4 * pb.P);
  p.tlink = take(4 * pb.P);
  p.T = take(8 * (pb.P + pb.nimg + 64));
  p.neg = take(p.e_cap);
  p.owner = take(vol ? 8 * 3 * pb.P : 0);
  p.piv = take(vol ? 8 * p.e_cap : 0);
  p.colptr = take(vol ? 8 * p.e_cap : 0);
  p.arena = take(vol ? 8 * (p.arena_cap + ARENA_SLACK) : 0);
  p.cleared = take(vol ? p.e_cap : 0);
  p.claim = take(vol ? 8 * 3 * pb.P : 0);
  for (int i = 0; i < 4; ++i) p.list[i] = take(vol ? 4 * p.e_cap : 0);
  p.eapp = take(vol ? 4 * pb.P : 0);
  if (vol && side_h0) p.T0 = take(8 * (pb.P + pb.nimg + 64));
  p.total = o;
  return p;
}

cr_status ensure_scratch(cr_context* ctx, size_t bytes) {
  if (ctx->scratch_bytes >= bytes) return CR_OK;
  if (ctx->scratch) {
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  const size_t want = align_up(bytes + bytes / 8, 1 << 21);
  if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
    (void)hipGetLastError();
    ctx->scratch = nullptr;
    return fail(CR_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(want) + " scratch bytes failed");
  }
  ctx->scratch_bytes = want;
  return CR_OK;
}

cr_status ensure_stage(cr_context* ctx, size_t bytes) {
  if (ctx->stage_pending) {
    HIP_TRY(hipEventSynchronize(ctx->stage_done));
    ctx->stage_pending = false;
  }
  if (ctx->host_stage_bytes >= bytes) return CR_OK;
  if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
  ctx->host_stage = nullptr;
  const size_t want = align_up(bytes, 1 << 16);
  if (hipHostMalloc((void**)&ctx->host_stage, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->host_stage_bytes = 0;
    return fail(CR_ERR_OUT_OF_MEMORY, "pinned staging allocation failed");
  }
  ctx->host_stage_bytes = want;
  return CR_OK;
}

template <class T>
T* at(cr_context* ctx, size_t off) {
  return reinterpret_cast<T*>(ctx->scratch + off);
}

// stage boundaries; A and B close the two higher-degree stages (2D: degree 1
// then nothing; 3D: degree 2 then degree 1)
// EV_H0S: the start of degree 0 when it runs on the side stream
enum { EV_START = 0, EV_STENCIL, EV_SORT, EV_H0, EV_A, EV_B, EV_ROWS, EV_H0S, EV_N };

// Records stage boundary `i` when stage timing is on.
void mark(cr_context* ctx, int i, hipStream_t s) {
  if (ctx->timing) (void)hipEventRecord(ctx->ev[i], s);
}

// Rounds of the degree-1 reduction, then its asynchronous tail.  With host
// synchronisation allowed (plain call) the host checks every ROUND_BATCH rounds
// whether the rounds are over (no column left, or a round left to the tail);
// otherwise a fixed budget of rounds is enqueued (rounds return at once when
// their lists are empty or were left to the tail).  The tail then reduces
// whatever is left, in one launch (it returns at once when nothing is).
// Columns that yield (wave_yield) take more rounds, so within the budget they
// yield only in the first YIELD_ROUNDS rounds.
constexpr int ROUND_BATCH = 4;
constexpr int ROUND_BUDGET = 128;
constexpr int YIELD_ROUNDS = 64;
constexpr int ROUND_LIMIT = 4096;

// side_start, if given, is called once the first SIDE_AFTER rounds have been
// enqueued and checked not to be the last (or right after the tail when the
// rounds end sooner), to start work beside the latency-bound later rounds and
// the tail.
constexpr int SIDE_AFTER = 20;

cr_status run_rounds(cr_context* ctx, const RedCtx& R, uint32_t* lists[4], unsigned long long* counts,
                     hipStream_t s, const std::function<cr_status()>& side_start = nullptr) {
  ctx->rounds = 0;
  if (!ctx->sync_allowed) {
    // CR_ROUND_BUDGET / CR_YIELD_ROUNDS override the budget (e.g. small, so that
    // the tail does most of the reduction of a small batch)
    const int budget = (int)std::max<uint64_t>(1, std::min<uint64_t>(env_u64("CR_ROUND_BUDGET", ROUND_BUDGET), 1 << 16));
    const int yields = (int)std::min<uint64_t>(env_u64("CR_YIELD_ROUNDS", YIELD_ROUNDS), (uint64_t)budget);
    launch_h1_rounds(RGRID, R, lists, counts, 0, budget, yields, s);
    launch_h1_async(R, lists, counts, budget, s);
    return CR_OK;
  }
  // Batches of rounds are enqueued one ahead of the check: the counts left by
  // batch k-1 are read while batch k runs, so the GPU does not idle during the
  // host's round trip; rounds after the end return at once.
  cr_status rc = ensure_stage(ctx, 64);
  if (rc != CR_OK) return rc;
  for (hipEvent_t& e : ctx->round_ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  bool side_started = !side_start;
  auto start_side = [&]() -> cr_status {
    if (side_started) return CR_OK;
    side_started = true;
    return side_start();
  };
  // Batch k's read-back is enqueued only once batch k-1's has been checked, so
  // that the tail, when that check ends the loop, follows the rounds directly:
  // behind a read-back it would wait for the copy, whose kernel finds no free
  // slot while the side stream's degree-0 merge fills the GPU (~0.85 ms on the
  // 256^3 volume).
  int round_end = ROUND_LIMIT;
  for (int k = 0; k * ROUND_BATCH < ROUND_LIMIT; ++k) {
    const int r = k * ROUND_BATCH;
    launch_h1_rounds(RGRID, R, lists, counts, r, ROUND_BATCH, ROUND_LIMIT, s);
    if (k > 0) {
      HIP_TRY(hipEventSynchronize(ctx->round_ev[(k - 1) & 1]));
      const char* prev = ctx->host_stage + 32 * ((k - 1) & 1);
      unsigned long long left[2] = {0, 0};
      uint32_t ab[2] = {0, 0};
      std::memcpy(left, prev, 16);
      std::memcpy(ab, prev + 16, 8);
      ctx->rounds = r;
      // also once at most twice the tail's threshold is left: the batch just
      // enqueued reaches the threshold (or the tail takes the lists its last
      // round builds), and another batch would run as empty rounds
      const uint64_t n_left = left[0] + left[1];
      if (n_left == 0 || ab[0] || ab[1] || (R.async_max && n_left <= 2ull * R.async_max)) {
        round_end = r + ROUND_BATCH;
        break;
      }
    }
    if (r + ROUND_BATCH >= SIDE_AFTER) {
      rc = start_side();
      if (rc != CR_OK) return rc;
    }
    const int cur = (r + ROUND_BATCH) % 3;  // the count pair the next round reads
    char* slot = ctx->host_stage + 32 * (k & 1);
    HIP_TRY(hipMemcpyAsync(slot, counts + 2 * cur, 16, hipMemcpyDeviceToHost, s));
    static_assert(offsetof(Status, tail_round) == offsetof(Status, abort) + 4, "abort and tail_round are adjacent");
    HIP_TRY(hipMemcpyAsync(slot + 16, &R.st->abort, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->round_ev[k & 1], s));
  }
  // the tail first: its workgroups (one per CU) are dispatched before the side
  // stream's degree-0 kernels, which fill the remaining wave slots beside them
  launch_h1_async(R, lists, counts, round_end, s);
  return start_side();
}

// Copies the image descriptors and stencil tiles of ctx->prob into scratch.
// Asynchronous through the pinned stage unless `sync` (then the copy is
// complete on return, as graph capture needs).
cr_status upload_descriptors(cr_context* ctx, hipStream_t s, bool sync) {
  const Problem& pb = ctx->prob;
  const Plan& p = ctx->plan;
  const size_t bi = sizeof(ImgDesc) * pb.nimg, bt = sizeof(int4) * pb.tiles.size();
  cr_status rc = ensure_stage(ctx, bi + bt);
  if (rc != CR_OK) return rc;
  std::memcpy(ctx->host_stage, pb.imgs.data(), bi);
  std::memcpy(ctx->host_stage + bi, pb.tiles.data(), bt);
  HIP_TRY(hipMemcpyAsync(at<ImgDesc>(ctx, p.imgs), ctx->host_stage, bi, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<int4>(ctx, p.tiles), ctx->host_stage + bi, bt, hipMemcpyHostToDevice, s));
  if (sync) {
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    HIP_TRY(hipEventRecord(ctx->stage_done, s));
    ctx->stage_pending = true;
  }
  return CR_OK;
}

// The same copies from the problem's own (pageable) host vectors, with no
// pinned staging buffer: the runtime stages pageable memory itself before the
// call returns, so the vectors may change afterwards.
cr_status upload_descriptors_pageable(cr_context* ctx, hipStream_t s) {
  const Problem& pb = ctx->prob;
  const Plan& p = ctx->plan;
  HIP_TRY(hipMemcpyAsync(at<ImgDesc>(ctx, p.imgs), pb.imgs.data(), sizeof(ImgDesc) * pb.nimg,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<int4>(ctx, p.tiles), pb.tiles.data(), sizeof(int4) * pb.tiles.size(),
                         hipMemcpyHostToDevice, s));
  return CR_OK;
}

// Enqueues every stage up to sorted canonical keys.  Returns the buffer holding
// them.  With upload = false the descriptors are already in scratch and only
// kernels are enqueued.
cr_status enqueue_pipeline(cr_context* ctx, const float* image, hipStream_t s, uint64_t** cand_out,
                           bool upload = true) {
  const Problem& pb = ctx->prob;
  const Plan& p = ctx->plan;
  const Layout L = pb.L;
  Status* st = at<Status>(ctx, p.status);
  unsigned long long* cnt = at<unsigned long long>(ctx, p.counters);
  uint32_t* img_status = at<uint32_t>(ctx, p.img_status);
  uint32_t* img_pairs = at<uint32_t>(ctx, p.img_pairs);
  ImgDesc* d_imgs = at<ImgDesc>(ctx, p.imgs);
  int4* d_tiles = at<int4>(ctx, p.tiles);

  if (upload) {
    cr_status rc = upload_descriptors(ctx, s, false);
    if (rc != CR_OK) return rc;
  }

  // zero the status words, counters and per-image counts (one contiguous range)
  launch_fill_u32(reinterpret_cast<uint32_t*>(st), 0, (p.img_pairs + 4 * (pb.nimg + 1) - p.status) / 4, s);

  uint64_t* surv = at<uint64_t>(ctx, p.surv_a);
  uint64_t* surv_tmp = at<uint64_t>(ctx, p.surv_b);
  int32_t* vlink = at<int32_t>(ctx, p.vlink);
  int32_t* tlink = at<int32_t>(ctx, p.tlink);
  mark(ctx, EV_START, s);
  uint8_t* eapp = (pb.ndim == 3 && pb.maxdim >= 1) ? at<uint8_t>(ctx, p.eapp) : nullptr;
  const cr_tuning& tu = ctx->tune[pb.ndim];
  launch_apparent(pb.ndim, pb.tile, (int)pb.tiles.size(), image, d_imgs, d_tiles, L, surv, p.surv_cap, &cnt[C_SURV],
                  vlink, tlink, eapp, img_status, st, s);
  mark(ctx, EV_STENCIL, s);
  void* hist = at<char>(ctx, p.hist);
  uint64_t* skeys = launch_sort(surv, surv_tmp, &cnt[C_SURV], p.surv_cap, 2 + L.ib + 32 + L.kb, hist, s);
  launch_dim_bounds(skeys, &cnt[C_SURV], p.surv_cap, L, &cnt[C_DIM], s);
  mark(ctx, EV_SORT, s);
  uint64_t* cand = (skeys == surv) ? surv_tmp : surv;  // the other buffer collects the rows

  EmitCtx E;
  E.img = image;
  E.imgs = d_imgs;
  E.L = L;
  E.cand = cand;
  E.cand_cap = p.surv_cap;
  E.cand_count = &cnt[C_CAND];
  E.img_pairs = img_pairs;
  E.st = st;

  uint8_t* neg = at<uint8_t>(ctx, p.neg);
  launch_fill_u32(reinterpret_cast<uint32_t*>(neg), 0, p.e_cap / 4, s);
  uint64_t* T = at<uint64_t>(ctx, p.T);
  // Degree 0 of a volume depends on nothing that degrees 1 and 2 compute, so a
  // plain call runs it on a second stream, on its own merge structure, started
  // once the reduction has reached its latency-bound rounds.
  const bool side_h0 = p.T0 != 0;
  struct Join {  // every return after the fork makes s wait for the side stream
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    ~Join() {
      if (e) (void)hipStreamWaitEvent(s, e, 0);
    }
  } join;
  std::function<cr_status()> fork_h0;
  if (side_h0) {
    if (!ctx->side) HIP_TRY(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    if (!ctx->fork_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    if (!ctx->join_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
    // the fork event is recorded before the reduction (degree 0 needs only the
    // sorted cells), the side work enqueued later, when fork_h0 is called
    fork_h0 = [&]() -> cr_status {
      HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
      mark(ctx, EV_H0S, ctx->side);
      launch_h0(tu.grid, skeys, &cnt[C_DIM], d_imgs, L, vlink, at<uint64_t>(ctx, p.T0), neg, E, st, ctx->side);
      mark(ctx, EV_H0, ctx->side);
      HIP_TRY(hipEventRecord(ctx->join_ev, ctx->side));
      join.s = s;
      join.e = ctx->join_ev;
      return CR_OK;
    };
  } else {
    launch_h0(tu.grid, skeys, &cnt[C_DIM], d_imgs, L, vlink, T, neg, E, st, s);
    mark(ctx, EV_H0, s);
  }

  uint64_t* owner = at<uint64_t>(ctx, p.owner);
  if (pb.ndim == 2) {
    if (pb.maxdim >= 1) launch_dual(tu.grid, 2, skeys, &cnt[C_DIM], d_imgs, L, tlink, neg, nullptr, 1, T, E, st, s);
    mark(ctx, EV_A, s);
    mark(ctx, EV_B, s);
  } else if (pb.maxdim >= 1) {
    // degree 2 first (dual union-find over every surviving square); it marks the
    // squares that give birth to a void, whose degree-1 columns are zero
    uint8_t* cleared = at<uint8_t>(ctx, p.cleared);
    launch_fill_u32(reinterpret_cast<uint32_t*>(cleared), 0, p.e_cap / 4, s);
    launch_dual(tu.grid, 3, skeys, &cnt[C_DIM], d_imgs, L, tlink, nullptr, cleared, pb.maxdim >= 2, T, E, st, s);
    mark(ctx, EV_A, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(owner), 0xFFFFFFFFu, 2 * 3 * pb.P, s);
    launch_fill_u32(at<uint32_t>(ctx, p.claim), 0, 2 * 3 * pb.P, s);
    RedCtx R = make_redctx(image, d_imgs, L, skeys, &cnt[C_DIM], cleared, eapp, owner, at<uint64_t>(ctx, p.claim),
                           at<uint64_t>(ctx, p.piv), at<uint64_t>(ctx, p.colptr), at<uint64_t>(ctx, p.arena),
                           p.arena_cap, &cnt[C_ARENA], &cnt[C_WORK], st);
    R.long_len = (uint32_t)std::min(tu.long_len, 32);
    R.yield_iters = (uint32_t)tu.yield_iters;
    R.wave_short = (uint32_t)tu.wave_short;
    R.front_cap = (uint32_t)tu.front_cap;
    R.wave_yield = (uint32_t)tu.wave_yield;
    // a batch's rounds hold the columns of many volumes: a workgroup per column
    // pays off only in rounds of few of them, and the narrow wavefront
    // configuration already from fewer columns than for one volume (automatic
    // values; measured on 32 x 128^3 forward+backward: 56.6 -> 50.4 ms with 256
    // and 2048; a single 256^3 volume is fastest with 1024 and 8192)
    const bool many = pb.nimg >= 8;
    R.group_max = tu.group_max ? (uint32_t)tu.group_max : (many ? 256u : 1024u);
    R.narrow_min = tu.narrow_min ? (uint32_t)tu.narrow_min : (many ? 2048u : 8192u);
    // thresholds between thread and wave mode and the wave-mode front capacity
    // (CR_LONG_LEN / CR_YIELD_ITERS / CR_WAVE_SHORT / CR_FRONT_CAP override them,
    // e.g. to exercise wave mode and its tail merges on small inputs)
    if (const char* v = getenv("CR_LONG_LEN")) R.long_len = (uint32_t)strtoul(v, nullptr, 10);
    if (const char* v = getenv("CR_YIELD_ITERS")) R.yield_iters = (uint32_t)strtoul(v, nullptr, 10);
    if (const char* v = getenv("CR_WAVE_SHORT")) R.wave_short = (uint32_t)strtoul(v, nullptr, 10);
    if (const char* v = getenv("CR_MID_CAP")) R.mid_cap = (uint32_t)strtoul(v, nullptr, 10);
    if (const char* v = getenv("CR_NARROW_MIN")) R.narrow_min = (uint32_t)strtoul(v, nullptr, 10);
    if (const char* v = getenv("CR_GROUP_MAX")) R.group_max = (uint32_t)strtoul(v, nullptr, 10);
    if (const char* v = getenv("CR_WAVE_YIELD")) R.wave_yield = (uint32_t)strtoul(v, nullptr, 10);
    // a round of at most two columns has nothing to run beside its longest
    // column, which then does not yield (256^3 degree 1 62.0 -> 60.3 ms;
    // larger thresholds measured erratic: 4 and 16 slower, 8 faster)
    if (const char* v = getenv("CR_YIELD_FEW")) R.yield_few = (uint32_t)strtoul(v, nullptr, 10);
    // rounds of at most this many columns are left to the asynchronous tail
    // (CR_ASYNC_MAX overrides; 0 keeps rounds to the end).  Measured: the 256^3
    // volume 64.0 ms without the tail, 59.8 / 58.9 / 59.3 ms with 2048 / 4096 /
    // 8192; the 32 x 128^3 batch 47.9 ms without, 44.2 / 45.3 / 56.1 ms with
    // 256 / 1024 / 4096 (its tail holds the columns of many volumes)
    R.async_max = many ? 256u : 4096u;
    if (const char* v = getenv("CR_ASYNC_MAX")) R.async_max = (uint32_t)strtoul(v, nullptr, 10);
    R.async_base = &cnt[C_BASE];
    if (const char* v = getenv("CR_GROUP_CAP")) {
      const unsigned long f = strtoul(v, nullptr, 10);
      R.group_cap = (uint32_t)(f < FRONT_CAP_MIN ? FRONT_CAP_MIN : (f > 4096 ? 4096 : f));
    }
    if (const char* v = getenv("CR_NARROW_CAP")) {
      const unsigned long f = strtoul(v, nullptr, 10);
      R.narrow_cap = (uint32_t)(f < FRONT_CAP_MIN ? FRONT_CAP_MIN : (f > FRONT_CAP_NARROW_MAX ? FRONT_CAP_NARROW_MAX : f));
    }
    if (const char* v = getenv("CR_FRONT_CAP")) {
      const unsigned long f = strtoul(v, nullptr, 10);
      R.front_cap = (uint32_t)(f < FRONT_CAP_MIN ? FRONT_CAP_MIN : (f > FRONT_CAP_MAX ? FRONT_CAP_MAX : f));
    }
    uint32_t* lists[4] = {at<uint32_t>(ctx, p.list[0]), at<uint32_t>(ctx, p.list[1]), at<uint32_t>(ctx, p.list[2]),
                          at<uint32_t>(ctx, p.list[3])};
    // the first round's columns in spatial order: their keys sorted by (image,
    // Khalimsky index) in the two halves of T, free once degree 2 is done
    // (256^3 volume: the first round 3.35 -> 2.82 ms for ~0.2 ms of keys and
    // four sort passes; CR_SPATIAL=0 keeps rank order)
    if (env_u64("CR_SPATIAL", 1)) {
      const uint64_t half = (pb.P + pb.nimg + 64) / 2;
      launch_h1_spatial_keys(tu.grid, R, T, half, &cnt[C_SPATIAL], s);
      R.spatial = launch_sort(T, T + half, &cnt[C_SPATIAL], half, L.ib + L.kb, hist, s);
      R.n_spatial = &cnt[C_SPATIAL];
    }
    if (side_h0) HIP_TRY(hipEventRecord(ctx->fork_ev, s));
    cr_status rrc = run_rounds(ctx, R, lists, &cnt[C_LIST], s, fork_h0);
    if (rrc != CR_OK) return rrc;
    launch_h1_emit(tu.grid, R, E, s);
    mark(ctx, EV_B, s);
  } else {
    mark(ctx, EV_A, s);
    mark(ctx, EV_B, s);
  }
  if (side_h0) {  // degree 0's rows are in
    join.e = nullptr;
    HIP_TRY(hipStreamWaitEvent(s, ctx->join_ev, 0));
  }
  // canonical order: sort the row keys.  The survivor keys are dead now, so
  // their buffer is the scratch of this sort.
  *cand_out = launch_sort(cand, skeys, &cnt[C_CAND], p.surv_cap, L.ib + 2 + 2 * L.pb, hist, s);
  mark(ctx, EV_ROWS, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CR_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return CR_OK;
}

struct HostCounters {
  Status st;
  unsigned long long cnt[C_WORDS];
};

cr_status read_counters(cr_context* ctx, hipStream_t s, HostCounters* h) {
  const Plan& p = ctx->plan;
  cr_status rc = ensure_stage(ctx, sizeof(HostCounters));
  if (rc != CR_OK) return rc;
  HIP_TRY(hipMemcpyAsync(ctx->host_stage, ctx->scratch + p.status, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(ctx->host_stage + sizeof(Status), ctx->scratch + p.counters, 8 * C_WORDS,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ctx->timing) {
    float ms[6] = {};
    for (int i = 0; i < 6; ++i) (void)hipEventElapsedTime(&ms[i], ctx->ev[i], ctx->ev[i + 1]);
    const bool vol = ctx->prob.ndim == 3;
    if (ctx->plan.T0) {  // degree 0 ran on the side stream; degree 2 follows the sort
      (void)hipEventElapsedTime(&ms[2], ctx->ev[EV_H0S], ctx->ev[EV_H0]);
      (void)hipEventElapsedTime(&ms[3], ctx->ev[EV_SORT], ctx->ev[EV_A]);
    }
    ctx->stage_ms[0] = ms[0];
    ctx->stage_ms[1] = ms[1];
    ctx->stage_ms[2] = ms[2];
    ctx->stage_ms[3] = vol ? ms[4] : ms[3];  // degree 1
    ctx->stage_ms[4] = vol ? ms[3] : 0.0f;   // degree 2
    ctx->stage_ms[5] = ms[5];
  }
  std::memcpy(&h->st, ctx->host_stage, sizeof(Status));
  std::memcpy(h->cnt, ctx->host_stage + sizeof(Status), 8 * C_WORDS);
  cr_stats& S = ctx->stats;
  S.n_pixels = (int64_t)ctx->prob.P;
  S.n_cells = (int64_t)ctx->prob.N;
  for (int i = 0; i < 4; ++i) S.survivors[i] = (int64_t)h->cnt[C_DIM + i];
  S.n_rows = (int64_t)h->cnt[C_CAND];
  S.arena_used = (int64_t)h->cnt[C_ARENA];
  S.red_adds = (int64_t)h->st.adds;
  S.red_merged = (int64_t)h->st.merged;
  S.red_rounds = ctx->rounds;
  S.arena_reruns = ctx->reruns;
  return CR_OK;
}

cr_status status_error(const Status& st, bool* arena_overflow) {
  *arena_overflow = false;
  if (st.nan_input) return fail(CR_ERR_NAN_INPUT, "input contains NaN");
  if (st.overflow) {
    *arena_overflow = (st.overflow & OVF_ARENA) != 0;
    std::string what;
    if (st.overflow & OVF_SURVIVORS) what += " survivors";
    if (st.overflow & OVF_ARENA) what += " column-arena";
    if (st.overflow & OVF_ROWS) what += " rows";
    if (st.overflow & OVF_COLUMN) what += " column-length";
    return fail(CR_ERR_OUT_OF_MEMORY, "scratch capacity exceeded:" + what);
  }
  if (st.iter_cap) return fail(CR_ERR_INTERNAL, "iteration cap reached");
  if (st.internal) return fail(CR_ERR_INTERNAL, "internal consistency check failed");
  return CR_OK;
}

struct BatchArgs {
  int n_images;
  const float* packed;
  const int64_t* pixel_offsets;
  const int64_t* shapes;
  int ndim, maxdim;
  uint32_t flags;
  int32_t* dim;
  float* birth;
  float* death;
  int64_t* birth_pixel;
  int64_t* death_pixel;
  int64_t capacity;
  int64_t* pair_offsets;
  int32_t* status;
};

cr_status check_batch_args(cr_context* ctx, const BatchArgs& a) {
  if (!ctx) return fail(CR_ERR_INVALID_ARGUMENT, "ctx is NULL");
  if (!a.packed || !a.pixel_offsets || !a.pair_offsets || !a.status)
    return fail(CR_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  if (a.capacity < 0 || (a.capacity > 0 && (!a.dim || !a.birth || !a.death || !a.birth_pixel || !a.death_pixel)))
    return fail(CR_ERR_INVALID_ARGUMENT, "bad output buffers");
  if (a.flags != 0) return fail(CR_ERR_INVALID_ARGUMENT, "flags must be 0");
  if (a.ndim < 1 || a.ndim > 3) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  if (a.n_images < 1) return fail(CR_ERR_INVALID_ARGUMENT, "n_images must be >= 1");
  if (a.pixel_offsets[0] != 0) return fail(CR_ERR_INVALID_ARGUMENT, "pixel_offsets[0] must be 0");
  return CR_OK;
}

// Enqueues the batched pipeline for ctx->prob / ctx->plan / ctx->scratch:
// every stage, the row gather and the per-image offsets.  No synchronisation.
cr_status enqueue_batch(cr_context* ctx, const BatchArgs& a, hipStream_t s, bool upload) {
  ctx->timing = false;
  ctx->sync_allowed = false;
  uint64_t* cand = nullptr;
  cr_status rc = enqueue_pipeline(ctx, a.packed, s, &cand, upload);
  if (rc != CR_OK) return rc;
  const Plan& p = ctx->plan;
  launch_gather(ctx->tune[grid_ndim(a.ndim)].grid, cand, at<unsigned long long>(ctx, p.counters) + C_CAND,
                (uint64_t)a.capacity, a.packed, at<ImgDesc>(ctx, p.imgs), ctx->prob.L, a.dim, a.birth, a.death,
                a.birth_pixel, a.death_pixel, s);
  launch_img_offsets(at<uint32_t>(ctx, p.img_pairs), at<uint32_t>(ctx, p.img_status), at<Status>(ctx, p.status),
                     a.capacity, a.n_images, a.pair_offsets, a.status, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CR_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return CR_OK;
}

cr_status check_tuning(int ndim, const cr_tuning& t) {
  int ext[3];
  if (!stencil_tile(ndim, t.tile, ext)) return fail(CR_ERR_INVALID_ARGUMENT, "tile variant out of range");
  if (t.grid < 64 || t.grid > 65536) return fail(CR_ERR_INVALID_ARGUMENT, "grid must be in [64, 65536]");
  if (t.long_len < 0 || t.yield_iters < 1 || t.wave_short < 0 || t.wave_yield < 0 || t.group_max < 0 ||
      t.narrow_min < 0)
    return fail(CR_ERR_INVALID_ARGUMENT, "reduction thresholds out of range");
  if (t.front_cap < (int)FRONT_CAP_MIN || t.front_cap > (int)FRONT_CAP_MAX)
    return fail(CR_ERR_INVALID_ARGUMENT, "front_cap out of range");
  return CR_OK;
}

// ---- tuning cache (CR_TUNE_CACHE) --------------------------------------------
constexpr int TUNE_FIELDS = 9;
void tuning_to_array(const cr_tuning& t, int32_t a[TUNE_FIELDS]) {
  const int32_t v[TUNE_FIELDS] = {t.tile, t.grid, t.long_len, t.yield_iters, t.wave_short, t.front_cap,
                                  t.wave_yield, t.group_max, t.narrow_min};
  for (int i = 0; i < TUNE_FIELDS; ++i) a[i] = v[i];
}
cr_tuning tuning_from_array(const int32_t a[TUNE_FIELDS]) {
  cr_tuning t;
  t.tile = a[0]; t.grid = a[1]; t.long_len = a[2]; t.yield_iters = a[3]; t.wave_short = a[4];
  t.front_cap = a[5]; t.wave_yield = a[6]; t.group_max = a[7]; t.narrow_min = a[8];
  return t;
}
int ceil_log2(uint64_t x) {
  int b = 0;
  while (b < 63 && (1ull << b) < x) ++b;
  return b;
}

// Key of a batched call: device arch, ndim, maxdim (clamped), and the image
// and pixel counts rounded up to powers of two.
std::string cache_key(const cr_context* ctx, int n_images, const int64_t* shapes, int ndim, int maxdim) {
  uint64_t P = 0;
  for (int i = 0; i < n_images; ++i) {
    uint64_t p = 1;
    for (int a = 0; a < ndim; ++a) p *= (uint64_t)std::max<int64_t>(1, shapes[(int64_t)i * ndim + a]);
    P += p;
  }
  std::ostringstream k;
  k << ctx->arch << "/nd" << ndim << "/md" << std::min(maxdim, ndim - 1) << "/img" << ceil_log2((uint64_t)n_images)
    << "/px" << ceil_log2(P);
  return k.str();
}

// Reads the cache file: a JSON object of "key": [9 integers] entries.
void cache_load(cr_context* ctx) {
  if (ctx->cache_loaded) return;
  ctx->cache_loaded = true;
  const char* path = getenv("CR_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  size_t i = 0;
  while ((i = text.find('"', i)) != std::string::npos) {
    const size_t j = text.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = text.substr(i + 1, j - i - 1);
    const size_t lb = text.find('[', j), rb = text.find(']', j);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    int32_t a[TUNE_FIELDS];
    int n = 0;
    std::istringstream nums(text.substr(lb + 1, rb - lb - 1));
    std::string tok;
    while (n < TUNE_FIELDS && std::getline(nums, tok, ',')) a[n++] = (int32_t)strtol(tok.c_str(), nullptr, 10);
    if (n == TUNE_FIELDS) ctx->cache[key] = tuning_from_array(a);
    i = rb + 1;
  }
}

// Writes the cache (all entries this context knows) to CR_TUNE_CACHE, through
// a temporary file renamed over it.
void cache_store(cr_context* ctx) {
  const char* path = getenv("CR_TUNE_CACHE");
  if (!path || !*path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& e : ctx->cache) {
    int32_t a[TUNE_FIELDS];
    tuning_to_array(e.second, a);
    fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d, %d, %d, %d, %d]%s\n", e.first.c_str(), a[0], a[1], a[2], a[3], a[4],
            a[5], a[6], a[7], a[8], ++k < ctx->cache.size() ? "," : "");
  }
  fprintf(f, "}\n");
  if (fclose(f) == 0) (void)rename(tmp.c_str(), path);
}

// For the duration of one batched call: the cached tuning of its key, when the
// context has one and the caller has not set the tuning for this ndim.
struct CachedTuning {
  cr_context* ctx = nullptr;
  int nd = 0;
  cr_tuning saved{};
  bool swapped = false;
  CachedTuning(cr_context* c, int n_images, const int64_t* shapes, int ndim, int maxdim) : ctx(c) {
    if (!c || !shapes || n_images < 1 || ndim < 1 || ndim > 3 || maxdim < 0) return;
    nd = grid_ndim(ndim);
    c->stats.tuning_from_cache = 0;
    if (c->tune_set[nd] || c->in_autotune || !getenv("CR_TUNE_CACHE")) return;
    cache_load(c);
    const auto it = c->cache.find(cache_key(c, n_images, shapes, ndim, maxdim));
    if (it == c->cache.end() || check_tuning_quiet(nd, it->second)) return;
    saved = c->tune[nd];
    c->tune[nd] = it->second;
    swapped = true;
    c->stats.tuning_from_cache = 1;
  }
  ~CachedTuning() {
    if (swapped) ctx->tune[nd] = saved;
  }
  // true if t is out of range (a stale or edited cache entry is ignored)
  static bool check_tuning_quiet(int nd, const cr_tuning& t) {
    const std::string keep = g_err;
    const bool bad = check_tuning(nd, t) != CR_OK;
    g_err = keep;
    return bad;
  }
};


// Scratch, problem and plan of a context, swapped in and out around work on a
// graph's own scratch.
struct ScratchState {
  char* scratch;
  size_t bytes;
  Problem prob;
  Plan plan;
};
void swap_state(cr_context* ctx, ScratchState& st) {
  std::swap(ctx->scratch, st.scratch);
  std::swap(ctx->scratch_bytes, st.bytes);
  std::swap(ctx->prob, st.prob);
  std::swap(ctx->plan, st.plan);
}

}  // namespace

struct cr_graph {
  cr_context* ctx = nullptr;
  ScratchState own{};  // the graph's scratch, problem and plan
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* cr_last_error(void) { return g_err.c_str(); }

cr_status cr_create(cr_context** out, int device, cr_alloc_fn alloc, cr_free_fn free_fn, void* user) {
  if (!out) return fail(CR_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(CR_ERR_INVALID_ARGUMENT, "alloc and free must both be given or both be NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(CR_ERR_INVALID_ARGUMENT, "no such device");
  HIP_TRY(hipSetDevice(device));
  cr_context* c = new (std::nothrow) cr_context();
  if (!c) return fail(CR_ERR_OUT_OF_MEMORY, "context allocation failed");
  c->device = device;
  {
    const cr_status src = noalloc_setup(device, &c->noalloc);
    if (src != CR_OK) {
      delete c;
      return src;
    }
  }
  for (int d = 0; d < 4; ++d) c->tune[d] = default_tuning(d);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      c->arch = prop.gcnArchName;
      c->arch = c->arch.substr(0, c->arch.find(':'));
    } else {
      (void)hipGetLastError();
      c->arch = "unknown";
    }
  }
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  if (hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return fail(CR_ERR_HIP, "hipEventCreate failed");
  }
  *out = c;
  return CR_OK;
}

void cr_destroy(cr_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->bwd_flag) (void)hipFree(ctx->bwd_flag);
  if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
  if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
  for (hipEvent_t e : ctx->round_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->ev_ready)
    for (int i = 0; i < EV_N; ++i) (void)hipEventDestroy(ctx->ev[i]);
  delete ctx;
}

cr_status cr_persistence(cr_context* ctx, const float* image, int ndim, const int64_t* shape, int maxdim,
                         uint32_t flags, void* stream, cr_diagram* out) {
  if (!ctx || !out) return fail(CR_ERR_INVALID_ARGUMENT, "ctx or out is NULL");
  out->n = 0;
  out->dim = nullptr; out->birth = nullptr; out->death = nullptr;
  out->birth_pixel = nullptr; out->death_pixel = nullptr; out->block = nullptr;
  if (!image) return fail(CR_ERR_INVALID_ARGUMENT, "image is NULL");
  if (flags & ~CR_FLAG_STAGE_TIMES) return fail(CR_ERR_INVALID_ARGUMENT, "unknown flags");
  HIP_TRY(hipSetDevice(ctx->device));
  if ((flags & CR_FLAG_STAGE_TIMES) && !ctx->ev_ready) {
    for (int i = 0; i < EV_N; ++i) HIP_TRY(hipEventCreate(&ctx->ev[i]));
    ctx->ev_ready = true;
  }
  ctx->timing = (flags & CR_FLAG_STAGE_TIMES) != 0;
  ctx->sync_allowed = true;
  hipStream_t s = (hipStream_t)stream;
  if (ndim < 1 || ndim > 3) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  cr_status rc = build_problem(ctx->prob, 1, nullptr, shape, ndim, maxdim, ctx->tune[grid_ndim(ndim)].tile);
  if (rc != CR_OK) return rc;
  // CR_ARENA_ENTRIES fixes the column arena of the first attempt (e.g. small,
  // to drive the overflow-and-rerun path on a small volume)
  const uint64_t arena_env = env_u64("CR_ARENA_ENTRIES", 0);
  uint64_t arena = arena_env ? arena_env : ctx->arena_entries;
  for (int attempt = 0; attempt < 4; ++attempt) {
    ctx->plan = make_plan(ctx->prob, arena, /*side_h0=*/true);
    rc = ensure_scratch(ctx, ctx->plan.total);
    if (rc != CR_OK) return rc;
    uint64_t* cand = nullptr;
    rc = enqueue_pipeline(ctx, image, s, &cand);
    if (rc != CR_OK) return rc;
    HostCounters h;
    rc = read_counters(ctx, s, &h);
    if (rc != CR_OK) return rc;
    bool arena_over = false;
    rc = status_error(h.st, &arena_over);
    if (rc != CR_OK) {
      if (arena_over && attempt < 3 && ctx->plan.arena_cap < ARENA_MAX) {
        // the arena top counts the entries asked for before the abort, a
        // lower bound of the need
        arena = std::max<uint64_t>(arena * 4, h.cnt[C_ARENA] * 2);
        if (!arena_env) ctx->arena_entries = arena;
        ++ctx->reruns;
        continue;  // rerun the whole pipeline with a larger column arena
      }
      return rc;
    }
    const int64_t n = (int64_t)h.cnt[C_CAND];
    out->n = n;
    if (n == 0) return CR_OK;
    const size_t bytes = align_up(4 * n, 256) * 2 + align_up(4 * n, 256) + 2 * align_up(8 * n, 256);
    void* block = nullptr;
    if (ctx->alloc) {
      block = ctx->alloc(bytes, stream, ctx->user);
    } else if (hipMalloc(&block, bytes) != hipSuccess) {
      (void)hipGetLastError();
      block = nullptr;
    }
    if (!block) {
      out->n = 0;
      return fail(CR_ERR_OUT_OF_MEMORY, "output allocation failed");
    }
    char* b = (char*)block;
    out->block = block;
    out->dim = (int32_t*)b;
    b += align_up(4 * n, 256);
    out->birth = (float*)b;
    b += align_up(4 * n, 256);
    out->death = (float*)b;
    b += align_up(4 * n, 256);
    out->birth_pixel = (int64_t*)b;
    b += align_up(8 * n, 256);
    out->death_pixel = (int64_t*)b;
    launch_gather(ctx->tune[grid_ndim(ndim)].grid, cand, at<unsigned long long>(ctx, ctx->plan.counters) + C_CAND, (uint64_t)n,
                  image,
                  at<ImgDesc>(ctx, ctx->plan.imgs), ctx->prob.L, out->dim, out->birth, out->death,
                  out->birth_pixel, out->death_pixel, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CR_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return CR_OK;
  }
  return fail(CR_ERR_OUT_OF_MEMORY, "column arena still too small after retries");
}

void cr_diagram_free(cr_context* ctx, cr_diagram* d) {
  if (!d) return;
  if (d->block) {
    if (ctx && ctx->free_fn) ctx->free_fn(d->block, nullptr, ctx->user);
    else (void)hipFree(d->block);
  }
  d->n = 0;
  d->block = nullptr;
  d->dim = nullptr; d->birth = nullptr; d->death = nullptr;
  d->birth_pixel = nullptr; d->death_pixel = nullptr;
}

cr_status cr_batched_workspace_size(cr_context* ctx, int n_images, const int64_t* shapes, int ndim, int maxdim,
                                    size_t* bytes) {
  if (!bytes) return fail(CR_ERR_INVALID_ARGUMENT, "NULL argument");
  *bytes = 0;
  if (ndim < 1 || ndim > 3) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  Problem pb;
  const CachedTuning cached(ctx, n_images, shapes, ndim, maxdim);
  const int tile = ctx ? ctx->tune[grid_ndim(ndim)].tile : default_tuning(grid_ndim(ndim)).tile;
  cr_status rc = build_problem(pb, n_images, nullptr, shapes, ndim, maxdim, tile);
  if (rc != CR_OK) return rc;
  *bytes = make_plan(pb, batch_arena(ctx, pb)).total;
  return CR_OK;
}

cr_status cr_reserve(cr_context* ctx, size_t bytes) {
  if (!ctx) return fail(CR_ERR_INVALID_ARGUMENT, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  return ensure_scratch(ctx, bytes);
}

cr_status cr_persistence_batched(cr_context* ctx, int n_images, const float* packed, const int64_t* pixel_offsets,
                                 const int64_t* shapes, int ndim, int maxdim, uint32_t flags, void* stream,
                                 int32_t* dim, float* birth, float* death, int64_t* birth_pixel,
                                 int64_t* death_pixel, int64_t capacity, int64_t* pair_offsets, int32_t* status) {
  const BatchArgs a{n_images, packed, pixel_offsets, shapes, ndim, maxdim, flags, dim, birth, death,
                    birth_pixel, death_pixel, capacity, pair_offsets, status};
  cr_status rc = check_batch_args(ctx, a);
  if (rc != CR_OK) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  ctx->last_batched_valid = false;
  const CachedTuning cached(ctx, n_images, shapes, ndim, maxdim);
  rc = build_problem(ctx->prob, n_images, pixel_offsets, shapes, ndim, maxdim, ctx->tune[grid_ndim(ndim)].tile);
  if (rc != CR_OK) return rc;
  ctx->plan = make_plan(ctx->prob, batch_arena(ctx, ctx->prob));
  rc = ensure_scratch(ctx, ctx->plan.total);
  if (rc != CR_OK) return rc;
  ctx->last_noalloc = false;
  rc = enqueue_batch(ctx, a, s, true);
  if (rc != CR_OK) return rc;
  ctx->last_batched_valid = true;
  return CR_OK;
}

cr_status cr_persistence_batched_noalloc(cr_context* ctx, int n_images, const float* packed,
                                         const int64_t* pixel_offsets, const int64_t* shapes, int ndim, int maxdim,
                                         uint32_t flags, void* stream, int32_t* dim, float* birth, float* death,
                                         int64_t* birth_pixel, int64_t* death_pixel, int64_t capacity,
                                         int64_t* pair_offsets, int32_t* status) {
  const BatchArgs a{n_images, packed, pixel_offsets, shapes, ndim, maxdim, flags, dim, birth, death,
                    birth_pixel, death_pixel, capacity, pair_offsets, status};
  cr_status rc = check_batch_args(ctx, a);
  if (rc != CR_OK) return rc;
  if (!ctx->noalloc) return fail(CR_ERR_INTERNAL, "the context has no static scratch");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  ctx->last_batched_valid = false;
  const CachedTuning cached(ctx, n_images, shapes, ndim, maxdim);
  rc = build_problem(ctx->prob, n_images, pixel_offsets, shapes, ndim, maxdim, ctx->tune[grid_ndim(ndim)].tile);
  if (rc != CR_OK) return rc;
  const Plan plan = make_plan(ctx->prob, noalloc_arena(ctx->prob));
  if (plan.total > CR_NOALLOC_SCRATCH_BYTES)
    return fail(CR_ERR_TOO_LARGE, "the batch needs " + std::to_string(plan.total) +
                                      " bytes of scratch; the static scratch of the allocation-free call holds " +
                                      std::to_string((size_t)CR_NOALLOC_SCRATCH_BYTES));
  ctx->plan = plan;
  // run on this device's static array (the kernels take its device address),
  // then give the context its own scratch back
  char* const own = ctx->scratch;
  const size_t own_bytes = ctx->scratch_bytes;
  ctx->scratch = ctx->noalloc;
  ctx->scratch_bytes = CR_NOALLOC_SCRATCH_BYTES;
  rc = upload_descriptors_pageable(ctx, s);
  if (rc == CR_OK) rc = enqueue_batch(ctx, a, s, false);
  ctx->scratch = own;
  ctx->scratch_bytes = own_bytes;
  if (rc != CR_OK) return rc;
  ctx->last_noalloc = true;
  ctx->last_batched_valid = true;
  return CR_OK;
}

cr_status cr_sync_status(cr_context* ctx, void* stream) {
  if (!ctx) return fail(CR_ERR_INVALID_ARGUMENT, "ctx is NULL");
  if (!ctx->last_batched_valid) return fail(CR_ERR_INVALID_ARGUMENT, "no batched call to report on");
  HIP_TRY(hipSetDevice(ctx->device));
  HostCounters h;
  char* const own = ctx->scratch;
  if (ctx->last_noalloc) ctx->scratch = ctx->noalloc;  // the counters of the last call are there
  cr_status rc = read_counters(ctx, (hipStream_t)stream, &h);
  ctx->scratch = own;
  if (rc != CR_OK) return rc;
  bool arena_over = false;
  rc = status_error(h.st, &arena_over);
  if (arena_over) grow_arena(ctx, ctx->plan.arena_cap, h.cnt[C_ARENA]);
  return rc;
}

// The context's argument-check flag, cleared on stream s (allocated on first use).
cr_status flag_begin(cr_context* ctx, hipStream_t s, uint32_t** bad) {
  if (!ctx->bwd_flag && hipMalloc(&ctx->bwd_flag, 256) != hipSuccess) {
    (void)hipGetLastError();
    ctx->bwd_flag = nullptr;
    return fail(CR_ERR_OUT_OF_MEMORY, "hipMalloc failed");
  }
  *bad = ctx->bwd_flag;
  launch_fill_u32(*bad, 0, 1, s);
  return CR_OK;
}

// Waits for stream s and reports the flag set by the kernels in between.
cr_status flag_end(cr_context* ctx, hipStream_t s, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CR_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  cr_status rc = ensure_stage(ctx, 4);
  if (rc != CR_OK) return rc;
  HIP_TRY(hipMemcpyAsync(ctx->host_stage, ctx->bwd_flag, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  uint32_t hb = 0;
  std::memcpy(&hb, ctx->host_stage, 4);
  if (hb) return fail(CR_ERR_INVALID_ARGUMENT, what);
  return CR_OK;
}

cr_status cr_persistence_backward(cr_context* ctx, const int64_t* birth_pixel, const int64_t* death_pixel,
                                  const float* grad_birth, const float* grad_death, int64_t n_pairs,
                                  float* grad_image, int64_t n_pixels, void* stream) {
  if (!ctx) return fail(CR_ERR_INVALID_ARGUMENT, "ctx is NULL");
  if (n_pairs < 0 || n_pixels < 0) return fail(CR_ERR_INVALID_ARGUMENT, "negative size");
  if (n_pairs == 0) return CR_OK;
  if (!birth_pixel || !death_pixel || !grad_image)
    return fail(CR_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  uint32_t* bad = nullptr;
  cr_status rc = flag_begin(ctx, s, &bad);
  if (rc != CR_OK) return rc;
  launch_backward(birth_pixel, death_pixel, grad_birth, grad_death, n_pairs, grad_image, n_pixels, bad, s);
  return flag_end(ctx, s, "a pixel index is out of range");
}

cr_status cr_lifetime_image(cr_context* ctx, const int32_t* dim, const float* birth, const float* death,
                            const int64_t* birth_pixel, const int64_t* death_pixel, int64_t n_pairs, int location,
                            float* out, int64_t n_pixels, void* stream) {
  if (!ctx) return fail(CR_ERR_INVALID_ARGUMENT, "ctx is NULL");
  if (n_pairs < 0 || n_pixels < 0) return fail(CR_ERR_INVALID_ARGUMENT, "negative size");
  if (location != 0 && location != 1) return fail(CR_ERR_INVALID_ARGUMENT, "location must be 0 (birth) or 1 (death)");
  if (n_pixels > 0 && !out) return fail(CR_ERR_INVALID_ARGUMENT, "out is NULL");
  if (n_pairs > 0 && (!dim || !birth || !death || !(location ? death_pixel : birth_pixel)))
    return fail(CR_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  uint32_t* bad = nullptr;
  cr_status rc = flag_begin(ctx, s, &bad);
  if (rc != CR_OK) return rc;
  launch_fill_u32(reinterpret_cast<uint32_t*>(out), 0, 3 * (uint64_t)n_pixels, s);
  launch_lifetime(dim, birth, death, location ? death_pixel : birth_pixel, n_pairs, out, n_pixels, location, bad, s);
  return flag_end(ctx, s, "a dimension or pixel index is out of range");
}

cr_status cr_pixel_coords(cr_context* ctx, const int64_t* pixel, int64_t n, int64_t base, int ndim,
                          const int64_t* shape, int32_t* xyz, void* stream) {
  if (!ctx) return fail(CR_ERR_INVALID_ARGUMENT, "ctx is NULL");
  if (n < 0) return fail(CR_ERR_INVALID_ARGUMENT, "negative size");
  if (ndim < 1 || ndim > 3 || !shape) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  int64_t ext[3] = {1, 1, 1};
  for (int a = 0; a < ndim; ++a) {
    if (shape[a] < 1 || shape[a] > (1 << 29)) return fail(CR_ERR_INVALID_ARGUMENT, "bad extent");
    ext[3 - ndim + a] = shape[a];
  }
  if (n == 0) return CR_OK;
  if (!pixel || !xyz) return fail(CR_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  uint32_t* bad = nullptr;
  cr_status rc = flag_begin(ctx, s, &bad);
  if (rc != CR_OK) return rc;
  launch_pixel_coords(pixel, n, base, ext, xyz, bad, s);
  return flag_end(ctx, s, "a pixel index is out of range");
}

cr_status cr_get_stage_times(cr_context* ctx, float* ms, int capacity, int* n_stages) {
  if (!ctx || (capacity > 0 && !ms)) return fail(CR_ERR_INVALID_ARGUMENT, "NULL argument");
  for (int i = 0; i < 6 && i < capacity; ++i) ms[i] = ctx->stage_ms[i];
  if (n_stages) *n_stages = 6;
  return CR_OK;
}

cr_status cr_get_stats(cr_context* ctx, cr_stats* out) {
  if (!ctx || !out) return fail(CR_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = ctx->stats;
  out->scratch_bytes = (int64_t)ctx->scratch_bytes;
  return CR_OK;
}


cr_status cr_get_tuning(cr_context* ctx, int ndim, cr_tuning* out) {
  if (!ctx || !out) return fail(CR_ERR_INVALID_ARGUMENT, "NULL argument");
  if (ndim < 1 || ndim > 3) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  *out = ctx->tune[grid_ndim(ndim)];
  return CR_OK;
}

cr_status cr_set_tuning(cr_context* ctx, int ndim, const cr_tuning* t) {
  if (!ctx || !t) return fail(CR_ERR_INVALID_ARGUMENT, "NULL argument");
  if (ndim < 1 || ndim > 3) return fail(CR_ERR_INVALID_ARGUMENT, "ndim must be 1, 2 or 3");
  ndim = grid_ndim(ndim);
  cr_status rc = check_tuning(ndim, *t);
  if (rc != CR_OK) return rc;
  ctx->tune[ndim] = *t;
  ctx->tune_set[ndim] = true;
  return CR_OK;
}

int cr_tile_variants(int ndim) { return (ndim == 2 || ndim == 3) ? N_TILE_VARIANTS : 0; }

cr_status cr_tile_shape(int ndim, int variant, int32_t extents[3]) {
  if (!extents) return fail(CR_ERR_INVALID_ARGUMENT, "extents is NULL");
  int e[3];
  if (!stencil_tile(ndim, variant, e)) return fail(CR_ERR_INVALID_ARGUMENT, "no such tile variant");
  for (int i = 0; i < 3; ++i) extents[i] = e[i];
  return CR_OK;
}

cr_status cr_batched_graph_create(cr_context* ctx, int n_images, const float* packed, const int64_t* pixel_offsets,
                                  const int64_t* shapes, int ndim, int maxdim, uint32_t flags, void* stream,
                                  int32_t* dim, float* birth, float* death, int64_t* birth_pixel,
                                  int64_t* death_pixel, int64_t capacity, int64_t* pair_offsets, int32_t* status,
                                  cr_graph** out) {
  if (!out) return fail(CR_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  const BatchArgs a{n_images, packed, pixel_offsets, shapes, ndim, maxdim, flags, dim, birth, death,
                    birth_pixel, death_pixel, capacity, pair_offsets, status};
  cr_status rc = check_batch_args(ctx, a);
  if (rc != CR_OK) return rc;
  if (!stream) return fail(CR_ERR_INVALID_ARGUMENT, "graph capture needs a non-default stream");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  cr_graph* g = new (std::nothrow) cr_graph();
  if (!g) return fail(CR_ERR_OUT_OF_MEMORY, "graph allocation failed");
  g->ctx = ctx;
  const CachedTuning cached(ctx, n_images, shapes, ndim, maxdim);
  rc = build_problem(g->own.prob, n_images, pixel_offsets, shapes, ndim, maxdim, ctx->tune[grid_ndim(ndim)].tile);
  if (rc != CR_OK) {
    delete g;
    return rc;
  }
  g->own.plan = make_plan(g->own.prob, batch_arena(ctx, g->own.prob));
  g->own.bytes = align_up(g->own.plan.total, 1 << 21);
  if (hipMalloc(&g->own.scratch, g->own.bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return fail(CR_ERR_OUT_OF_MEMORY, "graph scratch allocation failed");
  }
  // work on the graph's scratch: upload the descriptors once, then capture kernels only
  swap_state(ctx, g->own);
  rc = upload_descriptors(ctx, s, true);
  if (rc == CR_OK) {
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      rc = fail(CR_ERR_HIP, std::string("hipStreamBeginCapture failed: ") + hipGetErrorString(e));
    } else {
      rc = enqueue_batch(ctx, a, s, false);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(s, &graph);
      if (rc == CR_OK && e != hipSuccess)
        rc = fail(CR_ERR_HIP, std::string("hipStreamEndCapture failed: ") + hipGetErrorString(e));
      g->graph = graph;
      if (rc == CR_OK) {
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(CR_ERR_HIP, std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e));
      }
    }
  }
  swap_state(ctx, g->own);
  if (rc != CR_OK) {
    cr_graph_destroy(g);
    return rc;
  }
  *out = g;
  return CR_OK;
}

cr_status cr_graph_launch(cr_graph* g, void* stream) {
  if (!g || !g->exec) return fail(CR_ERR_INVALID_ARGUMENT, "graph is NULL");
  HIP_TRY(hipSetDevice(g->ctx->device));
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return CR_OK;
}

cr_status cr_graph_sync_status(cr_graph* g, void* stream) {
  if (!g) return fail(CR_ERR_INVALID_ARGUMENT, "graph is NULL");
  cr_context* ctx = g->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  swap_state(ctx, g->own);
  HostCounters h;
  cr_status rc = read_counters(ctx, (hipStream_t)stream, &h);
  swap_state(ctx, g->own);
  if (rc != CR_OK) return rc;
  bool arena_over = false;
  rc = status_error(h.st, &arena_over);
  if (arena_over) grow_arena(ctx, g->own.plan.arena_cap, h.cnt[C_ARENA]);
  return rc;
}

void cr_graph_destroy(cr_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->own.scratch) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g->own.scratch);
  }
  delete g;
}

cr_status cr_autotune_batched(cr_context* ctx, int n_images, const float* packed, const int64_t* pixel_offsets,
                              const int64_t* shapes, int ndim, int maxdim, void* stream, int32_t* dim, float* birth,
                              float* death, int64_t* birth_pixel, int64_t* death_pixel, int64_t capacity,
                              int64_t* pair_offsets, int32_t* status, int repeats, cr_tuning* chosen) {
  const BatchArgs a{n_images, packed, pixel_offsets, shapes, ndim, maxdim, 0u, dim, birth, death,
                    birth_pixel, death_pixel, capacity, pair_offsets, status};
  cr_status rc = check_batch_args(ctx, a);
  if (rc != CR_OK) return rc;
  if (repeats < 1) return fail(CR_ERR_INVALID_ARGUMENT, "repeats must be >= 1");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int nd = grid_ndim(ndim);
  const cr_tuning start = ctx->tune[nd];
  struct InTune {  // the candidates' own calls do not consult the tuning cache
    cr_context* c;
    ~InTune() { c->in_autotune = false; }
  } in_tune{ctx};
  ctx->in_autotune = true;
  // time one candidate: a warm-up call, then `repeats` timed calls
  auto time_it = [&](const cr_tuning& t, float* ms) -> cr_status {
    ctx->tune[nd] = t;
    for (int r = 0; r <= repeats; ++r) {
      if (r == 1) HIP_TRY(hipEventRecord(e0, s));
      cr_status c = cr_persistence_batched(ctx, n_images, packed, pixel_offsets, shapes, ndim, maxdim, 0, stream,
                                           dim, birth, death, birth_pixel, death_pixel, capacity, pair_offsets,
                                           status);
      if (c != CR_OK) return c;
    }
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    cr_status c = cr_sync_status(ctx, stream);
    if (c != CR_OK) return c;
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    *ms /= (float)repeats;
    return CR_OK;
  };
  cr_tuning best = start;
  float best_ms = 0.0f;
  rc = time_it(best, &best_ms);
  // coordinate descent: one parameter at a time, in the order they matter
  const bool red = ndim == 3 && maxdim >= 1;
  for (int coord = 0; rc == CR_OK && coord < (red ? 9 : 2); ++coord) {
    std::vector<int> vals;
    if (coord == 0) for (int v = 0; v < N_TILE_VARIANTS; ++v) vals.push_back(v);
    if (coord == 1) vals = {512, 1024, 2048, 4096, 8192};
    if (coord == 2) vals = {512, 1024, 2048, 4032};
    if (coord == 3) vals = {8, 16, 32};
    if (coord == 4) vals = {0, 4096, 16384, 65536, 1 << 30};
    if (coord == 5) vals = {16, 128, 1024};
    if (coord == 6) vals = {0, 32, 64, 128};
    if (coord == 7) vals = {0, 128, 256, 1024};
    if (coord == 8) vals = {0, 2048, 8192};
    for (int v : vals) {
      cr_tuning t = best;
      int* field = coord == 0 ? &t.tile : coord == 1 ? &t.grid : coord == 2 ? &t.front_cap
                 : coord == 3 ? &t.long_len : coord == 4 ? &t.wave_short : coord == 5 ? &t.yield_iters
                 : coord == 6 ? &t.wave_yield : coord == 7 ? &t.group_max : &t.narrow_min;
      if (*field == v) continue;
      *field = v;
      float ms = 0.0f;
      rc = time_it(t, &ms);
      if (rc != CR_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tune[nd] = rc == CR_OK ? best : start;
  if (rc == CR_OK && chosen) *chosen = best;
  if (rc == CR_OK && getenv("CR_TUNE_CACHE")) {  // record the choice for this key
    cache_load(ctx);
    ctx->cache[cache_key(ctx, n_images, shapes, ndim, maxdim)] = best;
    cache_store(ctx);
  }
  return rc;
}

}  // extern "C"
