/*
 * cr.h -- C ABI of libcr: persistent homology over Z/2 of the weighted cubical
 * complex (V-construction) of 1D signals, 2D images and 3D volumes on one AMD
 * MI355X.
 *
 * The problem is the one Kaji, Sudo and Ahara state for Cubical Ripser
 * (arXiv:2005.12692): an image is a real function on a regular grid (Sec. 2);
 * its cubical complex has the cells of the grid, each valued by the maximum of
 * its vertices (Sec. 2); the result is a set of bars [birth, death) of
 * dimension 0, 1 or 2, with infinite bars marked (Sec. 1).  Connectivity is 4-
 * (2D) or 6-neighbour (3D) (Sec. 2).  Coefficients are Z/2.
 *
 * Conventions for every call:
 *  - Arrays are C order; x (the last axis) is the fastest ("the cell to the
 *    right is (1,0,0)", Fig. 1).  A pixel index is a flat index into the input
 *    buffer passed to the call.
 *  - Values are float32.  -0.0 is read as +0.0.  NaN is an error
 *    (CR_ERR_NAN_INPUT).  +inf and -inf are ordinary values; +inf marks pixels
 *    outside a non-rectangular domain (Sec. 2).
 *  - Only bars of positive length are reported (zero-length pairs are not).  An
 *    essential bar has death = +INFINITY and death_pixel = -1; a full grid has
 *    exactly one, in dimension 0, born at the global minimum.
 *  - birth == image[birth_pixel] and death == image[death_pixel] bit for bit:
 *    the pixel of a cell is its vertex of largest value, ties broken towards
 *    the larger flat index (the paper's "location" of a cycle is "a
 *    representative", Example 4.6; this fixes one).
 *  - Rows of one image are in canonical order: ascending (dim, birth_pixel,
 *    death_pixel), an essential bar after every finite one.  Two runs on the
 *    same input give identical bytes.
 *  - Device pointers are HIP device memory of the context's device; "stream"
 *    is a hipStream_t (NULL = the default stream).  All device work is enqueued
 *    on that stream.
 *  - Every entry point returns a cr_status; on failure no output is written or
 *    allocated and cr_last_error() describes the cause.  No C++ exception
 *    crosses this boundary.  A context is not thread-safe: use one per host
 *    thread.
 */
#ifndef CR_H
#define CR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cr_status {
  CR_OK = 0,
  CR_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad ndim/shape, maxdim < 0, ... */
  CR_ERR_NAN_INPUT = 2,        /* a pixel is NaN */
  CR_ERR_TOO_LARGE = 3,        /* the cell index or key layout would overflow */
  CR_ERR_CAPACITY = 4,         /* a caller-provided buffer is too small */
  CR_ERR_OUT_OF_MEMORY = 5,    /* device or host allocation failed */
  CR_ERR_HIP = 6,              /* a HIP runtime call failed */
  CR_ERR_INTERNAL = 7          /* an internal consistency check failed */
} cr_status;

typedef struct cr_context cr_context;

/* Optional allocator for the plain call's output block (e.g. a framework's
 * caching allocator).  alloc returns device memory of at least `bytes` usable
 * on `stream`, or NULL on failure; free releases it.  With NULL callbacks the
 * library uses hipMalloc / hipFree. */
typedef void* (*cr_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*cr_free_fn)(void* ptr, void* stream, void* user);

/* Creates a context on HIP device `device`.  The context owns its scratch
 * memory (grown on demand, freed by cr_destroy). */
cr_status cr_create(cr_context** out, int device, cr_alloc_fn alloc, cr_free_fn free_fn, void* user);
void cr_destroy(cr_context* ctx);

/* Description of the last failure on the calling thread; valid until the next
 * call on this thread.  Never NULL. */
const char* cr_last_error(void);

/* flags bits */
#define CR_FLAG_STAGE_TIMES 1u /* record HIP events between stages (see cr_get_stage_times) */

/* A diagram in structure-of-arrays form.  The five arrays are device pointers
 * into one block allocated by the plain call (through the context allocator);
 * the caller owns it and releases it with cr_diagram_free. */
typedef struct cr_diagram {
  int64_t n;             /* number of rows (host value) */
  int32_t* dim;          /* 0 .. ndim-1 */
  float* birth;          /* == image[birth_pixel] */
  float* death;          /* == image[death_pixel]; +INFINITY if essential */
  int64_t* birth_pixel;  /* flat index into the input */
  int64_t* death_pixel;  /* -1 if essential */
  void* block;           /* the allocation holding the arrays (NULL if n == 0) */
} cr_diagram;

/* The persistence diagram of one image or volume (Sec. 2: filtration by the
 * maximum over each cell's vertices, sort, apparent pairs, degree 0 by
 * union-find, higher degrees by coboundary reduction with clearing).
 *   image : device, prod(shape) floats, C order; not modified, not retained.
 *   ndim  : 1, 2 or 3 (a 1D signal is a 1 x n image: it lies on one line of
 *           the grid, Sec. 2).  shape : host, ndim extents >= 1, C order.
 *   maxdim: highest dimension reported; >= 0, clamped to ndim-1.
 *   flags : 0 or CR_FLAG_STAGE_TIMES.
 * Host waits: the call returns after the rows are counted (one wait for the
 * stream), then allocates `out` and enqueues the final copy on `stream`.  A
 * volume with maxdim >= 1 also waits while the degree-1 reduction runs: its
 * rounds are enqueued in batches of four and the host reads the count of
 * columns still active one batch behind (an event wait per batch, about 4 on a
 * 256^3 volume; the GPU is never left idle by them), until a round has at most
 * 4096 columns (256 in a call of 8 or more volumes; CR_ASYNC_MAX in the
 * environment overrides it, 0 = never); the columns left are then reduced in
 * one launch without rounds (the asynchronous tail), enqueued right behind the
 * batch running when the count read shows at most twice that many.  If the reduction's
 * column arena (the stored columns) overflows, the whole pipeline is rerun with
 * a larger arena, at most three times (cr_stats.arena_reruns counts reruns);
 * CR_ARENA_ENTRIES in the environment fixes the first attempt's arena.
 * Errors: INVALID_ARGUMENT, NAN_INPUT, TOO_LARGE (more than 2^30 cells),
 * OUT_OF_MEMORY, HIP, INTERNAL. */
cr_status cr_persistence(cr_context* ctx, const float* image, int ndim, const int64_t* shape, int maxdim,
                         uint32_t flags, void* stream, cr_diagram* out);

/* Releases a diagram returned by cr_persistence; sets out->n = 0. */
void cr_diagram_free(cr_context* ctx, cr_diagram* d);

/* Diagrams of n_images images of one ndim and possibly different shapes,
 * packed back to back in one device buffer, computed together in one pass of
 * every stage (the images share each launch).  Each image's diagram is the one
 * cr_persistence gives; the batch serves the paper's many-image use, e.g.
 * lifetime-enhanced images of a whole dataset fed to a network (Example 4.7).
 *   packed        : device floats; image i occupies [pixel_offsets[i], pixel_offsets[i+1]).
 *   pixel_offsets : host, n_images+1 entries, pixel_offsets[0] = 0, consistent with shapes.
 *   shapes        : host, n_images*ndim extents, C order per image (ndim 1, 2 or 3).
 *   dim..death_pixel: device arrays of `capacity` rows (caller-provided).
 *   pair_offsets  : device, n_images+1 int64: rows of image i are
 *                   [pair_offsets[i], pair_offsets[i+1]) in canonical order;
 *                   pair_offsets[n_images] is the total (also when it exceeds capacity).
 *   status        : device, n_images int32, per image: 0 (its rows are complete),
 *                   CR_ERR_NAN_INPUT (it holds NaN), CR_ERR_CAPACITY (its rows do
 *                   not all fit below capacity), or, when the call stopped early
 *                   for every image, CR_ERR_OUT_OF_MEMORY (the column arena of
 *                   the degree-1 reduction ran out) or CR_ERR_INTERNAL.
 * Pixel indices index `packed`.  Never synchronises and never stops short of a
 * complete reduction: it enqueues a fixed budget of reduction rounds (rounds
 * return at once once the columns are few enough for the asynchronous tail, or
 * none are left), then the tail, which reduces the columns still left to the
 * end in one launch.  When the
 * device-side row count exceeds capacity the rows beyond it are dropped and
 * the total in pair_offsets[n_images] tells the capacity needed.  The column
 * arena holds max(the context's arena, 16 entries per pixel) 64-bit entries;
 * after cr_sync_status (or cr_graph_sync_status) has reported that it ran out,
 * the context's arena is at least 4 times larger (CR_ARENA_ENTRIES fixes it).
 * Host-side argument errors are returned directly.  Call cr_sync_status after
 * the stream completes to learn device-side failures (NaN, capacity, arena,
 * internal). */
cr_status cr_persistence_batched(cr_context* ctx, int n_images, const float* packed, const int64_t* pixel_offsets,
                                 const int64_t* shapes, int ndim, int maxdim, uint32_t flags, void* stream,
                                 int32_t* dim, float* birth, float* death, int64_t* birth_pixel,
                                 int64_t* death_pixel, int64_t capacity, int64_t* pair_offsets, int32_t* status);

/* Device scratch bytes a batched call of these images needs (the same
 * arguments as cr_persistence_batched, host only; no device work), and a
 * reservation of that much scratch in the context ahead of time: a batched
 * call whose need fits the reservation allocates no device memory, so it can
 * be enqueued where allocation is not allowed (the pinned host buffer that
 * uploads the image descriptors is allocated by the context's first batched
 * call).  cr_batched_workspace_size takes ctx = NULL for a context's defaults
 * (then it makes no HIP call at all).  cr_reserve never shrinks the scratch; it
 * synchronises the device when it has to grow it.  Errors: INVALID_ARGUMENT,
 * TOO_LARGE (more than 2^30 cells in an image, 2^31 pixels or 2^32 cells in a
 * call, or a key layout beyond 64 bits), OUT_OF_MEMORY. */
cr_status cr_batched_workspace_size(cr_context* ctx, int n_images, const int64_t* shapes, int ndim, int maxdim,
                                    size_t* bytes);
cr_status cr_reserve(cr_context* ctx, size_t bytes);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): cr_persistence_batched with
 * the same arguments and results, run on a scratch array that the library
 * holds in static device memory, CR_NOALLOC_SCRATCH_BYTES on every GPU it runs
 * on (set up by cr_create, kept until the process ends).  The call makes no
 * device or pinned-host allocation: the image descriptors are copied from
 * pageable host memory, and the column arena of a volume's reduction is 16
 * entries per pixel (CR_ARENA_ENTRIES overrides it).  A batch whose scratch
 * (cr_batched_workspace_size's plan with that arena) exceeds the array is
 * rejected with CR_ERR_TOO_LARGE before any device work.  Every call on one GPU
 * shares that GPU's array, from any context: calls that overlap on one GPU
 * (other streams, other contexts or threads) race and give undefined results;
 * the array keeps the last call's contents, and the call clears what must
 * start at zero.  cr_sync_status reports on it like on a batched call until
 * the next batched call on the context. */
#define CR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
cr_status cr_persistence_batched_noalloc(cr_context* ctx, int n_images, const float* packed,
                                         const int64_t* pixel_offsets, const int64_t* shapes, int ndim, int maxdim,
                                         uint32_t flags, void* stream, int32_t* dim, float* birth, float* death,
                                         int64_t* birth_pixel, int64_t* death_pixel, int64_t capacity,
                                         int64_t* pair_offsets, int32_t* status);

/* Synchronises `stream` and returns the device-side status of the last
 * batched call on this context (CR_OK, CR_ERR_NAN_INPUT, CR_ERR_CAPACITY,
 * CR_ERR_OUT_OF_MEMORY for scratch exhaustion, or CR_ERR_INTERNAL). */
cr_status cr_sync_status(cr_context* ctx, void* stream);

/* Gradient of a loss L(birth, death) with respect to the image.  A cell takes
 * the value of its largest vertex (the V-construction, Sec. 2), so each bar end
 * is the value of one pixel, its location (Example 4.6):
 * birth_i = image[birth_pixel_i] and death_i = image[death_pixel_i], hence
 *   grad_image[birth_pixel_i] += grad_birth_i,  grad_image[death_pixel_i] += grad_death_i
 * (rows with death_pixel -1 contribute only their birth).  All arrays are device
 * arrays of n_pairs rows; grad_birth or grad_death may be NULL (zero).
 * grad_image (n_pixels floats) is accumulated into, not overwritten.  Pixel
 * indices outside [0, n_pixels) give CR_ERR_INVALID_ARGUMENT (after the stream
 * completes: this call synchronises once).  Sums over rows sharing a pixel use
 * float atomics, so their rounding order is not fixed. */
cr_status cr_persistence_backward(cr_context* ctx, const int64_t* birth_pixel, const int64_t* death_pixel,
                                  const float* grad_birth, const float* grad_death, int64_t n_pairs,
                                  float* grad_image, int64_t n_pixels, void* stream);

/* The lifetime-enhanced image of Sec. 4 (localised features), its three
 * persistence channels: for d = 0, 1, 2,
 *   out[d * n_pixels + p] = max (death_i - birth_i) over the rows i with
 *                           dim_i == d located at pixel p, and 0 where none is,
 * the difference taken in float32.  A row is located at its birth pixel
 * (location 0) or at its death pixel (location 1, the paper's
 * "--location death"; rows with death_pixel -1 are then skipped).  With birth
 * locations an essential bar's lifetime is +INFINITY.  Rows with a lifetime
 * that is not positive leave the image alone.  The rows are device arrays of
 * n_pairs entries in any order: a plain diagram with n_pixels the image's
 * size, or a batched one with n_pixels the packed size (image i's channel d is
 * then out[d * n_pixels + pixel_offsets[i] ...]).  out: device, 3 * n_pixels
 * floats, overwritten.  Stacking the image on top gives the paper's
 * four-channel image.  A dimension outside 0..2 or a pixel index outside
 * [0, n_pixels) gives CR_ERR_INVALID_ARGUMENT once the stream has completed
 * (this call synchronises `stream` once). */
cr_status cr_lifetime_image(cr_context* ctx, const int32_t* dim, const float* birth, const float* death,
                            const int64_t* birth_pixel, const int64_t* death_pixel, int64_t n_pairs, int location,
                            float* out, int64_t n_pixels, void* stream);

/* Locations of pixels as the (x, y, z) columns of the paper's output rows
 * (Sec. 3: the location of the cell giving birth to, or killing, a cycle):
 * for each of the n device entries of `pixel`, q = pixel[i] - base is a flat
 * C-order index into an image of `shape` (host, ndim extents, ndim 1..3) and
 *   xyz[3 i] = x (the last axis), xyz[3 i + 1] = y, xyz[3 i + 2] = z,
 * axes the image does not have being 0; pixel[i] == -1 (no death pixel) gives
 * (-1, -1, -1).  `base` is 0 for a plain diagram and pixel_offsets[i] for image
 * i of a batched one.  xyz: device, 3 n int32.  An index outside the image
 * gives CR_ERR_INVALID_ARGUMENT once the stream has completed (this call
 * synchronises `stream` once). */
cr_status cr_pixel_coords(cr_context* ctx, const int64_t* pixel, int64_t n, int64_t base, int ndim,
                          const int64_t* shape, int32_t* xyz, void* stream);

/* Sizes seen by the last plain or batched call on this context. */
typedef struct cr_stats {
  int64_t n_pixels;
  int64_t n_cells;
  int64_t survivors[4]; /* cells of each dimension left after apparent pairs */
  int64_t n_rows;       /* rows of positive length, essential bars included */
  int64_t arena_used;   /* 64-bit entries of column storage used by the reduction */
  int64_t red_adds;     /* column additions performed by the reduction */
  int64_t red_merged;   /* list entries read by those additions */
  int64_t red_rounds;   /* rounds of the degree-1 reduction before its asynchronous tail (plain call) */
  int64_t arena_reruns; /* plain calls on this context that reran with a larger column arena */
  int64_t scratch_bytes; /* device scratch the context owns now (0 until a call needs it) */
  int64_t tuning_from_cache; /* 1 if the last batched call ran with a CR_TUNE_CACHE entry */
} cr_stats;
cr_status cr_get_stats(cr_context* ctx, cr_stats* out);

/* Stage durations in milliseconds of the last plain call made with
 * CR_FLAG_STAGE_TIMES, measured with HIP events on the call's stream, in this
 * order: 0 stencil (filtration, apparent pairs, survivor compaction), 1 sort of
 * the surviving cells, 2 degree 0 (forest roots and union-find), 3 degree 1
 * (dual union-find of an image, or the coboundary reduction of a volume),
 * 4 degree 2 of a volume (dual union-find), 5 sort of the output rows.  A stage
 * that did not run reports 0.  Writes min(capacity, 6) values and sets
 * *n_stages = 6. */
cr_status cr_get_stage_times(cr_context* ctx, float* ms, int capacity, int* n_stages);

/* ---- launch parameters, autotuning and graphs (batched form) ------------------ */

/* Launch parameters of one ndim.  They change speed only: every setting gives
 * the same diagrams. */
typedef struct cr_tuning {
  int32_t tile;         /* stencil tile shape, 0 .. cr_tile_variants(ndim)-1 (see cr_tile_shape);
                           a call whose images all have one row (1D signals) uses a one-row
                           layout of its own instead */
  int32_t grid;         /* workgroups of the grid-stride kernels (union-find, output), 64 .. 65536 */
  int32_t long_len;     /* degree-1 reduction of a volume: a stored column longer than this
                           continues one per wavefront instead of one per thread (values
                           above 32, the keys a thread holds in registers, act as 32) */
  int32_t yield_iters;  /* ... a column reduced one per thread moves to a wavefront after this
                           many additions (>= 1) */
  int32_t wave_short;   /* ... a list of at most this many short columns is run one per wavefront */
  int32_t front_cap;    /* ... keys of a wavefront's LDS front list, 128 .. 4032 */
  int32_t wave_yield;   /* ... a column reduced one per wavefront (or workgroup) is stored
                           after this many additions in one round and continues in the next,
                           so that the rounds stay short and the columns of different images
                           (or regions) do not wait for one long column; 0 = never.  In a
                           batched call it applies to the first 64 rounds only. */
  int32_t group_max;    /* ... a round of at most this many long columns runs one workgroup
                           per column; 0 = automatic (256 for a call of 8 or more volumes,
                           else 1024).  Rounds small enough for the asynchronous tail do
                           not run at all. */
  int32_t narrow_min;   /* ... a round of at least this many long columns runs the narrow
                           wavefront configuration; 0 = automatic (2048 for a call of 8 or
                           more volumes, else 8192) */
} cr_tuning;

/* The parameters the context uses for ndim (1, 2 or 3; 1D signals share the
 * 2D setting), and a validated setter (INVALID_ARGUMENT for a value out of
 * range).
 *
 * Tuning cache: when the environment variable CR_TUNE_CACHE names a file, the
 * autotuner records its choice there (a JSON object, one entry per key
 * "<gcn arch>/nd<ndim>/md<maxdim>/img<log2 images>/px<log2 pixels>", the
 * exponents rounded up), and a batched call or graph of a context on which
 * cr_set_tuning was not called for that ndim uses the entry of its key when
 * there is one (the file is read once per context). */
cr_status cr_get_tuning(cr_context* ctx, int ndim, cr_tuning* out);
cr_status cr_set_tuning(cr_context* ctx, int ndim, const cr_tuning* t);

/* Number of stencil tile shapes for ndim (0 for another ndim), and the
 * extents (z, y, x) of shape `variant`; a 2D tile has z extent 1. */
int cr_tile_variants(int ndim);
cr_status cr_tile_shape(int ndim, int variant, int32_t extents[3]);

/* Autotuner: runs the batched call on the caller's batch (same arguments and
 * output buffers as cr_persistence_batched) for candidate parameter sets --
 * one parameter at a time: tile shape, grid, then for volumes with maxdim >= 1
 * the front-list capacity and the reduction thresholds -- each as one warm-up
 * call plus `repeats` calls
 * timed with HIP events on `stream`, keeps the fastest, makes it the context's
 * setting for ndim and copies it to *chosen (may be NULL).  Synchronises;
 * returns the first error of a candidate run (the previous setting is then
 * kept).  The outputs hold the diagrams of the last run. */
cr_status cr_autotune_batched(cr_context* ctx, int n_images, const float* packed, const int64_t* pixel_offsets,
                              const int64_t* shapes, int ndim, int maxdim, void* stream, int32_t* dim, float* birth,
                              float* death, int64_t* birth_pixel, int64_t* death_pixel, int64_t capacity,
                              int64_t* pair_offsets, int32_t* status, int repeats, cr_tuning* chosen);

/* A batched call captured in a HIP graph: every kernel of cr_persistence_batched
 * for these arguments (shapes, device buffers and the context's current
 * tuning fixed at creation), on scratch memory the graph owns, so that a
 * replay enqueues no host work and allocates nothing.  Creation uploads the
 * image descriptors (synchronously) and captures on `stream`, which must not be
 * the default stream.  cr_graph_launch replays it on any stream of the device;
 * the input buffer is read at replay time, so new pixel values of the same
 * shapes need no new graph.  cr_graph_sync_status synchronises `stream` and
 * reports the device-side status of the last replay (as cr_sync_status).
 * The context must outlive the graph; replays of one graph must not overlap. */
typedef struct cr_graph cr_graph;
cr_status cr_batched_graph_create(cr_context* ctx, int n_images, const float* packed, const int64_t* pixel_offsets,
                                  const int64_t* shapes, int ndim, int maxdim, uint32_t flags, void* stream,
                                  int32_t* dim, float* birth, float* death, int64_t* birth_pixel,
                                  int64_t* death_pixel, int64_t capacity, int64_t* pair_offsets, int32_t* status,
                                  cr_graph** out);
cr_status cr_graph_launch(cr_graph* g, void* stream);
cr_status cr_graph_sync_status(cr_graph* g, void* stream);
void cr_graph_destroy(cr_graph* g);

#ifdef __cplusplus
}
#endif
#endif /* CR_H */
