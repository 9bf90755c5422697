// Shared between the degree-1 reduction kernels and the host layer.
#pragma once
#include "cr_emit.h"

namespace cr {

constexpr uint32_t RED_ITER_CAP = 1u << 24;

struct RedCtx {
  const float* img;
  const ImgDesc* imgs;
  Layout L;
  const uint64_t* skeys;
  const unsigned long long* dim_count;
  const uint8_t* cleared;  // per square rank: 1 = birth of degree 2 (zero column)
  const uint8_t* eapp;     // per edge (4 * anchor pixel + axis): apparent partner square (2 * axis + dir), 0xFF if none
  uint64_t* owner;         // per edge (3 * anchor pixel + axis of the edge): (owning column << 32) |
                           // arena offset of that column's stored list; NO_OWNER if none
  uint64_t* claim;         // per edge: claim_word(round, column) of the leftmost proposer in the latest
                           // round that proposed it (larger rounds win), 0 if none
  uint64_t* piv;           // per column: key of its pivot edge (the proposed one while active)
  uint64_t* col_ptr;       // per column: arena offset of its stored list (length word, then keys)
  uint64_t* arena;         // stored lists: a length word followed by that many ascending keys
  uint64_t arena_cap;
  unsigned long long* arena_top;
  Status* st;
  unsigned long long* work;  // column counter of the wave-mode round
  uint32_t long_len;       // stored columns longer than this continue in wave mode (<= 32: after the
                           // first round thread mode holds a column of up to 32 keys in registers)
  uint32_t yield_iters;    // thread mode hands a column to wave mode after this many additions
  uint32_t wave_short;     // a short list of at most this many columns is run in wave mode too
  uint32_t front_cap;      // keys of the wave-mode LDS front list
  uint32_t mid_cap;        // the wave-mode middle list is folded into the tail beyond this many keys
  uint32_t narrow_min;     // a wave-mode round of at least this many columns runs in the narrow configuration
  uint32_t narrow_cap;     // keys of the narrow configuration's front list
  uint32_t group_max;      // a wave-mode round of at most this many columns runs a workgroup per column
  uint32_t group_cap;      // keys of the group mode's front list
  uint32_t wave_yield;     // a wave- or group-mode column stores itself and continues in the next round
                           // after this many additions in one round (0: never)
  uint32_t yield_few;      // ... except in a round of at most this many columns
  uint32_t* yield_list;    // the next round's long list and its count (set per round)
  unsigned long long* yield_count;
  uint32_t round;          // the round of this launch
  uint32_t async_max;      // a round (after the first) of at most this many columns, and every
                           // later one, is left to the asynchronous tail (0: never)
  unsigned long long* async_base;  // arena offset at the start of the tail (lists from there on
                                   // were written during it)
  const uint64_t* spatial;         // the first round's columns in the order of their squares in the
  const unsigned long long* n_spatial;  // grid (column << 32 | image and index; cleared ones last,
                                        // their field all ones) and their count; count 0 (or no
                                        // array): rank order
};

// Proposal word of column c in round r: the round in the high half (a later
// round always wins, so proposals never need clearing), the column inverted in
// the low half (the leftmost proposer of a round has the largest word).
__device__ inline unsigned long long claim_word(uint32_t round, uint32_t c) {
  return ((unsigned long long)(round + 1) << 32) | (0xFFFFFFFFu - c);
}
constexpr uint64_t NO_OWNER = ~0ull;
constexpr uint64_t ARENA_SLACK = 64;       // readable entries past the arena end (wave loads of 64 words)
constexpr uint64_t ARENA_MAX = (1ull << 32) - ARENA_SLACK;  // offsets fit the low half of an owner word
constexpr uint32_t FRONT_CAP_MIN = 128;    // wave-mode LDS front list capacity bounds
constexpr uint32_t FRONT_CAP_MAX = 4032;  // two wavefronts' front lists, stage and pending list fit 160 KiB of LDS
constexpr uint32_t FRONT_CAP_NARROW_MAX = 320;  // narrow configuration: eight two-wave workgroups per CU

RedCtx make_redctx(const float* img, const ImgDesc* imgs, Layout L, const uint64_t* skeys,
                   const unsigned long long* dim_count, const uint8_t* cleared, const uint8_t* eapp,
                   uint64_t* owner, uint64_t* claim,
                   uint64_t* piv, uint64_t* col_ptr, uint64_t* arena, uint64_t arena_cap,
                   unsigned long long* arena_top, unsigned long long* work, Status* st);

// Enqueues rounds [round0, round0 + nrounds) of the reduction.  lists: two
// ping-pong pairs of column lists (short columns for thread mode, long ones for
// wave mode): round r reads pair r & 1 (round 0 reads every column) and builds
// pair (r + 1) & 1; list 2k is short, 2k+1 long.  counts: three pairs of their
// device counts, rotating: round r reads pair r % 3, builds pair (r + 1) % 3 and
// clears pair (r + 2) % 3 for the round after (all zero before round 0).
// Columns yield after R.wave_yield additions only in rounds below yield_rounds.
void launch_h1_rounds(int grid, const RedCtx& R, uint32_t* lists[4], unsigned long long* counts, int round0,
                      int nrounds, int yield_rounds, hipStream_t s);
// The asynchronous tail: every column still listed after the rounds -- those of
// the round recorded in R.st->tail_round, else of round round_end (the round
// after the last one enqueued) -- reduced to its end without round barriers.
void launch_h1_async(const RedCtx& R, uint32_t* lists[4], unsigned long long* counts, int round_end, hipStream_t s);
void launch_h1_emit(int grid, const RedCtx& R, const EmitCtx& E, hipStream_t s);
// Keys (column << 32 | image << kb | Khalimsky index) of every column, at
// out[column] (a cleared column's low field all ones), and n_out = their number,
// or 0 when there are more than cap squares or the image and index fields
// exceed 32 bits.  Sorted by their low 32 bits they give the first round a
// spatial order.
void launch_h1_spatial_keys(int grid, const RedCtx& R, uint64_t* out, uint64_t cap, unsigned long long* n_out,
                            hipStream_t s);

}  // namespace cr
