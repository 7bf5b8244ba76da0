// Queue claims of the persistent traversal kernel: the index arithmetic by which a wave hands
// queue entries to its idle lanes.  Plain integer code, compiled for the device (the traversal
// kernel) and for the host (a CPU model that replays it over random schedules with bounds
// assertions), so the two run the same arithmetic.
//
// The entries [0, n) of one depth are split into kWorkSlices contiguous slices, each with its
// own claim counter.  A wave keeps a wave-uniform pool [pool_next, pool_end) of entries it
// claimed but has not handed out.  When its idle lanes need `want` entries and the pool holds
// fewer, it adds `take` = max(chunk, want - have) to the counter of its current slice (one
// atomic) and clamps the returned range to the slice; a claim that reaches the slice's end
// moves the wave on to the next slice, and once it has seen every slice end it is drained.
//
// Invariants (checked by the CPU model): every index handed to a lane lies in [0, n) and in the
// slice it was claimed from; no index is handed out twice; pool_next <= pool_end <= the end of
// the slice the pool came from; every entry is handed out once all waves are drained.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nrrs {

constexpr uint32_t kClaimNone = 0xFFFFFFFFu;

struct ClaimState {
  uint32_t pool_next, pool_end;  // claimed entries not handed out yet
  uint32_t slice, slices_left;   // current slice, slices this wave has not seen end
  uint32_t s_lo, s_hi;           // bounds of the current slice
  bool drained;                  // every slice has ended for this wave
};

__host__ __device__ inline uint32_t slice_bound(uint32_t n, uint32_t slice, uint32_t slices) {
  return (uint32_t)((uint64_t)n * slice / slices);
}

__host__ __device__ inline ClaimState claim_start(uint32_t n, uint32_t first_slice, uint32_t slices) {
  ClaimState c;
  c.pool_next = c.pool_end = 0;
  c.slice = first_slice % slices;
  c.slices_left = slices;
  c.s_lo = slice_bound(n, c.slice, slices);
  c.s_hi = slice_bound(n, c.slice + 1, slices);
  c.drained = n == 0;
  return c;
}

// Entries the pool holds, and whether the wave must claim from a counter for `want` lanes.
__host__ __device__ inline bool claim_needed(const ClaimState& c, uint32_t want) {
  return c.pool_end - c.pool_next < want && !c.drained;
}

// Amount added to the slice counter by one claim.
__host__ __device__ inline uint32_t claim_amount(const ClaimState& c, uint32_t want, uint32_t chunk) {
  const uint32_t have = c.pool_end - c.pool_next;
  return want - have > chunk ? want - have : chunk;
}

// Entry for the idle lane of rank `rank` (0-based among `want` idle lanes) and the wave's new
// state.  `claimed`: a claim was made, `off` being the counter value before adding `take`.
// Returns kClaimNone when no entry is left for the lane.
__host__ __device__ inline uint32_t claim_hand_out(ClaimState& c, uint32_t n, uint32_t slices, uint32_t want,
                                                   uint32_t rank, bool claimed, uint32_t off, uint32_t take) {
  const uint32_t have = c.pool_end - c.pool_next;
  uint32_t my = rank < have ? c.pool_next + rank : kClaimNone;
  if (claimed) {
    const uint32_t size = c.s_hi - c.s_lo;
    const uint32_t fresh = c.s_lo + (off < size ? off : size);
    const uint64_t e = (uint64_t)off + take;
    const uint32_t end = c.s_lo + (uint32_t)(e < size ? e : size);
    if (rank >= have) my = fresh + (rank - have) < end ? fresh + (rank - have) : kClaimNone;
    c.pool_end = end;
    const uint32_t next = fresh + (want - have);
    c.pool_next = next < end ? next : end;
    if (end == c.s_hi) {
      --c.slices_left;
      c.drained = c.slices_left == 0;
      c.slice = c.slice + 1 == slices ? 0 : c.slice + 1;
      c.s_lo = slice_bound(n, c.slice, slices);
      c.s_hi = slice_bound(n, c.slice + 1, slices);
    }
  } else {
    c.pool_next += want < have ? want : have;
  }
  return my;
}

// No entry is left for this wave: drained and the pool is empty.
__host__ __device__ inline bool claim_exhausted(const ClaimState& c) { return c.drained && c.pool_next >= c.pool_end; }

}  // namespace nrrs
