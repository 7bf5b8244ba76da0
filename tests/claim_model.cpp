// CPU model of the persistent traversal's queue claims: waves of 64 lanes take queue entries
// through the same claim arithmetic as the kernel (claim.hpp), under random schedules (which
// wave runs next, how long each ray takes), with assertions on every index handed out.
// Prints "claims ok <cases>" and exits 0, or prints the failed check and exits 1.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2510_07868_amd/csrc/claim.hpp"

using nrrs::ClaimState;

namespace {

constexpr uint32_t kSlices = 8;  // the kernel's kWorkSlices
int failures = 0;

#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      std::printf("FAILED %s: ", #cond);                  \
      std::printf(__VA_ARGS__);                           \
      std::printf("\n");                                  \
      ++failures;                                         \
      return false;                                       \
    }                                                     \
  } while (0)

struct Wave {
  ClaimState c;
  bool exhausted = false;
  uint32_t steps[64] = {};  // remaining steps of each lane's ray (0 = idle)
  uint32_t slice_lo[64] = {}, slice_hi[64] = {};
};

// One depth of one launch: `waves` waves over n entries.
bool run_case(uint32_t n, uint32_t waves, uint32_t chunk, uint32_t refill, uint32_t max_steps, uint64_t seed) {
  std::mt19937_64 rng(seed);
  std::vector<uint32_t> counter(kSlices, 0);
  std::vector<uint8_t> taken(n, 0);
  std::vector<Wave> w(waves);
  for (uint32_t k = 0; k < waves; ++k) w[k].c = nrrs::claim_start(n, k / 2, kSlices);  // 2 waves per block
  uint32_t live = waves;
  std::vector<uint8_t> done(waves, 0);
  uint64_t guard = 0;
  while (live) {
    CHECK(++guard < 100000000ull, "no progress n=%u", n);
    const uint32_t k = (uint32_t)(rng() % waves);
    if (done[k]) continue;
    Wave& v = w[k];
    // claims for the idle lanes (the kernel's condition: `refill` idle lanes, or all idle)
    if (!v.exhausted) {
      uint64_t idle = 0;
      for (int l = 0; l < 64; ++l)
        if (v.steps[l] == 0) idle |= 1ull << l;
      const uint32_t want = (uint32_t)__builtin_popcountll(idle);
      if (idle && (want >= refill || idle == ~0ull)) {
        const ClaimState before = v.c;
        const bool claim = nrrs::claim_needed(v.c, want);
        uint32_t off = 0, take = 0;
        if (claim) {
          take = nrrs::claim_amount(v.c, want, chunk);
          off = counter[v.c.slice];
          counter[v.c.slice] += take;
          CHECK((uint64_t)counter[v.c.slice] < (1ull << 32), "counter wrap");
        }
        uint32_t rank = 0;
        for (int l = 0; l < 64; ++l) {
          if (!(idle >> l & 1)) continue;
          ClaimState c = before;  // every lane evaluates the same wave-uniform update
          const uint32_t my = nrrs::claim_hand_out(c, n, kSlices, want, rank, claim, off, take);
          if (rank == 0) v.c = c;
          CHECK(c.pool_next == v.c.pool_next && c.pool_end == v.c.pool_end && c.slice == v.c.slice,
                "state not uniform");
          if (my != nrrs::kClaimNone) {
            CHECK(my < n, "index %u beyond n=%u", my, n);
            CHECK(!taken[my], "index %u handed out twice (n=%u)", my, n);
            // the entry comes from the old pool or from the slice just claimed from
            const bool from_pool = rank < before.pool_end - before.pool_next;
            if (from_pool) {
              CHECK(my >= before.pool_next && my < before.pool_end, "pool entry %u outside the pool", my);
            } else {
              CHECK(my >= before.s_lo && my < before.s_hi, "entry %u outside its slice [%u,%u)", my, before.s_lo,
                    before.s_hi);
            }
            taken[my] = 1;
            v.steps[l] = 1 + (uint32_t)(rng() % max_steps);
          }
          ++rank;
        }
        CHECK(v.c.pool_next <= v.c.pool_end, "pool_next %u > pool_end %u", v.c.pool_next, v.c.pool_end);
        CHECK(v.c.pool_end <= n, "pool_end %u > n %u", v.c.pool_end, n);
        CHECK(v.c.s_lo <= v.c.s_hi && v.c.s_hi <= n, "slice bounds");
        v.exhausted = nrrs::claim_exhausted(v.c);
      }
    }
    // one traversal step for every busy lane
    bool busy = false;
    for (int l = 0; l < 64; ++l)
      if (v.steps[l]) {
        --v.steps[l];
        busy = true;
      }
    if (!busy && v.exhausted) {
      done[k] = 1;
      --live;
    }
  }
  for (uint32_t i = 0; i < n; ++i) CHECK(taken[i], "entry %u never handed out (n=%u waves=%u)", i, n, waves);
  return true;
}

}  // namespace

int main() {
  const uint32_t ns[] = {0, 1, 3, 7, 8, 9, 63, 64, 65, 1000, 4099, 65537, 300001};
  const uint32_t wavess[] = {1, 3, 16, 112};
  const uint32_t chunks[] = {0, 32, 64, 128, 4096};
  const uint32_t refills[] = {1, 8, 16, 48, 64};
  int cases = 0;
  uint64_t seed = 1;
  for (uint32_t n : ns)
    for (uint32_t waves : wavess)
      for (uint32_t chunk : chunks)
        for (uint32_t refill : refills) {
          if (n > 100000 && (waves < 16 || refill != 16)) continue;
          run_case(n, waves, chunk, refill, 1 + (uint32_t)(seed % 40), seed);
          ++seed;
          ++cases;
        }
  if (failures) {
    std::printf("claims: %d failed checks\n", failures);
    return 1;
  }
  std::printf("claims ok %d\n", cases);
  return 0;
}
