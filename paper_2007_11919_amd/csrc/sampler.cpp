// Landmark sampler (host).  Section 3.1 draws the landmark subset at
// random; the draw is pinned to a published recipe so that any two
// implementations agree bit for bit:
//   SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) for raw 64-bit words,
//   Lemire's multiply-and-reject method (ACM TOMACS 2019) for a uniform
//   integer below k, and a partial Fisher-Yates shuffle of 0..n-1 whose
//   first l slots are the landmarks, returned in ascending order.
#include <stdint.h>

#include <algorithm>
#include <unordered_map>
#include <vector>

#include "mds_internal.h"

namespace mds {
namespace {

class SplitMix64 {
 public:
  explicit SplitMix64(uint64_t seed) : s_(seed) {}
  uint64_t operator()() {
    s_ += 0x9E3779B97F4A7C15ull;
    uint64_t z = s_;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }

 private:
  uint64_t s_;
};

// uniform in [0, k), k >= 1
uint64_t below(SplitMix64& g, uint64_t k) {
  unsigned __int128 prod = (unsigned __int128)g() * k;
  uint64_t low = (uint64_t)prod;
  if (low < k) {
    const uint64_t threshold = (0 - k) % k;  // (2^64 - k) mod k
    while (low < threshold) {
      prod = (unsigned __int128)g() * k;
      low = (uint64_t)prod;
    }
  }
  return (uint64_t)(prod >> 64);
}

}  // namespace

void sample_landmarks_host(int64_t n, int64_t l, uint64_t seed, int64_t* out) {
  SplitMix64 g(seed);
  // Virtual identity permutation: only displaced slots are stored.
  std::unordered_map<int64_t, int64_t> slot;
  slot.reserve((size_t)(2 * l + 16));
  auto at = [&slot](int64_t i) {
    auto it = slot.find(i);
    return it == slot.end() ? i : it->second;
  };
  for (int64_t i = 0; i < l; ++i) {
    const int64_t j = i + (int64_t)below(g, (uint64_t)(n - i));
    const int64_t vi = at(i), vj = at(j);
    slot[i] = vj;
    slot[j] = vi;
  }
  for (int64_t i = 0; i < l; ++i) out[i] = at(i);
  std::sort(out, out + l);
}

}  // namespace mds

extern "C" uint64_t mds_debug_bounded(uint64_t seed, uint64_t k, int32_t draws, uint64_t* out) {
  // Test hook: the first `draws` bounded draws below k from SplitMix64(seed).
  mds::SplitMix64 g(seed);
  for (int32_t i = 0; i < draws; ++i) out[i] = mds::below(g, k);
  return draws;
}
