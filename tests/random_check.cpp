// Host check of the library's random block rule (random_block, shared by the
// device kernels): prints the block of draw u for a grid of seeds, counters
// and partition sizes, for comparison with the oracle's own implementation.
#include <cstdio>

#include "../paper_2310_17137_amd/csrc/ap_internal.h"

int main() {
  const unsigned long long seeds[4] = {0ull, 1ull, 12345ull, 0x9000000000000005ull};
  const unsigned long long us[6] = {0ull, 1ull, 2ull, 977ull, 123456789ull, 1ull << 40};
  const int ms[5] = {1, 3, 7, 977, 2147483647};
  for (unsigned long long s : seeds)
    for (unsigned long long u : us)
      for (int m : ms) std::printf("%llu %llu %d %d\n", s, u, m, ap::random_block(s, u, m));
  return 0;
}
