// Host check of the library's division by a per-frame divisor (wt_internal.h: fastdiv) against the hardware
// divide: edge divisors (1, powers of two and their neighbours, 2^31, 2^32 - 1), random divisors of every
// magnitude, and for each, edge numerators, multiples of d and their predecessors, and random numerators.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "wt_internal.h"
int main() {
  std::mt19937_64 rng(1);
  uint64_t bad = 0, n_checked = 0;
  std::vector<uint32_t> ds = {1, 2, 3, 5, 7, 640, 641, 1279, 1280, 1920, 1921, 2000, 3840, 4095, 4096, 65535, 65536,
                              65537, 0x7fffffffu, 0x80000000u, 0x80000001u, 0xfffffffeu, 0xffffffffu};
  for (int i = 0; i < 2000; ++i) ds.push_back((uint32_t)(rng() >> (32 + rng() % 32)) | 1u);
  for (int i = 0; i < 2000; ++i) ds.push_back((uint32_t)(rng() % 70000) + 1);
  for (uint32_t d : ds) {
    if (d == 0) continue;
    wt::FastDiv f = wt::make_fastdiv(d);
    std::vector<uint32_t> ns = {0, 1, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0xffffffffu, 0xfffffffeu, 0x80000000u};
    for (int k = 0; k < 3000; ++k) ns.push_back((uint32_t)rng());
    for (int k = 1; k < 200; ++k) { uint64_t q = (uint64_t)k * d; if (q < (1ull << 32)) { ns.push_back((uint32_t)q); ns.push_back((uint32_t)(q - 1)); } }
    for (uint32_t n : ns) { ++n_checked; if (wt::fastdiv(n, f) != n / d) { if (bad < 10) printf("bad n=%u d=%u got %u want %u\n", n, d, wt::fastdiv(n, f), n / d); ++bad; } }
  }
  printf("checked %llu, bad %llu\n", (unsigned long long)n_checked, (unsigned long long)bad);
  return bad != 0;
}
