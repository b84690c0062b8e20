// Host build of the library's FP64 -> FP16 / BF16 rounding (wt_internal.h: round_f64_bits). Reads FP64 bit
// patterns (hex, one per line) on stdin and prints "f16 bf16" result bit patterns (hex), one line each.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "wt_internal.h"
int main() {
  unsigned long long u;
  while (scanf("%llx", &u) == 1) {
    double v;
    std::memcpy(&v, &u, 8);
    printf("%04x %04x\n", (unsigned)wt::round_f64_bits<10, 15>(v), (unsigned)wt::round_f64_bits<7, 127>(v));
  }
  return 0;
}
