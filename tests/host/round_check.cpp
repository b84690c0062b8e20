// Host build of the library's FP64 -> FP16 / BF16 rounding (wt_internal.h: f64_to_f16_bits, f64_to_bf16_bits,
// FP32 rounded to odd and then to nearest). Reads FP64 bit patterns (hex, one per line) on stdin and prints
// "f16 bf16" result bit patterns (hex), one line each.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "wt_internal.h"
int main() {
  unsigned long long u;
  while (scanf("%llx", &u) == 1) {
    double v;
    std::memcpy(&v, &u, 8);
    printf("%04x %04x\n", (unsigned)wt::f64_to_f16_bits(v), (unsigned)wt::f64_to_bf16_bits(v));
  }
  return 0;
}
