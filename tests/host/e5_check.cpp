// Host build of the library's E5B9G9R9 packing (wt_common.h: e5_pack, the code the tile kernels run). Reads three
// FP32 bit patterns (hex) per line on stdin and prints the packed word (hex), one line each.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "wt_common.h"
int main() {
  unsigned a, b, c;
  while (scanf("%x %x %x", &a, &b, &c) == 3) {
    float r, g, bl;
    std::memcpy(&r, &a, 4);
    std::memcpy(&g, &b, 4);
    std::memcpy(&bl, &c, 4);
    printf("%08x\n", (unsigned)wt::e5_pack(r, g, bl));
  }
  return 0;
}
