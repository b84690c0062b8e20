// Host check of the library's -ln(1 - alpha) (wt_internal.h: neg_log1m) against the C library's log1p in double:
// every FP32 alpha below 2^-100 and above 2^-16 up to 1/2 at a stride of 7 bit patterns plus every one of the
// first and last 4096 (the series branch, denormals included), and every 61st FP32 value in (1/2, 1 - 2^-24]
// (the base-2 logarithm branch, here with the host's log2f); maximum relative error in units of 2^-24.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "wt_internal.h"
int main() {
  double worst_lo = 0.0, worst_hi = 0.0;
  float at_lo = 0.f, at_hi = 0.f;
  auto check = [](float al, double& worst, float& at) {
    const double ref = -std::log1p(-(double)al);
    const double got = (double)wt::neg_log1m(al);
    const double err = ref == 0.0 ? std::fabs(got) : std::fabs(got - ref) / ref;
    if (err > worst) { worst = err; at = al; }
  };
  const uint32_t half = 0x3f000000u, top = 0x3f7fffffu;  // 0.5f and 1 - 2^-24
  auto lo = [&](uint32_t b) { float al; std::memcpy(&al, &b, 4); check(al, worst_lo, at_lo); };
  auto hi = [&](uint32_t b) { float al; std::memcpy(&al, &b, 4); check(al, worst_hi, at_hi); };
  for (uint32_t b = 0; b < 4096; ++b) { lo(b); lo(half - b); }
  for (uint32_t b = 0; b <= 0x0d800000u; b += 7) lo(b);           // up to 2^-100
  for (uint32_t b = 0x37800000u; b <= half; b += 7) lo(b);          // 2^-16 .. 1/2
  for (uint32_t b = half + 1; b <= top; b += 61) hi(b);
  hi(top);
  for (uint32_t b = top - 4096; b <= top; ++b) hi(b);
  const double ulp = std::ldexp(1.0, -24);
  printf("series: max %.2f ulp at %.9g; log2: max %.2f ulp at %.9g\n", worst_lo / ulp, at_lo, worst_hi / ulp, at_hi);
  return !(worst_lo < 4 * ulp && worst_hi < 4 * ulp);
}
