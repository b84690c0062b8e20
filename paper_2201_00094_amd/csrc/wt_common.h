// Device helpers shared by the libwt kernels: tile addressing, storage conversions, wavefront reductions.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_internal.h"

namespace wt {

struct bf16_t {
  uint16_t u;
};

template <typename T>
__device__ __forceinline__ float widen(T v);
template <>
__device__ __forceinline__ float widen<float>(float v) { return v; }
template <>
__device__ __forceinline__ float widen<__half>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ float widen<bf16_t>(bf16_t v) { return __uint_as_float((uint32_t)v.u << 16); }

// Round an FP64 on-chip sum to the storage type once, to nearest even (FP32 by the hardware conversion, FP16 and
// BF16 through FP32 rounded to odd).
template <typename T>
__device__ __forceinline__ T narrow_d(double v);
template <>
__device__ __forceinline__ float narrow_d<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ __half narrow_d<__half>(double v) { return __ushort_as_half(f64_to_f16_bits(v)); }
template <>
__device__ __forceinline__ bf16_t narrow_d<bf16_t>(double v) { return bf16_t{f64_to_bf16_bits(v)}; }


// E5B9G9R9 coefficient storage (section 2.1): one 32-bit word per coefficient index holds the magnitudes of the
// three channels' coefficients, a shared 5-bit exponent (bias 15) in bits 27-31 and 9-bit mantissas without an
// implicit one, B in bits 18-26, G in 9-17, R in 0-8; value = mantissa * 2^(e - 24).
struct e5_t {
  uint32_t u;
};
template <typename T>
struct is_e5 {
  static constexpr bool value = false;
};
template <>
struct is_e5<e5_t> {
  static constexpr bool value = true;
};

// Shared-exponent encoding: clamp to [0, 511/512 * 2^16] (NaN and negatives to 0); exponent from the largest,
// e = max(-16, floor(log2 max)) + 16, bumped by one if the largest rounds to 512 at e; each mantissa is
// floor(v * 2^(24 - e) + 1/2). The scaled values are exact in FP32 (power-of-two scaling) and the rounding is
// taken in FP64, where adding 1/2 is exact. (The same rounding done exactly in FP32, as trunc(x) plus
// x - trunc(x) >= 1/2, made the glass frame's tile kernel slower: 3.25 -> 3.30 ms.)
__host__ __device__ __forceinline__ uint32_t e5_pack(float r, float g, float b) {
  float v[3] = {r, g, b};
  float mx = 0.f;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    v[q] = v[q] > 0.f ? fminf(v[q], 65408.f) : 0.f;
    mx = fmaxf(mx, v[q]);
  }
  int lead = -16;
  if (mx >= 0x1p-16f) {
    uint32_t u;
    __builtin_memcpy(&u, &mx, 4);
    lead = (int)((u >> 23) & 255u) - 127;
  }
  int es = lead + 16;
  if (floor((double)ldexpf(mx, 24 - es) + 0.5) == 512.0) ++es;
  uint32_t w = (uint32_t)es << 27;
#pragma unroll
  for (int q = 0; q < 3; ++q) w |= (uint32_t)floor((double)ldexpf(v[q], 24 - es) + 0.5) << (9 * q);
  return w;
}

__device__ __forceinline__ float e5_unpack(uint32_t w, int q) {
  return ldexpf((float)((w >> (9 * q)) & 511u), (int)(w >> 27) - 24);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Whether this workgroup may read the binned stream: the workspace header carries the stamp of a complete binning
// under the caller's layout and record format, and the tile the workgroup takes and that tile's record range lie
// inside the layout. Otherwise the first thread raises kWsErrMismatch (reported by wt_dropped_count) and the
// workgroup returns before it reads a record or writes an output. Uniform across the workgroup.
__device__ __forceinline__ bool binned_ok(const Binned& b, const Geom& g, uint32_t& tile) {
  // the stamp and the tile index are loaded together (order[] lies inside the layout, which the host checked
  // against the workspace size; its value is used only once the stamp matched and it is a tile of the layout).
  // Plain loads: the header was written by earlier kernels, and this kernel only raises error bits in it.
  const unsigned long long st = b.hdr->binned;
  tile = b.order[blockIdx.x];
  bool ok = st == b.stamp && tile < g.ntiles;
  if (ok) {
    const uint32_t beg = b.offsets[tile * g.NX], end = b.offsets[(tile + 1) * g.NX];
    ok = beg <= end && end <= b.cap;
  }
  if (!ok && threadIdx.x == 0) ws_raise(b.hdr, kWsErrMismatch);
  return ok;
}

// WT_DETERMINISTIC: the first thread applies records [beg, end) one after another in binned order (no two updates
// of an on-chip sum race, so every sum is taken in the same order on every run). Returns true when it did, so the
// caller skips its parallel loop; the caller's barrier follows as usual.
template <typename Fn>
__device__ __forceinline__ bool serial_records(const Geom& g, uint32_t beg, uint32_t end, Fn&& fn) {
  if (!g.serial) return false;
  if (threadIdx.x == 0)
    for (uint32_t i = beg; i < end; ++i) fn(i);
  return true;
}

// Tile of pixel p and its index inside the tile (row-major within the tile).
__device__ __forceinline__ void tile_locate(const Geom& g, uint32_t p, uint32_t& tile, uint32_t& local) {
  const uint32_t y = fastdiv(p, g.divW);
  const uint32_t x = p - y * g.W;
  tile = (y >> g.lTH) * g.tilesX + (x >> g.lTW);
  local = ((y & (g.TH - 1)) << g.lTW) + (x & (g.TW - 1));
}

__device__ __forceinline__ uint32_t tile_of(const Geom& g, uint32_t p) {
  const uint32_t y = fastdiv(p, g.divW);
  const uint32_t x = p - y * g.W;
  return (y >> g.lTH) * g.tilesX + (x >> g.lTW);
}

// Depth of a fragment as the method uses it: clamped to [0, 1]; with per-pixel bounds (lb: lo [TP], then hi [TP],
// as FP32 bit patterns) mapped onto the pixel's own range, x' = (x - lo) / (hi - lo), 0 when hi == lo
// (section 2.1, step 1). The map is taken in FP64, where both differences are exact and the division rounds
// once (correctly), so x' is the correctly rounded FP64 value of the exact quotient: x = lo and x = hi map to
// exactly 0 and 1, and the cell offsets below keep the accuracy of a plain FP32 depth.
__device__ __forceinline__ double unit_depth_d(float x, const uint32_t* lb, uint32_t TP, uint32_t lp) {
  const float xc = fminf(fmaxf(x, 0.f), 1.f);
  if (!lb) return (double)xc;
  const float lo = __uint_as_float(lb[lp]), hi = __uint_as_float(lb[TP + lp]);
  return hi > lo ? ((double)xc - (double)lo) / ((double)hi - (double)lo) : 0.0;
}

// Finest cell j of a fragment and the weights of its two endpoints: u = M x', j = min(floor(u), M - 1),
// t = u - j and omt = 1 - t. Both weights are rounded once from exact or FP64 values (1 - t formed from an
// already rounded t would lose its relative accuracy as t -> 1). For a plain FP32 depth every step is exact.
__device__ __forceinline__ void cell_coord(float x, const uint32_t* lb, uint32_t TP, uint32_t lp, uint32_t M,
                                           uint32_t& j, float& t, float& omt) {
  if (lb) {
    const double u = unit_depth_d(x, lb, TP, lp) * (double)M;
    j = min((uint32_t)u, M - 1);
    t = (float)(u - (double)j);
    omt = (float)((double)(j + 1) - u);
  } else {
    const float u = fminf(fmaxf(x, 0.f), 1.f) * (float)M;
    j = min((uint32_t)u, M - 1);
    t = u - (float)j;
    omt = 1.f - t;
  }
}

// Absorbance step a = -ln(1 - alpha) of a (non-NaN) coverage value, with alpha clamped to [0, 1 - 2^-24].
__device__ __forceinline__ float alpha_clamped(float al) { return al > 0.f ? fminf(al, kAlphaMax) : 0.f; }
__device__ __forceinline__ float absorbance(float al_clamped) { return neg_log1m(al_clamped); }

// What a forward binning stores for each alpha of a fragment: the absorbance step of the clamped alpha, computed
// once where the binning waits on memory rather than in every pass of the tile kernels; NaN stays NaN (the tile
// kernels skip such fragments). alpha_of gives the clamped alpha back, 1 - exp(-a), within a few ulp.
__device__ __forceinline__ float binned_absorbance(float al) { return isnan(al) ? al : absorbance(alpha_clamped(al)); }
__device__ __forceinline__ float alpha_of(float a) { return -expm1f(-a); }

}  // namespace wt
