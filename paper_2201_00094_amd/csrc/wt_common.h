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

// Round to the storage type, to nearest even.
template <typename T>
__device__ __forceinline__ T narrow(float v);
template <>
__device__ __forceinline__ float narrow<float>(float v) { return v; }
template <>
__device__ __forceinline__ __half narrow<__half>(float v) { return __float2half_rn(v); }
template <>
__device__ __forceinline__ bf16_t narrow<bf16_t>(float v) {
  uint32_t u = __float_as_uint(v);
  bf16_t r;
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    r.u = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    r.u = (uint16_t)(u >> 16);
  }
  return r;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Tile of pixel p and its index inside the tile (row-major within the tile).
__device__ __forceinline__ void tile_locate(const Geom& g, uint32_t p, uint32_t& tile, uint32_t& local) {
  const uint32_t y = p / g.W;
  const uint32_t x = p - y * g.W;
  tile = (y / g.TH) * g.tilesX + x / g.TW;
  local = (y & (g.TH - 1)) * g.TW + (x & (g.TW - 1));
}

__device__ __forceinline__ uint32_t tile_of(const Geom& g, uint32_t p) {
  const uint32_t y = p / g.W;
  const uint32_t x = p - y * g.W;
  return (y / g.TH) * g.tilesX + x / g.TW;
}

// Absorbance step a = -ln(1 - alpha) of a (non-NaN) coverage value, with alpha clamped to [0, 1 - 2^-24].
__device__ __forceinline__ float alpha_clamped(float al) { return al > 0.f ? fminf(al, kAlphaMax) : 0.f; }
__device__ __forceinline__ float absorbance(float al_clamped) { return -log1pf(-al_clamped); }

}  // namespace wt
