// Per-tile build, evaluate and resolve kernels over a binned fragment stream.
//
// One workgroup owns one screen tile. Its coefficient tile [tile_px][C][M] lives in LDS as FP32; every
// fragment of the tile is applied with LDS float atomics, so no per-fragment update ever leaves the compute
// unit. Global memory sees one coalesced load and/or store of each coefficient tile and of each
// accumulation tile, plus the streaming read of the binned fragments.
//
//   build     (section 2.3.1): chi += a (1 - x); for n = 0..N: d[2^n + k] -= a tau(2^n x - k),
//             k = min(floor(2^n x), 2^n - 1), tau(t) = t on [0, 1/2), 1 - t on [1/2, 1]; a = -ln(1 - alpha).
//             d = 2^(n/2) X_{n,k}, so the N + 2 updates of a fragment are plain products.
//   cells     (section 2.3): the Haar expansion is constant on the M cells of width 1/M; the inverse of the
//             level-scaled transform gives the cell values with one add and one subtract per coefficient.
//   evaluate  (sections 2.2, 2.3.2): u = M x, j = min(floor(u), M - 1), t = u - j,
//             A~ = (1 - t) Abar_{j-1} + t Abar_j (Abar_{-1} = 0), v = exp(-A~);
//             accumulate alpha rgb v and a per pixel.
//   resolve   (section 2.1 step 4): out = colour + bg exp(-sum a).
#include <algorithm>
#include <type_traits>

#include "wt_common.h"

namespace wt {

constexpr int kTileThreads = 512;

__device__ __forceinline__ void tile_origin(const Geom& g, uint32_t t, uint32_t& x0, uint32_t& y0) {
  x0 = (t % g.tilesX) * g.TW;
  y0 = (t / g.tilesX) * g.TH;
}

// Global element index of tile-local element e (per elements per pixel); false when the pixel is off-frame.
__device__ __forceinline__ bool tile_elem(const Geom& g, uint32_t x0, uint32_t y0, uint32_t e, uint32_t per,
                                          uint64_t& gi) {
  const uint32_t lp = e / per;
  const uint32_t rem = e - lp * per;
  const uint32_t px = x0 + (lp & (g.TW - 1));
  const uint32_t py = y0 + lp / g.TW;
  if (px >= g.W || py >= g.H) return false;
  gi = ((uint64_t)py * g.W + px) * per + rem;
  return true;
}

__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

template <int C>
__device__ __forceinline__ bool load_fragment(const Binned& b, uint32_t i, uint32_t& lp, float& x, float (&al)[C]) {
  lp = b.lpx[i];
  x = b.x[i];
  bool bad = isnan(x);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    al[c] = b.alpha[c * b.cap + i];
    bad |= isnan(al[c]);
  }
  return !bad;
}

// Build: the N + 2 coefficient updates of one fragment, per channel, into the LDS tile.
template <int C>
__device__ __forceinline__ void build_add(float* lc, const Geom& g, uint32_t lp, float x, const float (&al)[C]) {
  x = clamp01(x);
  float a[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    a[c] = absorbance(alpha_clamped(al[c]));
    atomicAdd(lc + (lp * C + c) * g.M, a[c] * (1.f - x));
  }
  for (uint32_t n = 0; n <= g.rank; ++n) {
    const uint32_t s = 1u << n;
    const float u = x * (float)s;
    const uint32_t k = min((uint32_t)u, s - 1);
    const float t = u - (float)k;
    const float tau = t < 0.5f ? t : 1.f - t;
#pragma unroll
    for (int c = 0; c < C; ++c) atomicAdd(lc + (lp * C + c) * g.M + s + k, -a[c] * tau);
  }
}

// Cell value Abar_j straight from the stored coefficients (used when M is too large to expand per pixel).
__device__ __forceinline__ float cell_from_coeffs(const float* cf, const Geom& g, uint32_t j) {
  float A = cf[0];
  for (uint32_t n = 0; n <= g.rank; ++n) {
    const uint32_t k = j >> (g.L - n);
    const float d = cf[(1u << n) + k];
    A += ((j >> (g.L - 1 - n)) & 1u) ? -d : d;
  }
  return A;
}

// In-place inverse of the level-scaled Haar transform for one pixel/channel: coefficients -> cell values.
template <int M>
__device__ __forceinline__ void synth_fixed(float* cf) {
  float v[M];
  v[0] = cf[0];
#pragma unroll
  for (int s = 1; s < M; s <<= 1) {
#pragma unroll
    for (int k = s - 1; k >= 0; --k) {
      const float d = cf[s + k];
      const float a = v[k];
      v[2 * k] = a + d;
      v[2 * k + 1] = a - d;
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) cf[j] = v[j];
}

__device__ __forceinline__ void synth(float* cf, uint32_t M) {
  switch (M) {
    case 2: synth_fixed<2>(cf); break;
    case 4: synth_fixed<4>(cf); break;
    case 8: synth_fixed<8>(cf); break;
    case 16: synth_fixed<16>(cf); break;
    default: synth_fixed<32>(cf); break;
  }
}

// Evaluate: visibility at the fragment's depth and its contribution to the accumulation tile.
template <int C, bool CELLS>
__device__ __forceinline__ void eval_add(const float* lc, float* la, const Geom& g, uint32_t lp, float x,
                                         const float (&al)[C], const float (&rgb)[3]) {
  x = clamp01(x);
  const float u = x * (float)g.M;
  const uint32_t j = min((uint32_t)u, g.M - 1);
  const float t = u - (float)j;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float* cf = lc + (lp * C + c) * g.M;
    float lo, hi;
    if (CELLS) {
      hi = cf[j];
      lo = j ? cf[j - 1] : 0.f;
    } else {
      hi = cell_from_coeffs(cf, g, j);
      lo = j ? cell_from_coeffs(cf, g, j - 1) : 0.f;
    }
    const float At = fmaf(t, hi, (1.f - t) * lo);
    const float v = __expf(-At);
    const float alc = alpha_clamped(al[c]);
    const float a = absorbance(alc);
    if (C == 1) {
      const float w = alc * v;
      atomicAdd(la + lp * 4 + 0, w * rgb[0]);
      atomicAdd(la + lp * 4 + 1, w * rgb[1]);
      atomicAdd(la + lp * 4 + 2, w * rgb[2]);
      atomicAdd(la + lp * 4 + 3, a);
    } else {
      atomicAdd(la + lp * 8 + c, alc * rgb[c] * v);
      atomicAdd(la + lp * 8 + 4 + c, a);
    }
  }
}

template <int C, bool CELLS>
__device__ __forceinline__ void eval_tile_fragments(const Binned& b, const Geom& g, uint32_t t, const float* lc,
                                                    float* la) {
  const uint32_t beg = b.offsets[t * g.NX], end = b.offsets[(t + 1) * g.NX];
  for (uint32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    uint32_t lp;
    float x, al[C], rgb[3];
    if (!load_fragment<C>(b, i, lp, x, al)) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q) rgb[q] = b.rgb[q * b.cap + i];
    eval_add<C, CELLS>(lc, la, g, lp, x, al, rgb);
  }
}

template <int C>
__device__ __forceinline__ void build_tile_fragments(const Binned& b, const Geom& g, uint32_t t, float* lc) {
  const uint32_t beg = b.offsets[t * g.NX], end = b.offsets[(t + 1) * g.NX];
  for (uint32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    uint32_t lp;
    float x, al[C];
    if (!load_fragment<C>(b, i, lp, x, al)) continue;
    build_add<C>(lc, g, lp, x, al);
  }
}

template <bool CELLS>
__device__ __forceinline__ void synth_tile(float* lc, const Geom& g) {
  if (CELLS)
    for (uint32_t q = threadIdx.x; q < g.tile_px * g.C; q += blockDim.x) synth(lc + q * g.M, g.M);
}

// ------------------------------------------------------------------------------------------- kernels

template <int C, typename TS>
__global__ __launch_bounds__(kTileThreads) void k_build(Binned b, Geom g, TS* __restrict__ coeffs) {
  extern __shared__ float smem[];
  float* lc = smem;
  const uint32_t t = blockIdx.x;
  uint32_t x0, y0;
  tile_origin(g, t, x0, y0);
  const uint32_t per = C * g.M, nel = g.tile_px * per;
  for (uint32_t e = threadIdx.x; e < nel; e += blockDim.x) {
    uint64_t gi;
    lc[e] = tile_elem(g, x0, y0, e, per, gi) ? widen<TS>(coeffs[gi]) : 0.f;
  }
  __syncthreads();
  build_tile_fragments<C>(b, g, t, lc);
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < nel; e += blockDim.x) {
    uint64_t gi;
    if (tile_elem(g, x0, y0, e, per, gi)) coeffs[gi] = narrow<TS>(lc[e]);
  }
}

template <int C, typename TS, bool CELLS>
__global__ __launch_bounds__(kTileThreads) void k_evaluate(Binned b, Geom g, const TS* __restrict__ coeffs,
                                                           float* __restrict__ accum) {
  extern __shared__ float smem[];
  const uint32_t per = C * g.M, nel = g.tile_px * per;
  float* lc = smem;
  float* la = smem + nel;
  const uint32_t t = blockIdx.x;
  uint32_t x0, y0;
  tile_origin(g, t, x0, y0);
  for (uint32_t e = threadIdx.x; e < nel; e += blockDim.x) {
    uint64_t gi;
    lc[e] = tile_elem(g, x0, y0, e, per, gi) ? widen<TS>(coeffs[gi]) : 0.f;
  }
  const uint32_t nacc = g.tile_px * g.AW;
  for (uint32_t e = threadIdx.x; e < nacc; e += blockDim.x) {
    uint64_t gi;
    la[e] = tile_elem(g, x0, y0, e, g.AW, gi) ? accum[gi] : 0.f;
  }
  __syncthreads();
  synth_tile<CELLS>(lc, g);
  __syncthreads();
  eval_tile_fragments<C, CELLS>(b, g, t, lc, la);
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < nacc; e += blockDim.x) {
    uint64_t gi;
    if (tile_elem(g, x0, y0, e, g.AW, gi)) accum[gi] = la[e];
  }
}

template <int C, typename TS, bool CELLS>
__global__ __launch_bounds__(kTileThreads) void k_render(Binned b, Geom g, TS* __restrict__ coeffs, float bg0,
                                                         float bg1, float bg2, float* __restrict__ out) {
  extern __shared__ float smem[];
  const uint32_t per = C * g.M, nel = g.tile_px * per;
  const uint32_t nacc = g.tile_px * g.AW;
  float* lc = smem;
  float* la = smem + nel;
  const uint32_t t = blockIdx.x;
  uint32_t x0, y0;
  tile_origin(g, t, x0, y0);
  for (uint32_t e = threadIdx.x; e < nel + nacc; e += blockDim.x) smem[e] = 0.f;
  __syncthreads();
  build_tile_fragments<C>(b, g, t, lc);
  __syncthreads();
  // Coefficients at storage precision: stored (optionally) and used for the evaluation.
  for (uint32_t e = threadIdx.x; e < nel; e += blockDim.x) {
    const TS s = narrow<TS>(lc[e]);
    lc[e] = widen<TS>(s);
    uint64_t gi;
    if (coeffs && tile_elem(g, x0, y0, e, per, gi)) coeffs[gi] = s;
  }
  __syncthreads();
  synth_tile<CELLS>(lc, g);
  __syncthreads();
  eval_tile_fragments<C, CELLS>(b, g, t, lc, la);
  __syncthreads();
  const float bg[3] = {bg0, bg1, bg2};
  for (uint32_t e = threadIdx.x; e < g.tile_px * 3; e += blockDim.x) {
    const uint32_t lp = e / 3, q = e - lp * 3;
    uint64_t gi;
    if (!tile_elem(g, x0, y0, e, 3, gi)) continue;
    const float colour = la[lp * g.AW + q];
    const float suma = (C == 1) ? la[lp * 4 + 3] : la[lp * 8 + 4 + q];
    out[gi] = colour + bg[q] * __expf(-suma);
  }
}

__global__ __launch_bounds__(256) void k_resolve(const float* __restrict__ accum, Geom g, float bg0, float bg1,
                                                 float bg2, float* __restrict__ out) {
  const float bg[3] = {bg0, bg1, bg2};
  const uint64_t n = (uint64_t)g.P * 3;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t p = e / 3;
    const uint32_t q = (uint32_t)(e - p * 3);
    const float colour = accum[p * g.AW + q];
    const float suma = (g.AW == 4) ? accum[p * 4 + 3] : accum[p * 8 + 4 + q];
    out[e] = colour + bg[q] * __expf(-suma);
  }
}

// ------------------------------------------------------------------------------------------- launchers

size_t lds_tile_bytes(const Geom& g, bool with_accum) {
  return (size_t)g.tile_px * (g.C * g.M + (with_accum ? g.AW : 0)) * sizeof(float);
}

template <typename K>
static hipError_t prep(K kernel, size_t lds) {
  if (lds > 65536) return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

// Dispatch on channels and storage type: f(std::integral_constant<int, C>, TS* tag) for the frame's values.
template <typename F>
static hipError_t dispatch(const Geom& g, F&& f) {
  if (g.C == 1) {
    if (g.dtype == WT_F32) return f(std::integral_constant<int, 1>{}, (float*)nullptr);
    if (g.dtype == WT_F16) return f(std::integral_constant<int, 1>{}, (__half*)nullptr);
    return f(std::integral_constant<int, 1>{}, (bf16_t*)nullptr);
  }
  if (g.dtype == WT_F32) return f(std::integral_constant<int, 3>{}, (float*)nullptr);
  if (g.dtype == WT_F16) return f(std::integral_constant<int, 3>{}, (__half*)nullptr);
  return f(std::integral_constant<int, 3>{}, (bf16_t*)nullptr);
}

hipError_t launch_build(const Geom& g, const Binned& b, void* coeffs, hipStream_t s) {
  const size_t lds = lds_tile_bytes(g, false);
  return dispatch(g, [&](auto cc, auto* tag) {
    constexpr int C = decltype(cc)::value;
    using TS = std::remove_pointer_t<decltype(tag)>;
    auto k = k_build<C, TS>;
    hipError_t err = prep(k, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(g.ntiles), dim3(kTileThreads), lds, s, b, g, (TS*)coeffs);
    return hipGetLastError();
  });
}

hipError_t launch_evaluate(const Geom& g, const Binned& b, const void* coeffs, float* accum, hipStream_t s) {
  const size_t lds = lds_tile_bytes(g, true);
  return dispatch(g, [&](auto cc, auto* tag) {
    constexpr int C = decltype(cc)::value;
    using TS = std::remove_pointer_t<decltype(tag)>;
    auto k = (g.M <= 32) ? k_evaluate<C, TS, true> : k_evaluate<C, TS, false>;
    hipError_t err = prep(k, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(g.ntiles), dim3(kTileThreads), lds, s, b, g, (const TS*)coeffs, accum);
    return hipGetLastError();
  });
}

hipError_t launch_render(const Geom& g, const Binned& b, const float* bg, void* coeffs, float* out, hipStream_t s) {
  const size_t lds = lds_tile_bytes(g, true);
  return dispatch(g, [&](auto cc, auto* tag) {
    constexpr int C = decltype(cc)::value;
    using TS = std::remove_pointer_t<decltype(tag)>;
    auto k = (g.M <= 32) ? k_render<C, TS, true> : k_render<C, TS, false>;
    hipError_t err = prep(k, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(g.ntiles), dim3(kTileThreads), lds, s, b, g, (TS*)coeffs, bg[0], bg[1], bg[2], out);
    return hipGetLastError();
  });
}

hipError_t launch_resolve(const Geom& g, const float* accum, const float* bg, float* out, hipStream_t s) {
  const uint64_t n = (uint64_t)g.P * 3;
  const unsigned grid = (unsigned)std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_resolve, dim3(grid), dim3(256), 0, s, accum, g, bg[0], bg[1], bg[2], out);
  return hipGetLastError();
}

}  // namespace wt
