// Gradient of the resolve with respect to alpha and colour, one workgroup per screen tile.
//
// Forward, per pixel and visibility channel c (colour channels q with c(q) = c):
//   out_q = sum_i alpha_i c_{i,q} v_i + bg_q exp(-sum_i a_i),  v_i = exp(-A~(x_i)),  a_i = -ln(1 - alpha_i),
//   A~(z) = (1 - t) Abar_{j-1} + t Abar_j  (u = M z, j = min(floor(u), M-1), t = u - j).
// With g = dL/dout:
//   dL/dc_{i,q}  = g_q alpha_i v_i
//   dL/dA~(x_i)  = -s_i,  s_i = alpha_i v_i sum_q g_q c_{i,q}
//   cell adjoint  Abar'_m = sum_i -s_i dA~(x_i)/dAbar_m   (two cells per fragment: (1 - t), t)
//   dL/da_i      = sum_m Abar'_m dAbar_m/da_i - exp(-sum a) sum_q g_q bg_q
//   dL/dalpha_i  = v_i sum_q g_q c_{i,q} + dL/da_i / (1 - alpha_i)
// The map a_i -> Abar_m is the build (section 2.3.1) followed by the Haar synthesis; composed, it is the
// average of the fragment's step over cell m, dAbar_m/da_i = clamp((m + 1) - M x_i, 0, 1). Its adjoint is
// therefore a suffix sum of the cell adjoints: with S_m = sum_{m' >= m} Abar'_{m'} and j = floor(M x_i),
//   sum_m Abar'_m dAbar_m/da_i = (j + 1 - M x_i) Abar'_j + S_{j+1},
// which needs O(M) work per pixel and O(1) per fragment for any rank.
#include <algorithm>

#include "wt_common.h"

namespace wt {

constexpr int kBwdThreads = 512;

__device__ __forceinline__ float clamp01_b(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

// Cell value Abar_j of one pixel/channel whose rows are TP floats apart: read directly (cells) or
// synthesised from the coefficients.
__device__ __forceinline__ float cell_value(const float* cf, uint32_t TP, const Geom& g, uint32_t j, bool cells) {
  if (cells) return cf[j * TP];
  float A = cf[0];
  for (uint32_t n = 0; n <= g.rank; ++n) {
    const uint32_t k = j >> (g.L - n);
    const float d = cf[((1u << n) + k) * TP];
    A += ((j >> (g.L - 1 - n)) & 1u) ? -d : d;
  }
  return A;
}

template <int M>
__device__ __forceinline__ void synth_fixed_b(float* cf, uint32_t TP) {
  float v[M];
  v[0] = cf[0];
#pragma unroll
  for (int s = 1; s < M; s <<= 1) {
#pragma unroll
    for (int k = s - 1; k >= 0; --k) {
      const float d = cf[(s + k) * TP];
      const float a = v[k];
      v[2 * k] = a + d;
      v[2 * k + 1] = a - d;
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) cf[j * TP] = v[j];
}

__device__ __forceinline__ void synth_b(float* cf, uint32_t TP, uint32_t M) {
  switch (M) {
    case 2: synth_fixed_b<2>(cf, TP); break;
    case 4: synth_fixed_b<4>(cf, TP); break;
    case 8: synth_fixed_b<8>(cf, TP); break;
    case 16: synth_fixed_b<16>(cf, TP); break;
    default: synth_fixed_b<32>(cf, TP); break;
  }
}

__global__ void k_zero_f32(float* __restrict__ p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

template <int C>
struct BFrag {
  uint32_t lp, src;
  float x, al[C], rgb[3];
};

// Record i of a binning made with stream indices; false for a NaN fragment.
template <int C>
__device__ __forceinline__ bool load_bfrag(const Binned& b, uint32_t i, BFrag<C>& f) {
  const uint32_t* r = b.head + (uint64_t)i * b.DH;
  const uint32_t* rt = b.tail + (uint64_t)i * b.DT;
  f.lp = r[0];
  f.x = __uint_as_float(r[1]);
  bool bad = isnan(f.x);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    f.al[c] = __uint_as_float(r[2 + c]);
    bad |= isnan(f.al[c]);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) f.rgb[q] = __uint_as_float(rt[q]);
  f.src = rt[3];
  return !bad;
}

// LDS rows of TP values: ladj [C*M] FP64 cell adjoints, then their suffix sums; lc [C*M] FP32 cell values;
// lg [3] dL/dout; lT [C] background transmittance.
template <int C, typename TS, bool CELLS>
__global__ __launch_bounds__(kBwdThreads) void k_backward(Binned b, Geom g, const TS* __restrict__ coeffs,
                                                          const float* __restrict__ accum, float bg0, float bg1,
                                                          float bg2, const float* __restrict__ grad_out,
                                                          float* __restrict__ grad_alpha,
                                                          float* __restrict__ grad_rgb) {
  extern __shared__ double smem_b[];
  const uint32_t TP = g.tile_px, per = C * g.M;
  double* ladj = smem_b;
  float* lc = (float*)(ladj + per * TP);
  float* lg = lc + per * TP;
  float* lT = lg + 3 * TP;
  uint32_t* lb = g.tight ? (uint32_t*)(lT + C * TP) : nullptr;  // per-pixel depth bounds
  uint32_t t;
  if (!binned_ok(b, g, t)) return;
  const uint32_t x0 = (t % g.tilesX) * g.TW, y0 = (t / g.tilesX) * g.TH;
  for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
    const uint32_t px = x0 + (lp & (g.TW - 1)), py = y0 + (lp >> g.lTW);
    const bool in = px < g.W && py < g.H;
    const uint64_t p = in ? (uint64_t)py * g.W + px : 0;
    for (uint32_t e = 0; e < per; ++e) {
      if constexpr (is_e5<TS>::value) {
        // packed storage (three channels): word [p][m] holds the magnitudes of coefficient m of every channel
        const uint32_t c = e / g.M, m = e - c * g.M;
        const float v = in ? e5_unpack(((const uint32_t*)coeffs)[p * g.M + m], c) : 0.f;
        lc[e * TP + lp] = m ? -v : v;
      } else {
        lc[e * TP + lp] = in ? widen<TS>(coeffs[p * per + e]) : 0.f;
      }
      ladj[e * TP + lp] = 0.0;
    }
    for (uint32_t q = 0; q < 3; ++q) lg[q * TP + lp] = in ? grad_out[p * 3 + q] : 0.f;
    for (uint32_t c = 0; c < C; ++c)
      lT[c * TP + lp] = in ? __expf(-accum[p * g.AW + (C == 1 ? 3 : 4 + c)]) : 0.f;
  }
  __syncthreads();
  if (CELLS)
    for (uint32_t q = threadIdx.x; q < TP * C; q += blockDim.x) {
      const uint32_t c = q / TP, lp = q - c * TP;
      synth_b(lc + (c * g.M) * TP + lp, TP, g.M);
    }
  __syncthreads();
  const uint32_t beg = b.offsets[t * g.NX], end = b.offsets[(t + 1) * g.NX];
  if (lb) {
    // depth bounds over the tile's valid fragments (section 2.1, step 1): u32 extremes of the FP32 bit patterns
    for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
      lb[lp] = __float_as_uint(1.f);
      lb[TP + lp] = 0u;
    }
    __syncthreads();
    for (uint32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
      BFrag<C> f;
      if (!load_bfrag<C>(b, i, f)) continue;
      const uint32_t xb = __float_as_uint(clamp01_b(f.x));
      atomicMin(lb + f.lp, xb);
      atomicMax(lb + TP + f.lp, xb);
    }
    __syncthreads();
  }
  // pass 1: cell adjoints (one thread in binned order under WT_DETERMINISTIC)
  const uint32_t i1 = g.serial ? (threadIdx.x ? end : beg) : beg + threadIdx.x, di1 = g.serial ? 1 : blockDim.x;
  for (uint32_t i = i1; i < end; i += di1) {
    BFrag<C> f;
    if (!load_bfrag<C>(b, i, f)) continue;
    uint32_t j;
    float tt, omt;
    cell_coord(f.x, lb, TP, f.lp, g.M, j, tt, omt);
    const float gq[3] = {lg[f.lp], lg[TP + f.lp], lg[2 * TP + f.lp]};
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float* cf = lc + (c * g.M) * TP + f.lp;
      const float hi = cell_value(cf, TP, g, j, CELLS);
      const float lo = j ? cell_value(cf, TP, g, j - 1, CELLS) : 0.f;
      const float v = __expf(-fmaf(tt, hi, omt * lo));
      const float alc = alpha_clamped(f.al[c]);
      const float gc = (C == 1) ? (gq[0] * f.rgb[0] + gq[1] * f.rgb[1] + gq[2] * f.rgb[2]) : gq[c] * f.rgb[c];
      const float s = alc * v * gc;
      double* adj = ladj + (c * g.M) * TP + f.lp;
      if (j) atomicAdd(adj + (j - 1) * TP, (double)(-s * omt));
      atomicAdd(adj + j * TP, (double)(-s * tt));
    }
  }
  __syncthreads();
  // suffix sums of the cell adjoints
  for (uint32_t q = threadIdx.x; q < TP * C; q += blockDim.x) {
    const uint32_t c = q / TP, lp = q - c * TP;
    double* adj = ladj + (c * g.M) * TP + lp;
    double run = 0.0;
    for (int m = (int)g.M - 1; m >= 0; --m) {
      run += adj[m * TP];
      adj[m * TP] = run;
    }
  }
  __syncthreads();
  // pass 2: per-fragment gradients, written at the fragment's stream position
  const float bg[3] = {bg0, bg1, bg2};
  for (uint32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    BFrag<C> f;
    if (!load_bfrag<C>(b, i, f)) continue;
    const uint64_t src = f.src;
    uint32_t j;
    float tt, omt;
    cell_coord(f.x, lb, TP, f.lp, g.M, j, tt, omt);
    const float gq[3] = {lg[f.lp], lg[TP + f.lp], lg[2 * TP + f.lp]};
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float* cf = lc + (c * g.M) * TP + f.lp;
      const float hi = cell_value(cf, TP, g, j, CELLS);
      const float lo = j ? cell_value(cf, TP, g, j - 1, CELLS) : 0.f;
      const float v = __expf(-fmaf(tt, hi, omt * lo));
      const float alc = alpha_clamped(f.al[c]);
      const double* S = ladj + (c * g.M) * TP + f.lp;
      const double Sj = S[j * TP];
      const double Sj1 = (j + 1 < g.M) ? S[(j + 1) * TP] : 0.0;
      const float through_cells = (float)((double)omt * (Sj - Sj1) + Sj1);
      const float gbg = (C == 1) ? (gq[0] * bg[0] + gq[1] * bg[1] + gq[2] * bg[2]) : gq[c] * bg[c];
      const float dLda = through_cells - gbg * lT[c * TP + f.lp];
      const float gc = (C == 1) ? (gq[0] * f.rgb[0] + gq[1] * f.rgb[1] + gq[2] * f.rgb[2]) : gq[c] * f.rgb[c];
      const bool inside = f.al[c] > 0.f && f.al[c] < kAlphaMax;
      grad_alpha[src * C + c] = inside ? v * gc + dLda / (1.f - alc) : 0.f;
      if (C == 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) grad_rgb[src * 3 + q] = gq[q] * alc * v;
      } else {
        grad_rgb[src * 3 + c] = gq[c] * alc * v;
      }
    }
  }
}

size_t lds_backward_bytes(const Geom& g) {
  return (size_t)g.tile_px * (12 * g.C * g.M + 4 * (3 + g.C) + (g.tight ? 8 : 0));
}

hipError_t launch_backward(const Geom& g, const Binned& b, const void* coeffs, const float* accum, const float* bg,
                           const float* grad_out, float* grad_alpha, float* grad_rgb, uint64_t count,
                           hipStream_t s) {
  if (count) {
    const unsigned za = (unsigned)std::min<uint64_t>((count * g.C + 255) / 256, 8192);
    const unsigned zr = (unsigned)std::min<uint64_t>((count * 3 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero_f32, dim3(za), dim3(256), 0, s, grad_alpha, count * g.C);
    hipLaunchKernelGGL(k_zero_f32, dim3(zr), dim3(256), 0, s, grad_rgb, count * 3);
  }
  const size_t lds = lds_backward_bytes(g);
  if (lds > kLdsBytes) return hipErrorNotSupported;
  hipError_t err = hipSuccess;
#define WT_BWD_LAUNCH(CC, TT, CELLS)                                                                              \
  do {                                                                                                           \
    auto k = k_backward<CC, TT, CELLS>;                                                                          \
    if (lds > 65536) err = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (err == hipSuccess)                                                                                       \
      hipLaunchKernelGGL(k, dim3(g.ntiles), dim3(kBwdThreads), lds, s, b, g, (const TT*)coeffs, accum, bg[0],     \
                         bg[1], bg[2], grad_out, grad_alpha, grad_rgb);                                          \
  } while (0)
#define WT_BWD_CELLS(CC, TT)               \
  do {                                     \
    if (g.M <= 32)                         \
      WT_BWD_LAUNCH(CC, TT, true);         \
    else                                   \
      WT_BWD_LAUNCH(CC, TT, false);        \
  } while (0)
#define WT_BWD_TYPE(CC)                                   \
  do {                                                    \
    if (g.dtype == WT_F32) WT_BWD_CELLS(CC, float);       \
    else if (g.dtype == WT_F16) WT_BWD_CELLS(CC, __half); \
    else if (g.dtype == WT_BF16) WT_BWD_CELLS(CC, bf16_t); \
    else if (CC == 3) WT_BWD_CELLS(CC, e5_t);             \
    else err = hipErrorInvalidValue;                      \
  } while (0)
  if (g.C == 1)
    WT_BWD_TYPE(1);
  else
    WT_BWD_TYPE(3);
#undef WT_BWD_TYPE
#undef WT_BWD_CELLS
#undef WT_BWD_LAUNCH
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

}  // namespace wt
