// Per-tile build, evaluate and resolve kernels over a binned fragment stream.
//
// One workgroup owns one screen tile. Its coefficient tile lives in LDS, coefficient-major
// ([channel * M + m][pixel]: the updates of a wavefront go to random pixels, hence random banks), and every
// fragment of the tile is applied with LDS atomics, so no per-fragment update leaves the compute unit.
// Global memory sees the streaming read of the binned records plus one coalesced load and/or store of each
// coefficient and accumulation tile.
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


// ------------------------------------------------------------------------------------------- tile addressing

struct TileRef {
  uint32_t x0, y0;   // origin in the frame
  uint32_t beg, end; // binned record range
};

__device__ __forceinline__ TileRef tile_ref(const Geom& g, const Binned& b, uint32_t t) {
  TileRef r;
  r.x0 = (t % g.tilesX) * g.TW;
  r.y0 = (t / g.tilesX) * g.TH;
  r.beg = b.offsets[t * g.NX];
  r.end = b.offsets[(t + 1) * g.NX];
  return r;
}

// Frame pixel of tile-local pixel lp, or false when it lies outside the frame.
__device__ __forceinline__ bool tile_pixel(const Geom& g, const TileRef& r, uint32_t lp, uint64_t& p) {
  p = 0;
  const uint32_t px = r.x0 + (lp & (g.TW - 1));
  const uint32_t py = r.y0 + (lp >> g.lTW);
  if (px >= g.W || py >= g.H) return false;
  p = (uint64_t)py * g.W + px;
  return true;
}

__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

// ------------------------------------------------------------------------------------------- records

template <int C>
struct Frag {
  uint32_t lp;
  float x;
  float al[C];  // absorbance a = -ln(1 - alpha) per channel (forward binning; NaN for a dropped fragment)
  float rgb[3];
};

template <bool NT>
__device__ __forceinline__ uint32_t load_word(const uint32_t* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Pixel, depth and alpha of record i; false for a NaN fragment (skipped, already counted as dropped).
template <int C, bool NT = false>
__device__ __forceinline__ bool load_head(const Binned& b, uint32_t i, Frag<C>& f) {
  const uint32_t* r = b.head + (uint64_t)i * b.DH;
  f.lp = load_word<NT>(r);
  f.x = __uint_as_float(load_word<NT>(r + 1));
  bool bad = isnan(f.x);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    f.al[c] = __uint_as_float(load_word<NT>(r + 2 + c));
    bad |= isnan(f.al[c]);
  }
  return !bad;
}

// The whole record, for the evaluate pass: its last read. At one channel the loads are non-temporal, so that the
// record lines of the tiles still being built stay in the caches for their second read (smoke frame: tile kernel
// 0.96 -> 0.89 ms; non-temporal loads in the build as well: 1.02 ms). At three channels a tile's records are few
// and the same loads made the glass frame's tile kernel slower (3.02 -> 3.11 ms), so there they stay ordinary.
template <int C>
__device__ __forceinline__ bool load_full(const Binned& b, uint32_t i, Frag<C>& f) {
  constexpr bool kNT = C == 1;
  const uint32_t* r = b.tail + (uint64_t)i * b.DT;
#pragma unroll
  for (int q = 0; q < 3; ++q) f.rgb[q] = __uint_as_float(load_word<kNT>(r + q));
  return load_head<C, kNT>(b, i, f);
}

// ------------------------------------------------------------------------------------------- depth bounds

// Per-pixel depth bounds of the tile (section 2.1, step 1): lb[lp] = lo, lb[TP + lp] = hi as FP32 bit patterns,
// over the clamped depths of the tile's valid fragments (non-negative floats order like their bit patterns, so
// LDS u32 min/max atomics take them). Ends with a barrier.
template <int C>
__device__ __forceinline__ void bounds_tile(const Binned& b, const Geom& g, const TileRef& r, uint32_t* lb) {
  const uint32_t TP = g.tile_px;
  for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
    lb[lp] = __float_as_uint(1.f);
    lb[TP + lp] = 0u;
  }
  __syncthreads();
  for (uint32_t i = r.beg + threadIdx.x; i < r.end; i += blockDim.x) {
    Frag<C> f;
    if (!load_head<C>(b, i, f)) continue;
    const uint32_t xb = __float_as_uint(fminf(fmaxf(f.x, 0.f), 1.f));
    atomicMin(lb + f.lp, xb);
    atomicMax(lb + TP + f.lp, xb);
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------------- build

// On-chip sums are FP64: on gfx950 an LDS FP64 atomic add sustains about nine times the rate of an FP32 one,
// and every FP32 term then rounds once while the sum rounds nowhere.
using acc_t = double;

// Binned records each thread keeps in flight in the build and evaluate loops (memory-level parallelism of one
// workgroup per compute unit).
constexpr int kBuildUnroll = 8;
constexpr int kEvalUnroll = 4;
// The evaluate loop of the two-pass tile kernel: six whole records per thread at three channels, where a tile holds
// a few thousand records (glass 3840x2160: 3.03 -> 2.96 ms; at one channel six were slower, 0.89 -> 0.93 ms).
template <int C>
constexpr int eval_unroll() { return C == 1 ? kEvalUnroll : 6; }

// The N + 2 coefficient updates of one fragment, per channel. lc is [C*M][TP] of acc_t.
template <int C>
__device__ __forceinline__ void build_add(acc_t* lc, const Geom& g, const Frag<C>& f, const uint32_t* lb) {
  const uint32_t TP = g.tile_px;
  const double xd = unit_depth_d(f.x, lb, TP, f.lp);
  float a[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    a[c] = f.al[c];  // binned records hold the absorbance
    atomicAdd(lc + (c * g.M) * TP + f.lp, (acc_t)(a[c] * (float)(1.0 - xd)));
  }
  for (uint32_t n = 0; n <= g.rank; ++n) {
    const uint32_t s = 1u << n;
    const double u = xd * (double)s;
    const uint32_t k = min((uint32_t)u, s - 1);
    const double t = u - (double)k;
    const float tau = (float)(t < 0.5 ? t : 1.0 - t);
#pragma unroll
    for (int c = 0; c < C; ++c) atomicAdd(lc + (c * g.M + s + k) * TP + f.lp, (acc_t)(-a[c] * tau));
  }
}

template <int C>
__device__ __forceinline__ void build_tile(const Binned& b, const Geom& g, const TileRef& r, acc_t* lc,
                                           const uint32_t* lb) {
  if (serial_records(g, r.beg, r.end, [&](uint32_t i) {
        Frag<C> f;
        if (load_head<C>(b, i, f)) build_add<C>(lc, g, f, lb);
      }))
    return;
  uint32_t i = r.beg + threadIdx.x;
  // two records per thread per step keep more loads in flight
  for (; i + blockDim.x < r.end; i += 2 * blockDim.x) {
    Frag<C> f0, f1;
    const bool ok0 = load_head<C>(b, i, f0);
    const bool ok1 = load_head<C>(b, i + blockDim.x, f1);
    if (ok0) build_add<C>(lc, g, f0, lb);
    if (ok1) build_add<C>(lc, g, f1, lb);
  }
  if (i < r.end) {
    Frag<C> f0;
    if (load_head<C>(b, i, f0)) build_add<C>(lc, g, f0, lb);
  }
}

// ------------------------------------------------------------------------------------------- cells

// Cell value Abar_j straight from the stored coefficients of one pixel/channel (column stride TP).
template <typename T>
__device__ __forceinline__ float cell_from_coeffs(const T* cf, uint32_t TP, const Geom& g, uint32_t j) {
  T A = cf[0];
  for (uint32_t n = 0; n <= g.rank; ++n) {
    const uint32_t k = j >> (g.L - n);
    const T d = cf[((1u << n) + k) * TP];
    A += ((j >> (g.L - 1 - n)) & 1u) ? -d : d;
  }
  return (float)A;
}

// Inverse of the level-scaled Haar transform on M values held in registers: coefficients -> cell values.
template <int M>
__device__ __forceinline__ void synth_regs(float (&v)[M]) {
  float w[M];
  w[0] = v[0];
#pragma unroll
  for (int s = 1; s < M; s <<= 1) {
#pragma unroll
    for (int k = s - 1; k >= 0; --k) {
      const float d = v[s + k];
      const float a = w[k];
      w[2 * k] = a + d;
      w[2 * k + 1] = a - d;
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = w[j];
}

// Cells of an FP32 coefficient tile, in place (one pixel/channel per thread).
template <int C, int M>
__device__ __forceinline__ void synth_tile_f32(float* lc, uint32_t TP) {
  for (uint32_t q = threadIdx.x; q < TP * C; q += blockDim.x) {
    const uint32_t c = q / TP, lp = q - c * TP;
    float* cf = lc + (c * M) * TP + lp;
    float v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = cf[m * TP];
    synth_regs<M>(v);
#pragma unroll
    for (int m = 0; m < M; ++m) cf[m * TP] = v[m];
  }
}

template <int C>
__device__ __forceinline__ void synth_tile_f32(float* lc, const Geom& g) {
  switch (g.M) {
    case 2: synth_tile_f32<C, 2>(lc, g.tile_px); break;
    case 4: synth_tile_f32<C, 4>(lc, g.tile_px); break;
    case 8: synth_tile_f32<C, 8>(lc, g.tile_px); break;
    case 16: synth_tile_f32<C, 16>(lc, g.tile_px); break;
    default: synth_tile_f32<C, 32>(lc, g.tile_px); break;
  }
}

// Writes M values of TS for one pixel/channel, 16 bytes at a time where the layout allows.
template <typename TS, int M>
__device__ __forceinline__ void store_row(TS* dst, const TS (&s)[M]) {
  if ((M * sizeof(TS)) % 16 == 0) {
#pragma unroll
    for (int k = 0; k < (int)(M * sizeof(TS) / 16); ++k) {
      uint4 u;
      __builtin_memcpy(&u, (const char*)s + 16 * k, 16);
      ((uint4*)dst)[k] = u;
    }
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) dst[m] = s[m];
  }
}

// FP64 coefficient tile -> storage precision (stored when coeffs is not null) -> FP32 cells in the first half
// of the same LDS region. Requires TP * C <= blockDim.x: each thread holds at most one pixel/channel.
template <int C, typename TS, int M>
__device__ __forceinline__ void coeffs_to_cells(const Geom& g, const TileRef& r, acc_t* lc64, TS* coeffs) {
  if constexpr (!is_e5<TS>::value) {  // packed storage runs the endpoint path only (make_geom)
  const uint32_t TP = g.tile_px;
  const uint32_t q = threadIdx.x;
  const bool have = q < TP * C;
  const uint32_t c = have ? q / TP : 0, lp = have ? q - c * TP : 0;
  float v[M];
  if (have) {
    TS s[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      s[m] = narrow_d<TS>(lc64[(c * M + m) * TP + lp]);
      v[m] = widen<TS>(s[m]);
    }
    uint64_t p;
    if (coeffs && tile_pixel(g, r, lp, p)) store_row<TS, M>(coeffs + (p * C + c) * M, s);
    synth_regs<M>(v);
  }
  __syncthreads();  // every FP64 value has been read before the FP32 cells overwrite the region
  if (have) {
    float* lc32 = (float*)lc64;
#pragma unroll
    for (int m = 0; m < M; ++m) lc32[(c * M + m) * TP + lp] = v[m];
  }
  }
}

template <int C, typename TS>
__device__ __forceinline__ void coeffs_to_cells(const Geom& g, const TileRef& r, acc_t* lc64, TS* coeffs) {
  switch (g.M) {
    case 2: coeffs_to_cells<C, TS, 2>(g, r, lc64, coeffs); break;
    case 4: coeffs_to_cells<C, TS, 4>(g, r, lc64, coeffs); break;
    case 8: coeffs_to_cells<C, TS, 8>(g, r, lc64, coeffs); break;
    case 16: coeffs_to_cells<C, TS, 16>(g, r, lc64, coeffs); break;
    default: coeffs_to_cells<C, TS, 32>(g, r, lc64, coeffs); break;
  }
}

// ------------------------------------------------------------------------------------------- endpoint masses
//
// A fragment's contribution to every coefficient depends on its depth only through its finest cell j and the
// offset t = M x - j in it: 1 - x and every tent tau(2^n x - k) are linear on a finest cell (their kinks lie on
// cell boundaries for n <= N). So the N + 2 closed-form updates of section 2.3.1 factor exactly through two
// endpoint masses, e_j += a (1 - t) and e_{j+1} += a t, per fragment and channel:
//   chi     = sum_m e_m (1 - m/M),   d_{n,k} = -sum_m e_m tau(2^n m / M - k),   sum a = sum_m e_m,
// with exact dyadic weights and all terms of one sign (no cancellation). Two LDS atomics per fragment instead
// of N + 2, and the absorbance total comes for free.

template <int C>
__device__ __forceinline__ void build_ep_add(acc_t* le, const Geom& g, const Frag<C>& f, const uint32_t* lb) {
  const uint32_t TP = g.tile_px, M1 = g.M + 1;
  uint32_t j;
  float t, omt;
  cell_coord(f.x, lb, TP, f.lp, g.M, j, t, omt);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float a = f.al[c];  // binned records hold the absorbance
    acc_t* e = le + (c * M1 + j) * TP + f.lp;
    atomicAdd(e, (acc_t)(a * omt));
    atomicAdd(e + TP, (acc_t)(a * t));
  }
}

template <int C>
__device__ __forceinline__ void build_ep_tile(const Binned& b, const Geom& g, const TileRef& r, acc_t* le,
                                              const uint32_t* lb) {
  if (serial_records(g, r.beg, r.end, [&](uint32_t i) {
        Frag<C> f;
        if (load_head<C>(b, i, f)) build_ep_add<C>(le, g, f, lb);
      }))
    return;
  uint32_t i = r.beg + threadIdx.x;
  // kBuildUnroll 12-byte head records per thread in flight per step
  for (; i + (kBuildUnroll - 1) * blockDim.x < r.end; i += kBuildUnroll * blockDim.x) {
    Frag<C> f[kBuildUnroll];
    bool ok[kBuildUnroll];
#pragma unroll
    for (int u = 0; u < kBuildUnroll; ++u) ok[u] = load_head<C>(b, i + u * blockDim.x, f[u]);
#pragma unroll
    for (int u = 0; u < kBuildUnroll; ++u)
      if (ok[u]) build_ep_add<C>(le, g, f[u], lb);
  }
  for (; i < r.end; i += blockDim.x) {
    Frag<C> f0;
    if (load_head<C>(b, i, f0)) build_ep_add<C>(le, g, f0, lb);
  }
}

// Coefficients (stored layout) and absorbance total of one pixel/channel from its M + 1 endpoint masses.
template <int M>
__device__ __forceinline__ void endpoints_to_coeffs(const acc_t (&e)[M + 1], acc_t (&cf)[M], acc_t& suma) {
  acc_t chi = 0, tot = 0;
#pragma unroll
  for (int m = 0; m <= M; ++m) {
    chi += e[m] * ((acc_t)(M - m) / (acc_t)M);
    tot += e[m];
  }
  cf[0] = chi;
  suma = tot;
#pragma unroll
  for (int s = 1; s < M; s <<= 1) {  // level n with s = 2^n; support of d_{n,k}: endpoints k w .. (k+1) w
    const int w = M / s;
#pragma unroll
    for (int k = 0; k < s; ++k) {
      acc_t acc = 0;
#pragma unroll
      for (int i = 1; i < w; ++i) acc += e[k * w + i] * ((acc_t)(2 * i <= w ? i : w - i) / (acc_t)w);
      cf[s + k] = -acc;
    }
  }
}

// Render: endpoint masses -> coefficients at storage precision (stored when coeffs is not null) -> FP32 cells,
// and the absorbance total, written over the endpoint region as floats: cells [C*M][TP], then suma [C][TP].
template <int C, typename TS, int M>
__device__ __forceinline__ void ep_render_convert(const Geom& g, const TileRef& r, acc_t* le, TS* coeffs) {
  const uint32_t TP = g.tile_px;
  const uint32_t q = threadIdx.x;
  const bool have = q < TP * C;
  const uint32_t c = have ? q / TP : 0, lp = have ? q - c * TP : 0;
  float v[M];
  float sa = 0.f;
  if (have) {
    acc_t e[M + 1], cf[M], suma;
#pragma unroll
    for (int m = 0; m <= M; ++m) e[m] = le[(c * (M + 1) + m) * TP + lp];
    endpoints_to_coeffs<M>(e, cf, suma);
    TS s[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      s[m] = narrow_d<TS>(cf[m]);
      v[m] = widen<TS>(s[m]);
    }
    uint64_t p;
    if (coeffs && tile_pixel(g, r, lp, p)) store_row<TS, M>(coeffs + (p * C + c) * M, s);
    synth_regs<M>(v);
    sa = (float)suma;
  }
  __syncthreads();  // every endpoint mass has been read before the FP32 values overwrite the region
  if (have) {
    float* lc32 = (float*)le;
#pragma unroll
    for (int m = 0; m < M; ++m) lc32[(c * M + m) * TP + lp] = v[m];
    lc32[(C * M + c) * TP + lp] = sa;
  }
}

template <int C, typename TS>
__device__ __forceinline__ void ep_render_convert(const Geom& g, const TileRef& r, acc_t* le, TS* coeffs) {
  switch (g.M) {
    case 2: ep_render_convert<C, TS, 2>(g, r, le, coeffs); break;
    case 4: ep_render_convert<C, TS, 4>(g, r, le, coeffs); break;
    case 8: ep_render_convert<C, TS, 8>(g, r, le, coeffs); break;
    case 16: ep_render_convert<C, TS, 16>(g, r, le, coeffs); break;
    default: ep_render_convert<C, TS, 32>(g, r, le, coeffs); break;
  }
}

// ------------------------------------------------------------------------------------------- E5B9G9R9 storage
//
// Three channels share one word per coefficient index (wt.h). Coefficient 0 (chi) is >= 0 and every wavelet
// coefficient <= 0 (section 2.3.1), so the words hold magnitudes and the sign is restored from the index.

__device__ __forceinline__ float e5_sign(uint32_t m) { return m ? -1.f : 1.f; }

// Render: endpoint masses -> coefficients -> FP32 -> packed (stored when coeffs is not null) -> the decoded
// values -> FP32 cells; then cells [3*M][TP] and the absorbance totals [3][TP] as floats over the endpoint region.
template <int M>
__device__ __forceinline__ void e5_render_convert(const Geom& g, const TileRef& r, acc_t* le, uint32_t* coeffs) {
  constexpr uint32_t C = 3;
  const uint32_t TP = g.tile_px;
  const uint32_t q = threadIdx.x;
  const bool have = q < TP * C;
  const uint32_t c = have ? q / TP : 0, lp = have ? q - c * TP : 0;
  float fv[M];
  float sa = 0.f;
  if (have) {
    acc_t e[M + 1], cf[M], suma;
#pragma unroll
    for (int m = 0; m <= M; ++m) e[m] = le[(c * (M + 1) + m) * TP + lp];
    endpoints_to_coeffs<M>(e, cf, suma);
#pragma unroll
    for (int m = 0; m < M; ++m) fv[m] = (float)cf[m];
    sa = (float)suma;
  }
  __syncthreads();  // every endpoint mass has been read
  float* lf = (float*)le;
  if (have) {
#pragma unroll
    for (int m = 0; m < M; ++m) lf[(c * M + m) * TP + lp] = fv[m];
  }
  __syncthreads();
  for (uint32_t px = threadIdx.x; px < TP; px += blockDim.x) {
    uint32_t w[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const float sg = e5_sign(m);
      w[m] = e5_pack(sg * lf[(0 * M + m) * TP + px], sg * lf[(1 * M + m) * TP + px], sg * lf[(2 * M + m) * TP + px]);
#pragma unroll
      for (uint32_t c2 = 0; c2 < C; ++c2) lf[(c2 * M + m) * TP + px] = sg * e5_unpack(w[m], c2);
    }
    uint64_t p;
    if (coeffs && tile_pixel(g, r, px, p)) store_row<uint32_t, M>(coeffs + p * M, w);
  }
  __syncthreads();
  if (have) {
    float v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = lf[(c * M + m) * TP + lp];
    synth_regs<M>(v);
#pragma unroll
    for (int m = 0; m < M; ++m) lf[(c * M + m) * TP + lp] = v[m];
    lf[(C * M + c) * TP + lp] = sa;
  }
}

// Build (accumulating): words += the coefficients of the endpoint masses (decoded, added in FP64, rounded to
// FP32 and packed again).
template <int M>
__device__ __forceinline__ void e5_build_store(const Geom& g, const TileRef& r, acc_t* le, uint32_t* coeffs) {
  constexpr uint32_t C = 3;
  const uint32_t TP = g.tile_px;
  const uint32_t q = threadIdx.x;
  const bool have = q < TP * C;
  const uint32_t c = have ? q / TP : 0, lp = have ? q - c * TP : 0;
  acc_t cf[M];
  if (have) {
    acc_t e[M + 1], suma;
#pragma unroll
    for (int m = 0; m <= M; ++m) e[m] = le[(c * (M + 1) + m) * TP + lp];
    endpoints_to_coeffs<M>(e, cf, suma);
  }
  __syncthreads();  // every endpoint mass has been read
  if (have) {
#pragma unroll
    for (int m = 0; m < M; ++m) le[(c * M + m) * TP + lp] = cf[m];
  }
  __syncthreads();
  for (uint32_t px = threadIdx.x; px < TP; px += blockDim.x) {
    uint64_t p;
    if (!tile_pixel(g, r, px, p)) continue;
    uint32_t* gp = coeffs + p * M;
    uint32_t w[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint32_t old = gp[m];
      const double sg = e5_sign(m);
      float v[C];
#pragma unroll
      for (uint32_t c2 = 0; c2 < C; ++c2) v[c2] = (float)(sg * le[(c2 * M + m) * TP + px] + (double)e5_unpack(old, c2));
      w[m] = e5_pack(v[0], v[1], v[2]);
    }
    store_row<uint32_t, M>(gp, w);
  }
}

template <typename F>
__device__ __forceinline__ void with_m(const Geom& g, F&& f) {
  switch (g.M) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 32>{}); break;
  }
}

// Load: words -> signed values of T in LDS [3*M][TP] (zero off-frame).
template <typename T>
__device__ __forceinline__ void e5_load_tile(const Geom& g, const TileRef& r, T* lc, const uint32_t* coeffs) {
  const uint32_t TP = g.tile_px, M = g.M;
  for (uint32_t q = threadIdx.x; q < TP * M; q += blockDim.x) {
    const uint32_t lp = q / M, m = q - lp * M;
    uint64_t p;
    const uint32_t w = tile_pixel(g, r, lp, p) ? coeffs[p * M + m] : 0u;
    const float sg = e5_sign(m);
#pragma unroll
    for (uint32_t c = 0; c < 3; ++c) lc[(c * M + m) * TP + lp] = (T)(sg * e5_unpack(w, c));
  }
}

// Build (accumulating): coeffs += coefficients of the endpoint masses, one pixel/channel per thread.
template <int C, typename TS, int M>
__device__ __forceinline__ void ep_build_store(const Geom& g, const TileRef& r, const acc_t* le, TS* coeffs) {
  const uint32_t TP = g.tile_px;
  const uint32_t q = threadIdx.x;
  if (q >= TP * C) return;
  const uint32_t c = q / TP, lp = q - c * TP;
  uint64_t p;
  if (!tile_pixel(g, r, lp, p)) return;
  acc_t e[M + 1], cf[M], suma;
#pragma unroll
  for (int m = 0; m <= M; ++m) e[m] = le[(c * (M + 1) + m) * TP + lp];
  endpoints_to_coeffs<M>(e, cf, suma);
  TS* gp = coeffs + (p * C + c) * M;
  TS s[M];
#pragma unroll
  for (int m = 0; m < M; ++m) s[m] = narrow_d<TS>(cf[m] + (acc_t)widen<TS>(gp[m]));
  store_row<TS, M>(gp, s);
}

template <int C, typename TS>
__device__ __forceinline__ void ep_build_store(const Geom& g, const TileRef& r, const acc_t* le, TS* coeffs) {
  switch (g.M) {
    case 2: ep_build_store<C, TS, 2>(g, r, le, coeffs); break;
    case 4: ep_build_store<C, TS, 4>(g, r, le, coeffs); break;
    case 8: ep_build_store<C, TS, 8>(g, r, le, coeffs); break;
    case 16: ep_build_store<C, TS, 16>(g, r, le, coeffs); break;
    default: ep_build_store<C, TS, 32>(g, r, le, coeffs); break;
  }
}

// ------------------------------------------------------------------------------------------- evaluate

// la is [AL][TP] of acc_t: rows 0..2 colour, then sum a (C = 1) or sum a_r, a_g, a_b (C = 3).
// lc holds FP32 cells (CELLS) or coefficients of type T (otherwise), [C*M][TP].
template <int C, bool CELLS, typename T, bool SUMA = true>
__device__ __forceinline__ void eval_add(const T* lc, acc_t* la, const Geom& g, const Frag<C>& f,
                                         const uint32_t* lb) {
  const uint32_t TP = g.tile_px;
  uint32_t j;
  float t, omt;
  cell_coord(f.x, lb, TP, f.lp, g.M, j, t, omt);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const T* cf = lc + (c * g.M) * TP + f.lp;
    float lo, hi;
    if (CELLS) {
      hi = (float)cf[j * TP];
      lo = j ? (float)cf[(j - 1) * TP] : 0.f;
    } else {
      hi = cell_from_coeffs<T>(cf, TP, g, j);
      lo = j ? cell_from_coeffs<T>(cf, TP, g, j - 1) : 0.f;
    }
    const float At = fmaf(t, hi, omt * lo);
    const float v = __expf(-At);
    const float alc = alpha_of(f.al[c]);
    if (C == 1) {
      const float w = alc * v;
      atomicAdd(la + 0 * TP + f.lp, (acc_t)(w * f.rgb[0]));
      atomicAdd(la + 1 * TP + f.lp, (acc_t)(w * f.rgb[1]));
      atomicAdd(la + 2 * TP + f.lp, (acc_t)(w * f.rgb[2]));
      if (SUMA) atomicAdd(la + 3 * TP + f.lp, (acc_t)f.al[c]);
    } else {
      atomicAdd(la + c * TP + f.lp, (acc_t)(alc * f.rgb[c] * v));
      if (SUMA) atomicAdd(la + (3 + c) * TP + f.lp, (acc_t)f.al[c]);
    }
  }
}

template <int C, bool CELLS, typename T, bool SUMA = true>
__device__ __forceinline__ void eval_tile(const Binned& b, const Geom& g, const TileRef& r, const T* lc,
                                          acc_t* la, const uint32_t* lb) {
  if (serial_records(g, r.beg, r.end, [&](uint32_t i) {
        Frag<C> f;
        if (load_full<C>(b, i, f)) eval_add<C, CELLS, T, SUMA>(lc, la, g, f, lb);
      }))
    return;
  uint32_t i = r.beg + threadIdx.x;
  // U whole records per thread in flight per step
  constexpr int U = eval_unroll<C>();
  for (; i + (U - 1) * blockDim.x < r.end; i += U * blockDim.x) {
    Frag<C> f[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ok[u] = load_full<C>(b, i + u * blockDim.x, f[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) eval_add<C, CELLS, T, SUMA>(lc, la, g, f[u], lb);
  }
  for (; i < r.end; i += blockDim.x) {
    Frag<C> f0;
    if (load_full<C>(b, i, f0)) eval_add<C, CELLS, T, SUMA>(lc, la, g, f0, lb);
  }
}

// ------------------------------------------------------------------------------------------- tile <-> global

// Coefficient tile between LDS ([C*M][TP] of T) and global memory ([P][C][M] of TS). Work item q covers VW
// consecutive elements of one pixel, so consecutive lanes touch consecutive global addresses.
// MODE 0: load (zero off-frame), 1: store, 2: round to TS in place and store when coeffs is not null.
template <int C, typename TS, int MODE, typename T>
__device__ __forceinline__ void coeff_tile_io(const Geom& g, const TileRef& r, T* lc, TS* coeffs) {
  if constexpr (is_e5<TS>::value) {
    // packed storage: loads only (stores run on the endpoint path, make_geom)
    if (MODE == 0) e5_load_tile<T>(g, r, lc, (const uint32_t*)coeffs);
  } else {
  const uint32_t TP = g.tile_px, per = C * g.M;
  const uint32_t VW = g.M < 4 ? g.M : 4;
  const uint32_t groups = per / VW;
  for (uint32_t q = threadIdx.x; q < TP * groups; q += blockDim.x) {
    const uint32_t lp = q / groups, e0 = (q - lp * groups) * VW;
    uint64_t p;
    const bool in = tile_pixel(g, r, lp, p);
    TS* gp = coeffs ? coeffs + p * per + e0 : nullptr;
    for (uint32_t e = 0; e < VW; ++e) {
      T* l = lc + (e0 + e) * TP + lp;  // row (c * M + m) = e0 + e
      if (MODE == 0) {
        *l = in ? (T)widen<TS>(gp[e]) : (T)0;
      } else if (MODE == 1) {
        if (in) gp[e] = narrow_d<TS>((double)*l);
      } else {
        const TS s = narrow_d<TS>((double)*l);
        *l = (T)widen<TS>(s);
        if (in && gp) gp[e] = s;
      }
    }
  }
  }
}

// ------------------------------------------------------------------------------------------- kernels

// LDS of the tile kernels, per pixel: render 8 (C M + AL) bytes, build 8 C M, evaluate 4 C M + 8 AL.
template <int C, typename TS>
__global__ __launch_bounds__(kTileThreads) void k_build(Binned b, Geom g, TS* __restrict__ coeffs) {
  extern __shared__ acc_t smem_d[];
  acc_t* lc = smem_d;
  uint32_t tile;
  if (!binned_ok(b, g, tile)) return;
  const TileRef r = tile_ref(g, b, tile);
  // per-pixel depth bounds after the coefficient region
  uint32_t* lb = g.tight ? (uint32_t*)(smem_d + (g.ep ? C * (g.M + 1) : C * g.M) * g.tile_px) : nullptr;
  if (lb) bounds_tile<C>(b, g, r, lb);
  if (g.ep) {
    for (uint32_t e = threadIdx.x; e < C * (g.M + 1) * g.tile_px; e += blockDim.x) lc[e] = 0.0;
    __syncthreads();
    build_ep_tile<C>(b, g, r, lc, lb);
    __syncthreads();
    if constexpr (is_e5<TS>::value)
      with_m(g, [&](auto mm) { e5_build_store<decltype(mm)::value>(g, r, lc, (uint32_t*)coeffs); });
    else
      ep_build_store<C, TS>(g, r, lc, coeffs);
    return;
  }
  coeff_tile_io<C, TS, 0>(g, r, lc, coeffs);
  __syncthreads();
  build_tile<C>(b, g, r, lc, lb);
  __syncthreads();
  coeff_tile_io<C, TS, 1>(g, r, lc, coeffs);
}

template <int C, typename TS, bool CELLS>
__global__ __launch_bounds__(kTileThreads) void k_evaluate(Binned b, Geom g, const TS* __restrict__ coeffs,
                                                           float* __restrict__ accum) {
  extern __shared__ acc_t smem_d[];
  const uint32_t TP = g.tile_px;
  acc_t* la = smem_d;                              // [AL][TP] FP64
  float* lc = (float*)(smem_d + g.AL * TP);        // [C*M][TP] FP32
  uint32_t* lb = g.tight ? (uint32_t*)(lc + C * g.M * TP) : nullptr;  // per-pixel depth bounds
  uint32_t tile;
  if (!binned_ok(b, g, tile)) return;
  const TileRef r = tile_ref(g, b, tile);
  if (lb) bounds_tile<C>(b, g, r, lb);
  coeff_tile_io<C, TS, 0>(g, r, lc, const_cast<TS*>(coeffs));
  for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
    uint64_t p;
    const bool in = tile_pixel(g, r, lp, p);
    for (uint32_t k = 0; k < 3; ++k) la[k * TP + lp] = in ? accum[p * g.AW + k] : 0.0;
    for (uint32_t c = 0; c < C; ++c)
      la[(3 + c) * TP + lp] = in ? accum[p * g.AW + (C == 1 ? 3 : 4 + c)] : 0.0;
  }
  __syncthreads();
  if (CELLS) synth_tile_f32<C>(lc, g);
  __syncthreads();
  eval_tile<C, CELLS, float>(b, g, r, lc, la, lb);
  __syncthreads();
  for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
    uint64_t p;
    if (!tile_pixel(g, r, lp, p)) continue;
    for (uint32_t k = 0; k < 3; ++k) accum[p * g.AW + k] = (float)la[k * TP + lp];
    for (uint32_t c = 0; c < C; ++c) accum[p * g.AW + (C == 1 ? 3 : 4 + c)] = (float)la[(3 + c) * TP + lp];
  }
}

template <int C, typename TS, bool CELLS>
__global__ __launch_bounds__(kTileThreads) void k_render(Binned b, Geom g, TS* __restrict__ coeffs, float bg0,
                                                         float bg1, float bg2, float* __restrict__ out) {
  extern __shared__ acc_t smem_d[];
  const uint32_t TP = g.tile_px;
  uint32_t tile;
  if (!binned_ok(b, g, tile)) return;
  const TileRef r = tile_ref(g, b, tile);
  const float bg[3] = {bg0, bg1, bg2};
  if (g.ep) {
    // LDS: endpoint masses [C*(M+1)][TP] FP64 (then FP32 cells [C*M][TP] and sums of a [C][TP] in their
    // place), colour sums [3][TP] FP64
    acc_t* le = smem_d;
    acc_t* la = smem_d + C * (g.M + 1) * TP;
    uint32_t* lb = g.tight ? (uint32_t*)(la + 3 * TP) : nullptr;  // per-pixel depth bounds
    if (lb) bounds_tile<C>(b, g, r, lb);
    for (uint32_t e = threadIdx.x; e < (C * (g.M + 1) + 3) * TP; e += blockDim.x) smem_d[e] = 0.0;
    __syncthreads();
    build_ep_tile<C>(b, g, r, le, lb);
    __syncthreads();
    if constexpr (is_e5<TS>::value)
      with_m(g, [&](auto mm) { e5_render_convert<decltype(mm)::value>(g, r, le, (uint32_t*)coeffs); });
    else
      ep_render_convert<C, TS>(g, r, le, coeffs);
    __syncthreads();
    const float* cells = (const float*)le;
    eval_tile<C, true, float, false>(b, g, r, cells, la, lb);
    __syncthreads();
    const float* sa = cells + C * g.M * TP;
    for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
      uint64_t p;
      if (!tile_pixel(g, r, lp, p)) continue;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        out[p * 3 + q] = (float)la[q * TP + lp] + bg[q] * __expf(-sa[(C == 1 ? 0 : q) * TP + lp]);
    }
    return;
  }
  acc_t* lc = smem_d;                    // [C*M][TP] FP64, then FP32 cells in its first half (CELLS)
  acc_t* la = smem_d + C * g.M * TP;     // [AL][TP] FP64
  uint32_t* lb = g.tight ? (uint32_t*)(la + g.AL * TP) : nullptr;  // per-pixel depth bounds
  if (lb) bounds_tile<C>(b, g, r, lb);
  for (uint32_t e = threadIdx.x; e < (C * g.M + g.AL) * TP; e += blockDim.x) smem_d[e] = 0.0;
  __syncthreads();
  build_tile<C>(b, g, r, lc, lb);
  __syncthreads();
  // coefficients at storage precision: stored (optionally) and used for the evaluation
  if (CELLS) {
    coeffs_to_cells<C, TS>(g, r, lc, coeffs);
    __syncthreads();
    eval_tile<C, true, float>(b, g, r, (const float*)lc, la, lb);
  } else {
    coeff_tile_io<C, TS, 2>(g, r, lc, coeffs);
    __syncthreads();
    eval_tile<C, false, acc_t>(b, g, r, lc, la, lb);
  }
  __syncthreads();
  for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
    uint64_t p;
    if (!tile_pixel(g, r, lp, p)) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float suma = (float)la[(3 + (C == 1 ? 0 : q)) * TP + lp];
      out[p * 3 + q] = (float)la[q * TP + lp] + bg[q] * __expf(-suma);
    }
  }
}

// ------------------------------------------------------------------------------------------- one pass, previous frame
//
// The single-pass variant the paper proposes as future work: the frame's coefficients are built in the same pass
// that shades its fragments, so the shading reconstructs visibility from the PREVIOUS frame's coefficients, read
// at each pixel's reprojected position (an integer pixel map supplied by the caller; identity without one). Each
// binned record is read once instead of twice.

// Row of M storage values of one pixel/channel, 16 bytes at a time where the layout allows.
template <typename TS, int M>
__device__ __forceinline__ void load_row(const TS* src, TS (&s)[M]) {
  if ((M * sizeof(TS)) % 16 == 0) {
#pragma unroll
    for (int k = 0; k < (int)(M * sizeof(TS) / 16); ++k) {
      const uint4 u = ((const uint4*)src)[k];
      __builtin_memcpy((char*)s + 16 * k, &u, 16);
    }
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) s[m] = src[m];
  }
}

// FP32 cells [C*M][TP] of the previous frame for the tile's pixels: pixel p reads the previous buffer at
// map[p] (p without a map). Zero (no history: visibility 1) without a previous buffer, for a map entry >= P and
// for pixels outside the frame.
template <int C, typename TS, int M>
__device__ __forceinline__ void prev_cells(const Geom& g, const TileRef& r, const TS* prev, const uint32_t* map,
                                           float* lc) {
  const uint32_t TP = g.tile_px;
  for (uint32_t q = threadIdx.x; q < TP * C; q += blockDim.x) {
    const uint32_t c = q / TP, lp = q - c * TP;
    uint64_t p;
    uint32_t src = 0xffffffffu;
    if (prev && tile_pixel(g, r, lp, p)) src = map ? map[p] : (uint32_t)p;
    float v[M];
    if (src < g.P) {
      if constexpr (is_e5<TS>::value) {
        uint32_t w[M];
        load_row<uint32_t, M>((const uint32_t*)prev + (uint64_t)src * M, w);
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = e5_sign(m) * e5_unpack(w[m], c);
      } else {
        TS s[M];
        load_row<TS, M>(prev + ((uint64_t)src * C + c) * M, s);
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = widen<TS>(s[m]);
      }
      synth_regs<M>(v);
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) v[m] = 0.f;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) lc[(c * M + m) * TP + lp] = v[m];
  }
}

// One fragment of the single pass: its two endpoint masses into this frame's build (le, [C*(M+1)][TP] FP64) and
// its colour, weighted by the previous frame's visibility (lc), into the colour sums (la, [3][TP] FP64).
template <int C>
__device__ __forceinline__ void temporal_add(acc_t* le, const float* lc, acc_t* la, const Geom& g,
                                             const Frag<C>& f) {
  const uint32_t TP = g.tile_px, M1 = g.M + 1;
  uint32_t j;
  float t, omt;
  cell_coord(f.x, nullptr, TP, f.lp, g.M, j, t, omt);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float a = f.al[c];  // binned records hold the absorbance
    const float alc = alpha_of(a);
    acc_t* e = le + (c * M1 + j) * TP + f.lp;
    atomicAdd(e, (acc_t)(a * omt));
    atomicAdd(e + TP, (acc_t)(a * t));
    const float* cf = lc + (c * g.M) * TP + f.lp;
    const float hi = cf[j * TP];
    const float lo = j ? cf[(j - 1) * TP] : 0.f;
    const float v = __expf(-fmaf(t, hi, omt * lo));
    if (C == 1) {
      const float w = alc * v;
      atomicAdd(la + 0 * TP + f.lp, (acc_t)(w * f.rgb[0]));
      atomicAdd(la + 1 * TP + f.lp, (acc_t)(w * f.rgb[1]));
      atomicAdd(la + 2 * TP + f.lp, (acc_t)(w * f.rgb[2]));
    } else {
      atomicAdd(la + c * TP + f.lp, (acc_t)(alc * f.rgb[c] * v));
    }
  }
}

// LDS: endpoint masses [C*(M+1)][TP] FP64 (then this frame's FP32 cells and sums of a in their place), colour sums
// [3][TP] FP64, previous cells [C*M][TP] FP32. prev and coeffs may be the same buffer when map is null: a tile
// reads the previous coefficients of its own pixels before it writes theirs.
template <int C, typename TS>
__global__ __launch_bounds__(kTileThreads) void k_render_temporal(Binned b, Geom g, const TS* prev,
                                                                  const uint32_t* __restrict__ map, TS* coeffs,
                                                                  float bg0, float bg1, float bg2,
                                                                  float* __restrict__ out) {
  extern __shared__ acc_t smem_d[];
  const uint32_t TP = g.tile_px;
  uint32_t tile;
  if (!binned_ok(b, g, tile)) return;
  const TileRef r = tile_ref(g, b, tile);
  const float bg[3] = {bg0, bg1, bg2};
  acc_t* le = smem_d;
  acc_t* la = smem_d + C * (g.M + 1) * TP;
  float* lc = (float*)(la + 3 * TP);
  for (uint32_t e = threadIdx.x; e < (C * (g.M + 1) + 3) * TP; e += blockDim.x) smem_d[e] = 0.0;
  with_m(g, [&](auto mm) { prev_cells<C, TS, decltype(mm)::value>(g, r, prev, map, lc); });
  __syncthreads();
  const bool serial = serial_records(g, r.beg, r.end, [&](uint32_t i) {
    Frag<C> f;
    if (load_full<C>(b, i, f)) temporal_add<C>(le, lc, la, g, f);
  });
  uint32_t i = serial ? r.end : r.beg + threadIdx.x;
  for (; i + (kEvalUnroll - 1) * blockDim.x < r.end; i += kEvalUnroll * blockDim.x) {
    Frag<C> f[kEvalUnroll];
    bool ok[kEvalUnroll];
#pragma unroll
    for (int u = 0; u < kEvalUnroll; ++u) ok[u] = load_full<C>(b, i + u * blockDim.x, f[u]);
#pragma unroll
    for (int u = 0; u < kEvalUnroll; ++u)
      if (ok[u]) temporal_add<C>(le, lc, la, g, f[u]);
  }
  for (; i < r.end; i += blockDim.x) {
    Frag<C> f0;
    if (load_full<C>(b, i, f0)) temporal_add<C>(le, lc, la, g, f0);
  }
  __syncthreads();
  if constexpr (is_e5<TS>::value)
    with_m(g, [&](auto mm) { e5_render_convert<decltype(mm)::value>(g, r, le, (uint32_t*)coeffs); });
  else
    ep_render_convert<C, TS>(g, r, le, coeffs);
  __syncthreads();
  const float* sa = (const float*)le + C * g.M * TP;
  for (uint32_t lp = threadIdx.x; lp < TP; lp += blockDim.x) {
    uint64_t p;
    if (!tile_pixel(g, r, lp, p)) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      out[p * 3 + q] = (float)la[q * TP + lp] + bg[q] * __expf(-sa[(C == 1 ? 0 : q) * TP + lp]);
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

// ------------------------------------------------------------------------------------------- chromatic composite
//
// Composite over a background image sampled through each pixel's screen-space refraction offset, with the
// chromatic-aberration gather of section 3: k taps along the offset, tap i at parameter t = i / (k - 1) displaced
// by s = 1 + dispersion (t - 1/2) times the offset, each a bilinear sample of the background (clamp to edge),
// weighted per channel by the spectral weights (red: the smoothstep formula falling from 1 at t = 1/3 to 0 at
// t = 1/2; blue: rising from 0 at t = 1/2 to 1 at t = 2/3; green: the remainder) and normalised per channel.

__device__ __forceinline__ float smoothstep_formula(float e0, float e1, float x) {
  const float u = fminf(fmaxf((x - e0) / (e1 - e0), 0.f), 1.f);
  return u * u * (3.f - 2.f * u);
}

// Tap i of k for one pixel: the bilinear sample of every channel with a non-zero spectral weight, accumulated
// into num/den. The tap position is split into the pixel's integer coordinate and the offset's own integer and
// fractional parts, so the bilinear fractions keep the offset's precision at any frame size.
__device__ __forceinline__ void chromatic_tap(const Geom& g, const float* __restrict__ bgimg, uint32_t x, uint32_t y,
                                              float dx, float dy, float dispersion, uint32_t i, uint32_t k,
                                              float (&num)[3], float (&den)[3]) {
  const float t = (float)i / (float)(k - 1);
  float w[3];
  w[0] = smoothstep_formula(0.5f, 1.f / 3.f, t);
  w[2] = smoothstep_formula(0.5f, 2.f / 3.f, t);
  w[1] = 1.f - w[0] - w[2];
  const float sc = 1.f + dispersion * (t - 0.5f);
  const float ox = sc * dx, oy = sc * dy;
  const float fox = floorf(ox), foy = floorf(oy);
  const float fx = ox - fox, fy = oy - foy;  // exact
  // sample position minus the half-texel shift: (x + ox, y + oy); the left/top texel and the clamped pair (the
  // integer parts are bounded before conversion, so a NaN or huge offset still addresses the image's edge)
  const long lx = (long)x + (long)fminf(fmaxf(fox, -1e9f), 1e9f);
  const long ly = (long)y + (long)fminf(fmaxf(foy, -1e9f), 1e9f);
  const int Wm = (int)g.W - 1, Hm = (int)g.H - 1;
  const int x0 = (int)min<long>(max<long>(lx, 0), Wm), x1 = (int)min<long>(max<long>(lx + 1, 0), Wm);
  const int y0 = (int)min<long>(max<long>(ly, 0), Hm), y1 = (int)min<long>(max<long>(ly + 1, 0), Hm);
  const float* r0 = bgimg + (uint64_t)y0 * g.W * 3;
  const float* r1 = bgimg + (uint64_t)y1 * g.W * 3;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (w[q] == 0.f) continue;  // depends on the tap only (a constant when k is)
    const float a = r0[x0 * 3 + q], b = r0[x1 * 3 + q], c = r1[x0 * 3 + q], d = r1[x1 * 3 + q];
    const float v = (1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * c + fx * d);
    num[q] += w[q] * v;
    den[q] += w[q];
  }
}

// One pixel per thread. K > 0 fixes the tap count at compile time (the weights fold to constants and the taps'
// loads issue together); K = 0 takes it from `taps`.
template <int K>
__global__ __launch_bounds__(256) void k_resolve_chromatic(const float* __restrict__ accum, Geom g,
                                                           const float* __restrict__ bgimg,
                                                           const float* __restrict__ offset, float dispersion,
                                                           uint32_t taps, float* __restrict__ out) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  const uint32_t y = fastdiv(p, g.divW);
  const uint32_t x = p - y * g.W;
  const float2 o = ((const float2*)offset)[p];
  float num[3] = {0.f, 0.f, 0.f}, den[3] = {0.f, 0.f, 0.f};
  if constexpr (K > 0) {
#pragma unroll
    for (uint32_t i = 0; i < (uint32_t)K; ++i) chromatic_tap(g, bgimg, x, y, o.x, o.y, dispersion, i, K, num, den);
  } else {
    for (uint32_t i = 0; i < taps; ++i) chromatic_tap(g, bgimg, x, y, o.x, o.y, dispersion, i, taps, num, den);
  }
  float colour[3], suma[3];
  if (g.AW == 4) {
    const float4 a = ((const float4*)accum)[p];
    colour[0] = a.x; colour[1] = a.y; colour[2] = a.z;
    suma[0] = suma[1] = suma[2] = a.w;
  } else {
    const float4 a = ((const float4*)accum)[2 * (uint64_t)p];
    const float4 b = ((const float4*)accum)[2 * (uint64_t)p + 1];
    colour[0] = a.x; colour[1] = a.y; colour[2] = a.z;
    suma[0] = b.x; suma[1] = b.y; suma[2] = b.z;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) out[(uint64_t)p * 3 + q] = colour[q] + __expf(-suma[q]) * (num[q] / den[q]);
}

// ------------------------------------------------------------------------------------------- launchers

// LDS of the render (with_accum) and build kernels: endpoint masses (+ three colour sums), or coefficient
// sums (+ AL accumulations).
size_t lds_tile_bytes(const Geom& g, bool with_accum) {
  const size_t bounds = g.tight ? 8ull * g.tile_px : 0;
  if (g.ep) return (size_t)g.tile_px * (g.C * (g.M + 1) + (with_accum ? 3 : 0)) * sizeof(acc_t) + bounds;
  return (size_t)g.tile_px * (g.C * g.M + (with_accum ? g.AL : 0)) * sizeof(acc_t) + bounds;
}

size_t lds_temporal_bytes(const Geom& g) {
  return (size_t)g.tile_px * ((g.C * (g.M + 1) + 3) * sizeof(acc_t) + g.C * g.M * sizeof(float));
}

static size_t lds_eval_bytes(const Geom& g) {
  return (size_t)g.tile_px * (4 * g.C * g.M + 8 * g.AL + (g.tight ? 8 : 0));
}

// The render kernel expands cells in registers, one pixel/channel per thread.
static bool render_cells(const Geom& g) { return g.M <= 32 && g.tile_px * g.C <= (uint32_t)kTileThreads; }

template <typename K>
static hipError_t prep(K kernel, size_t lds) {
  if (lds > 65536)
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
  if (g.dtype == WT_E5B9G9R9) {
    if (!g.ep) return hipErrorInvalidValue;  // make_geom puts packed storage on the endpoint path
    return f(std::integral_constant<int, 3>{}, (e5_t*)nullptr);
  }
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
  const size_t lds = lds_eval_bytes(g);
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
    auto k = render_cells(g) ? k_render<C, TS, true> : k_render<C, TS, false>;
    hipError_t err = prep(k, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(g.ntiles), dim3(kTileThreads), lds, s, b, g, (TS*)coeffs, bg[0], bg[1], bg[2], out);
    return hipGetLastError();
  });
}

hipError_t launch_render_temporal(const Geom& g, const Binned& b, const float* bg, const void* prev,
                                  const uint32_t* map, void* coeffs, float* out, hipStream_t s) {
  if (!g.ep) return hipErrorNotSupported;  // the API limits the one-pass render to the endpoint path
  const size_t lds = lds_temporal_bytes(g);
  return dispatch(g, [&](auto cc, auto* tag) {
    constexpr int C = decltype(cc)::value;
    using TS = std::remove_pointer_t<decltype(tag)>;
    auto k = k_render_temporal<C, TS>;
    hipError_t err = prep(k, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(g.ntiles), dim3(kTileThreads), lds, s, b, g, (const TS*)prev, map, (TS*)coeffs,
                       bg[0], bg[1], bg[2], out);
    return hipGetLastError();
  });
}

hipError_t launch_resolve_chromatic(const Geom& g, const float* accum, const float* bgimg, const float* offset,
                                   float dispersion, uint32_t taps, float* out, hipStream_t s) {
  const unsigned grid = (unsigned)(((uint64_t)g.P + 255) / 256);
  auto k = taps == 3 ? k_resolve_chromatic<3> : taps == 5 ? k_resolve_chromatic<5> : taps == 7 ? k_resolve_chromatic<7>
         : taps == 9 ? k_resolve_chromatic<9> : k_resolve_chromatic<0>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, accum, g, bgimg, offset, dispersion, taps, out);
  return hipGetLastError();
}

hipError_t launch_resolve(const Geom& g, const float* accum, const float* bg, float* out, hipStream_t s) {
  const uint64_t n = (uint64_t)g.P * 3;
  const unsigned grid = (unsigned)std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_resolve, dim3(grid), dim3(256), 0, s, accum, g, bg[0], bg[1], bg[2], out);
  return hipGetLastError();
}

}  // namespace wt
