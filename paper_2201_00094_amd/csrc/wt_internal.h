// Internal declarations shared by the libwt translation units: frame geometry, workspace layout and the
// kernel launchers. Nothing here is part of the public ABI (include/wt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt.h"

namespace wt {

// Workgroups of a grid are dealt to the eight XCDs of an MI355X round-robin (workgroup b runs on XCD b % 8),
// and each XCD has its own L2. The binning keeps one write frontier per (tile, XCD class) so that the
// partial cache lines of a frontier are filled inside a single L2 before they are written back.
constexpr uint32_t kClasses = 8;
constexpr uint32_t kCursorPad = 1;  // words per write cursor in the workspace's cursor tables
constexpr uint32_t kPer = 8;               // fragments per scatter thread (held in registers)
constexpr uint32_t kMaxLdsBins = 8192;     // bins one scatter table holds (super-tiles of a two-level binning)
constexpr uint32_t kMaxHistBins = 36864;   // tiles one histogram table holds (144 KB of LDS)
constexpr uint32_t kTwoLevelTiles = 4096;  // frames with more tiles are binned in two levels (super-tiles, then tiles)
constexpr uint32_t kMaxSupers = 1024;      // super-tiles of the first level at most
constexpr uint32_t kMaxSub = 64;           // tiles per super-tile at most
constexpr uint32_t kLdsBytes = 160 * 1024; // LDS of one CDNA4 compute unit (also the per-workgroup limit)
constexpr uint32_t kMaxTilePx = 2048;
constexpr uint32_t kTileThreads = 1024;    // workgroup size of the per-tile kernels
constexpr uint32_t kScanRange = 16384;     // segments one scan workgroup covers (a multiple of kClasses)
constexpr float kAlphaMax = 0.99999994f;   // 1 - 2^-24

// Division of 32-bit values by a divisor fixed per frame, without a hardware divide (Granlund and Montgomery,
// "Division by invariant integers using multiplication", 1994, the round-up form for unsigned 32-bit operands):
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0),
// t = mulhi(m, n), equals floor(n / d) for every n < 2^32 and 1 <= d < 2^32.
struct FastDiv {
  uint32_t m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  FastDiv f;
  f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 1 ? l - 1 : 0;
  return f;
}

__host__ __device__ inline uint32_t fastdiv(uint32_t n, const FastDiv& f) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t t = __umulhi(f.m, n);
#else
  const uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
#endif
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// -ln(1 - al) for al in [0, 1 - 2^-24] to a few ulp, in a few dozen instructions instead of a general-purpose
// log1p. For al <= 1/2 it is the series -ln(1 - al) = 2 atanh(u) = 2 (u + u^3/3 + u^5/5 + ...) with
// u = al / (2 - al) <= 1/3, summed to u^15/15 (what is left is below 2^-29 of the sum); 2u is formed as
// 2 al / (2 - al) so that denormal alphas do not underflow. Above 1/2, 1 - al is exact in FP32 (Sterbenz) and
// -ln(1 - al) = -log2(1 - al) ln 2.
__host__ __device__ inline float neg_log1m(float al) {
  if (al <= 0.5f) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float v = (2.f * al) * __builtin_amdgcn_rcpf(2.f - al);
#else
    const float v = (2.f * al) / (2.f - al);
#endif
    const float u2 = 0.25f * v * v;
    float p = 1.f / 15.f;
    p = fmaf(p, u2, 1.f / 13.f);
    p = fmaf(p, u2, 1.f / 11.f);
    p = fmaf(p, u2, 1.f / 9.f);
    p = fmaf(p, u2, 1.f / 7.f);
    p = fmaf(p, u2, 1.f / 5.f);
    p = fmaf(p, u2, 1.f / 3.f);
    p = fmaf(p, u2, 1.f);
    return v * p;
  }
#if defined(__HIP_DEVICE_COMPILE__)
  return -__log2f(1.f - al) * 0.693147182f;
#else
  return -log2f(1.f - al) * 0.693147182f;
#endif
}

// FP64 -> FP32 rounded to odd, as a bit pattern: the nearest FP32 value toward zero, with its last bit set when the
// conversion is inexact (NaN stays NaN; beyond the FP32 range the largest finite value, odd). Rounding that value
// once more, to nearest, into a format whose significand is at least two bits shorter at every magnitude (FP16 and
// BF16, subnormals included) gives the FP64 value rounded once: the odd last bit keeps a value that lies off a
// midpoint of the narrow format off it (Boldo and Melquiond, "Emulation of FMA and correctly rounded sums: proved
// algorithms using rounding to odd", IEEE Transactions on Computers, 2008). Two hardware conversions and a compare,
// where rounding the FP64 bit pattern with integer operations takes some fifty instructions.
__host__ __device__ inline uint32_t f64_to_f32_odd_bits(double v) {
  const float f = (float)v;
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  const double b = (double)f;
  if (b != v) {
    if (__builtin_fabs(b) > __builtin_fabs(v)) u -= 1u;  // rounded away from zero: one place back toward it
    u |= 1u;
  }
  return u;
}

// FP64 -> FP16 bit pattern, rounded once to nearest even: round to odd in FP32, then the FP32 -> FP16 conversion
// (to nearest even; one instruction on the GPU).
__host__ __device__ inline uint16_t f64_to_f16_bits(double v) {
  const uint32_t u = f64_to_f32_odd_bits(v);
  float f;
  __builtin_memcpy(&f, &u, 4);
  const _Float16 h = (_Float16)f;
  uint16_t r;
  __builtin_memcpy(&r, &h, 2);
  return r;
}

// FP64 -> BF16 bit pattern, rounded once to nearest even: round to odd in FP32, then to nearest even on the FP32
// bit pattern (a carry out of the mantissa moves into the exponent, up to infinity); NaN stays a quiet NaN.
__host__ __device__ inline uint16_t f64_to_bf16_bits(double v) {
  const uint32_t u = f64_to_f32_odd_bits(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Frame geometry as the kernels see it.
struct Geom {
  uint32_t W, H, P;      // frame
  uint32_t C, rank, M, L;// channels, rank, coefficients per channel (2^L), L = rank + 1
  uint32_t TW, TH;       // tile extent in pixels (powers of two)
  uint32_t lTW, lTH;     // log2 of TW, TH
  FastDiv divW;          // division by W
  uint32_t tilesX, tilesY, ntiles, tile_px;
  uint32_t NX;           // write-frontier classes (kClasses, or 1 when the tile count is large)
  uint32_t lds_bins;     // 1: LDS-staged scatter; 0: one global atomic per fragment
  uint32_t rb;           // bins of the scatter table (tiles of a one-level binning)
  uint32_t two;          // 1: two-level binning (super-tiles of SW x SH tiles, then tiles)
  uint32_t SW, SH, lSW, lSH, sX, sY, nsuper;
  uint32_t hrb;          // tiles per histogram table (range)
  uint32_t AW;           // accum floats per pixel in global memory: 4 (C = 1) or 8 (C = 3)
  uint32_t AL;           // accumulation floats per pixel in LDS: 4 (C = 1) or 6 (C = 3)
  uint32_t dtype;        // wt_dtype of the coefficient storage
  uint32_t ep;           // 1: the build accumulates endpoint masses (M <= 32, one pixel/channel per thread)
  uint32_t tight;        // 1: per-pixel depth bounds (WT_TIGHT_DEPTH); the tile kernels keep them in LDS
  uint32_t temporal;     // 1: tiles sized for the one-pass render against the previous frame (WT_TEMPORAL)
  uint32_t serial;       // 1: WT_DETERMINISTIC (stream-order binning by one thread, one thread per tile's records)
  uint32_t sthreads;     // scatter workgroup size
  uint32_t kper;         // fragments per scatter thread (4 or kPer)
  uint32_t chunk;        // fragments per scatter workgroup = sthreads * kper (also the class granularity)
};

// Binned fragment records, two arrays of structures in the same order:
//   head [cap][2 + C]: tile-local pixel index, depth, and per channel the absorbance -ln(1 - alpha) of the clamped
//                      alpha (forward binning) or alpha itself (binning for the gradient)   (all the build reads)
//   tail [cap][3 or 4]: rgb[3], then the stream index when recorded
constexpr uint32_t head_dwords(uint32_t C) { return 2 + C; }
constexpr uint32_t tail_dwords(bool with_index) { return 3 + (with_index ? 1 : 0); }
constexpr uint32_t record_dwords(uint32_t C, bool with_index) { return head_dwords(C) + tail_dwords(with_index); }

// The first bytes of every workspace: what the binning left there, so that each later call over the binned stream
// can check that the stream was binned completely, under its own layout, before it reads a table or a record.
struct WsHeader {
  unsigned long long dropped;  // fragments dropped by the last binning (pixel out of range, NaN)
  uint32_t errors;             // sticky kWsErr* bits, reported and cleared by wt_dropped_count
  uint32_t fault;              // the current binning's scatter refused to write (cleared by the count)
  unsigned long long counted;  // stamp of the last count: layout, record format and the stream counted
  unsigned long long binned;   // stamp of the last complete binning (layout and record format), or 0
  unsigned long long magic;    // kWsMagic once the device has written this header (fresh memory holds anything)
};
constexpr unsigned long long kWsMagic = 0x5754776f726b7370ull;
constexpr uint32_t kWsErrMismatch = 1u;  // a call over the binned stream found no complete binning in its layout
constexpr uint32_t kWsErrScatter = 2u;   // a scatter did not follow a count of the same stream and layout, or its
                                         // stream put more fragments in a tile than were counted

// Raise an error bit in a header, starting the error word from zero if the device never wrote this header.
__device__ __forceinline__ void ws_raise(WsHeader* h, uint32_t bit) {
  if (h->magic != kWsMagic) {
    h->errors = 0;
    h->magic = kWsMagic;
  }
  atomicOr(&h->errors, bit);
}

// 64-bit FNV-1a over 32-bit words; never 0 (0 marks "no binning").
__host__ __device__ inline unsigned long long stamp_words(const uint32_t* w, int n) {
  unsigned long long h = 0xcbf29ce484222325ull;
  for (int i = 0; i < n; ++i) {
    for (int b = 0; b < 4; ++b) {
      h ^= (w[i] >> (8 * b)) & 0xffu;
      h *= 0x100000001b3ull;
    }
  }
  return h ? h : 1ull;
}

// Device workspace: a header, the tile tables and the binned records.
struct Layout {
  size_t header;   // WsHeader (256 bytes reserved)
  size_t counts;   // uint32 [NX][ntiles]
  size_t offsets;  // uint32 [ntiles * NX + 1], tile-major: segment (t, x) = [off[t*NX+x], off[t*NX+x+1])
  size_t cursors;  // uint32 [NX][ntiles]
  size_t order;    // uint32 [ntiles]: tiles by descending fragment count (heaviest first)
  size_t scan;     // uint32 [G][1 + 256]: per-workgroup totals and size-class counts of a multi-workgroup scan
  size_t heads;    // uint32 [cap][head_dwords(C)]
  size_t tails;    // uint32 [cap][tail_dwords(true)]
  // two-level binning only: the first level over super-tiles
  size_t counts1;  // uint32 [NX][nsuper]
  size_t offsets1; // uint32 [nsuper * NX + 1]
  size_t cursors1; // uint32 [NX][nsuper]
  size_t order1;   // uint32 [nsuper] (unused order of the super-tiles)
  size_t heads1;   // uint32 [cap][head_dwords(C)]: tile-local pixel replaced by the super-tile-local pixel
  size_t tails1;   // uint32 [cap][tail_dwords(true)]
  size_t total;    // bytes
  uint64_t cap;    // fragment capacity
};

// Pointers into a workspace, as passed to kernels.
struct Binned {
  const uint32_t* offsets;
  const uint32_t* order;  // workgroup b processes tile order[b]
  const uint32_t* head;
  const uint32_t* tail;
  uint32_t DH, DT;        // dwords per head / tail entry
  WsHeader* hdr;          // checked by every tile kernel before it reads a table: hdr->binned == stamp
  unsigned long long stamp;
  uint64_t cap;           // records the layout holds
};

// backward = true picks tiles for the gradient kernel, which holds cell values and their adjoints.
Geom make_geom(const wt_frame_desc& d, bool backward = false);
// Geometry of the first binning level: super-tiles of g.SW x g.SH tiles as the bins, same chunking as g.
Geom super_geom(const Geom& g);
Layout make_layout(const Geom& g, uint64_t cap);
uint64_t capacity_for(const Geom& g, size_t ws_bytes);
size_t lds_tile_bytes(const Geom& g, bool with_accum);
size_t lds_backward_bytes(const Geom& g);
size_t lds_temporal_bytes(const Geom& g);
Binned binned_view(const Geom& g, const Layout& l, const void* ws, bool with_index);
// Stamp of a complete binning under this layout and record format, and of a count of this stream under it.
unsigned long long layout_stamp(const Geom& g, const Layout& l, bool with_index);
unsigned long long count_stamp(const Geom& g, const Layout& l, const wt_fragments& f);
// Fill n words at p with v (a kernel: safe inside captured graphs).
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);

// Launchers (return hipError_t of the launch).
hipError_t launch_bin(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                      hipStream_t s);
hipError_t launch_bin_count(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, hipStream_t s);
hipError_t launch_bin_scatter(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                              hipStream_t s);
hipError_t launch_build(const Geom& g, const Binned& b, void* coeffs, hipStream_t s);
hipError_t launch_evaluate(const Geom& g, const Binned& b, const void* coeffs, float* accum, hipStream_t s);
hipError_t launch_resolve(const Geom& g, const float* accum, const float* bg, float* out, hipStream_t s);
hipError_t launch_render(const Geom& g, const Binned& b, const float* bg, void* coeffs, float* out, hipStream_t s);
hipError_t launch_render_temporal(const Geom& g, const Binned& b, const float* bg, const void* prev,
                                  const uint32_t* map, void* coeffs, float* out, hipStream_t s);
hipError_t launch_resolve_chromatic(const Geom& g, const float* accum, const float* bgimg, const float* offset,
                                   float dispersion, uint32_t taps, float* out, hipStream_t s);
hipError_t launch_backward(const Geom& g, const Binned& b, const void* coeffs, const float* accum, const float* bg,
                           const float* grad_out, float* grad_alpha, float* grad_rgb, uint64_t count,
                           hipStream_t s);

}  // namespace wt
