// Ingest and screen-tile binning of an unordered fragment stream.
//
// The paper builds and evaluates inside a raster pipeline, where fragments of one screen region arrive on
// the same shader core (section 2.1). A stored stream carries no such locality, and on this GPU per-fragment
// random atomics into a frame-sized coefficient buffer run at a few billion fragments per second. So the
// stream is first regrouped by screen tile (a counting sort: histogram, scan, scatter), after which every
// per-pixel update of the build and evaluate passes happens in the LDS of the compute unit owning the tile.
//
// Kernels:
//   k_hist     reads pixel ids (4 B/fragment); per-workgroup LDS histogram per tile; range drops counted.
//   k_scan     exclusive scan of the (tile, class) counts into segment offsets and write cursors.
//   k_scatter  per chunk of kChunk fragments: LDS count, one cursor reservation per touched tile, then each
//              fragment is written (SoA) at its reserved slot. NaN fragments are counted and still binned;
//              the tile kernels skip them.
// A chunk's class is chunk % NX in both k_hist and k_scatter; with one chunk per scatter workgroup the class
// is also the XCD the workgroup runs on, so each (tile, class) write frontier is filled inside one L2.
#include <algorithm>

#include "wt_common.h"

namespace wt {

static uint32_t floor_pow2(uint32_t v) {
  uint32_t r = 1;
  while (r * 2 <= v) r *= 2;
  return r;
}

Geom make_geom(const wt_frame_desc& d, bool backward) {
  Geom g{};
  g.W = d.width;
  g.H = d.height;
  g.P = d.width * d.height;
  g.C = d.channels;
  g.rank = d.rank;
  g.L = d.rank + 1;
  g.M = 1u << g.L;
  g.AW = (d.channels == 3) ? 8 : 4;
  g.dtype = d.coeff_dtype;
  // Largest power-of-two tile whose FP32 coefficient tile fits the LDS budget, at most 32 x 32 pixels.
  const uint32_t per_px = g.C * g.M * 4;
  uint32_t px = std::max<uint32_t>(1, (backward ? kCoeffLdsBudget / 2 : kCoeffLdsBudget) / per_px);
  px = std::min<uint32_t>(floor_pow2(px), 1024);
  uint32_t e = 0;
  while ((1u << e) < px) ++e;
  g.TW = 1u << ((e + 1) / 2);
  g.TH = 1u << (e / 2);
  g.tile_px = g.TW * g.TH;
  g.tilesX = (g.W + g.TW - 1) / g.TW;
  g.tilesY = (g.H + g.TH - 1) / g.TH;
  g.ntiles = g.tilesX * g.tilesY;
  g.lds_bins = g.ntiles <= kMaxLdsBins ? 1 : 0;
  g.NX = g.lds_bins ? kClasses : 1;
  return g;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout make_layout(const Geom& g, uint64_t cap) {
  Layout l{};
  size_t o = 0;
  l.header = o;
  o += 256;
  l.counts = o;
  o = align256(o + 4ull * g.NX * g.ntiles);
  l.offsets = o;
  o = align256(o + 4ull * (g.NX * (uint64_t)g.ntiles + 1));
  l.cursors = o;
  o = align256(o + 4ull * g.NX * g.ntiles);
  l.lpx = o;
  o = align256(o + 4ull * cap);
  l.x = o;
  o = align256(o + 4ull * cap);
  l.alpha = o;
  o = align256(o + 4ull * cap * g.C);
  l.rgb = o;
  o = align256(o + 12ull * cap);
  l.idx = o;
  o = align256(o + 4ull * cap);
  l.total = o;
  l.cap = cap;
  return l;
}

uint64_t capacity_for(const Geom& g, size_t ws_bytes) {
  const size_t fixed = make_layout(g, 0).total;
  if (ws_bytes < fixed) return 0;
  const uint64_t per = 4 + 4 + 4ull * g.C + 12 + 4;
  uint64_t cap = (ws_bytes - fixed) / per;
  while (cap > 0 && make_layout(g, cap).total > ws_bytes) --cap;
  return cap;
}

Binned binned_view(const Geom& g, const Layout& l, const void* ws) {
  const char* b = (const char*)ws;
  Binned v;
  v.offsets = (const uint32_t*)(b + l.offsets);
  v.lpx = (const uint32_t*)(b + l.lpx);
  v.x = (const float*)(b + l.x);
  v.alpha = (const float*)(b + l.alpha);
  v.rgb = (const float*)(b + l.rgb);
  v.idx = (const uint32_t*)(b + l.idx);
  v.cap = l.cap;
  (void)g;
  return v;
}

struct BinOut {
  uint32_t* lpx;
  float* x;
  float* alpha;
  float* rgb;
  uint32_t* idx;  // nullptr: stream index not recorded
  uint64_t cap;
};

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_hist_lds(const uint32_t* __restrict__ pixel, uint32_t F, Geom g,
                                                  uint32_t* __restrict__ counts,
                                                  unsigned long long* __restrict__ dropped) {
  extern __shared__ uint32_t lh[];
  for (uint32_t t = threadIdx.x; t < g.ntiles; t += blockDim.x) lh[t] = 0;
  __syncthreads();
  const uint32_t cls = blockIdx.x % g.NX;
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + kChunk - 1) / kChunk);
  uint32_t nd = 0;
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint64_t base = (uint64_t)c * kChunk;
    const uint64_t end = std::min<uint64_t>(base + kChunk, F);
    for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
      const uint32_t p = pixel[i];
      if (p < g.P)
        atomicAdd(&lh[tile_of(g, p)], 1u);
      else
        ++nd;
    }
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < g.ntiles; t += blockDim.x) {
    const uint32_t v = lh[t];
    if (v) atomicAdd(&counts[cls * g.ntiles + t], v);
  }
  nd = wave_sum(nd);
  if ((threadIdx.x & 63) == 0 && nd) atomicAdd(dropped, (unsigned long long)nd);
}

// Fallback for very many tiles (large ranks on large frames): one global atomic per fragment, one class.
__global__ __launch_bounds__(256) void k_hist_global(const uint32_t* __restrict__ pixel, uint32_t F, Geom g,
                                                     uint32_t* __restrict__ counts,
                                                     unsigned long long* __restrict__ dropped) {
  uint32_t nd = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < F; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = pixel[i];
    if (p < g.P)
      atomicAdd(&counts[tile_of(g, p)], 1u);
    else
      ++nd;
  }
  nd = wave_sum(nd);
  if ((threadIdx.x & 63) == 0 && nd) atomicAdd(dropped, (unsigned long long)nd);
}

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 16;

// Exclusive scan over segments in (tile, class) order. counts/cursors are class-major [NX][ntiles].
__global__ __launch_bounds__(kScanThreads) void k_scan(const uint32_t* __restrict__ counts, Geom g,
                                                       uint32_t* __restrict__ offsets,
                                                       uint32_t* __restrict__ cursors) {
  __shared__ uint32_t sums[kScanThreads];
  const uint64_t n = (uint64_t)g.ntiles * g.NX;
  const uint32_t tid = threadIdx.x;
  uint32_t carry = 0;
  for (uint64_t seg = 0; seg < n; seg += (uint64_t)kScanThreads * kScanItems) {
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const uint64_t e = seg + (uint64_t)tid * kScanItems + k;
      v[k] = 0;
      if (e < n) {
        const uint32_t t = (uint32_t)(e / g.NX), x = (uint32_t)(e % g.NX);
        v[k] = counts[x * g.ntiles + t];
      }
      s += v[k];
    }
    sums[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const uint32_t add = tid >= (uint32_t)off ? sums[tid - off] : 0;
      __syncthreads();
      sums[tid] += add;
      __syncthreads();
    }
    uint32_t run = carry + (tid ? sums[tid - 1] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const uint64_t e = seg + (uint64_t)tid * kScanItems + k;
      if (e < n) {
        const uint32_t t = (uint32_t)(e / g.NX), x = (uint32_t)(e % g.NX);
        offsets[e] = run;
        cursors[x * g.ntiles + t] = run;
      }
      run += v[k];
    }
    carry += sums[kScanThreads - 1];
    __syncthreads();
  }
  if (tid == 0) offsets[n] = carry;
}

__device__ __forceinline__ void put_fragment(const wt_fragments& f, const Geom& g, const BinOut& o, uint64_t i,
                                             uint32_t pos, uint32_t local, uint32_t& nan_count) {
  const float d = f.depth[i];
  bool bad = isnan(d);
  o.lpx[pos] = local;
  o.x[pos] = d;
  for (uint32_t c = 0; c < g.C; ++c) {
    const float a = f.alpha[i * g.C + c];
    bad |= isnan(a);
    o.alpha[c * o.cap + pos] = a;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) o.rgb[q * o.cap + pos] = f.rgb[i * 3 + q];
  if (o.idx) o.idx[pos] = (uint32_t)i;
  nan_count += bad ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_scatter_lds(wt_fragments f, Geom g, uint32_t* __restrict__ cursors, BinOut o,
                                                     unsigned long long* __restrict__ dropped) {
  extern __shared__ uint32_t lh[];
  const uint32_t F = (uint32_t)f.count;
  const uint32_t cls = blockIdx.x % g.NX;
  const uint64_t base = (uint64_t)blockIdx.x * kChunk;
  const uint64_t end = std::min<uint64_t>(base + kChunk, F);
  for (uint32_t t = threadIdx.x; t < g.ntiles; t += blockDim.x) lh[t] = 0;
  __syncthreads();
  for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
    const uint32_t p = f.pixel[i];
    if (p < g.P) atomicAdd(&lh[tile_of(g, p)], 1u);
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < g.ntiles; t += blockDim.x) {
    const uint32_t v = lh[t];
    if (v) lh[t] = atomicAdd(&cursors[cls * g.ntiles + t], v);
  }
  __syncthreads();
  uint32_t nan_count = 0;
  for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
    const uint32_t p = f.pixel[i];
    if (p >= g.P) continue;
    uint32_t tile, local;
    tile_locate(g, p, tile, local);
    const uint32_t pos = atomicAdd(&lh[tile], 1u);
    put_fragment(f, g, o, i, pos, local, nan_count);
  }
  nan_count = wave_sum(nan_count);
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(dropped, (unsigned long long)nan_count);
}

__global__ __launch_bounds__(256) void k_scatter_global(wt_fragments f, Geom g, uint32_t* __restrict__ cursors,
                                                        BinOut o, unsigned long long* __restrict__ dropped) {
  uint32_t nan_count = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < f.count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = f.pixel[i];
    if (p >= g.P) continue;
    uint32_t tile, local;
    tile_locate(g, p, tile, local);
    const uint32_t pos = atomicAdd(&cursors[tile], 1u);
    put_fragment(f, g, o, i, pos, local, nan_count);
  }
  nan_count = wave_sum(nan_count);
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(dropped, (unsigned long long)nan_count);
}

hipError_t launch_bin(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                      hipStream_t s) {
  char* b = (char*)ws;
  uint32_t* counts = (uint32_t*)(b + l.counts);
  uint32_t* offsets = (uint32_t*)(b + l.offsets);
  uint32_t* cursors = (uint32_t*)(b + l.cursors);
  unsigned long long* dropped = (unsigned long long*)(b + l.header);
  const uint64_t ncount = (uint64_t)g.NX * g.ntiles;
  // zero the header's counters and the tile counts (fill kernels: safe inside captured graphs)
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)(b + l.header), (uint64_t)4, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((ncount + 255) / 256, 4096)), dim3(256), 0, s,
                     counts, ncount, 0u);
  const uint32_t F = (uint32_t)f.count;
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + kChunk - 1) / kChunk);
  if (F > 0) {
    if (g.lds_bins) {
      const uint32_t grid = std::min<uint32_t>(((nchunks + g.NX - 1) / g.NX) * g.NX, 2048);
      hipLaunchKernelGGL(k_hist_lds, dim3(grid), dim3(256), g.ntiles * 4, s, f.pixel, F, g, counts, dropped);
    } else {
      hipLaunchKernelGGL(k_hist_global, dim3(2048), dim3(256), 0, s, f.pixel, F, g, counts, dropped);
    }
  }
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts, g, offsets, cursors);
  if (F > 0) {
    BinOut o;
    o.lpx = (uint32_t*)(b + l.lpx);
    o.x = (float*)(b + l.x);
    o.alpha = (float*)(b + l.alpha);
    o.rgb = (float*)(b + l.rgb);
    o.idx = record_index ? (uint32_t*)(b + l.idx) : nullptr;
    o.cap = l.cap;
    if (g.lds_bins)
      hipLaunchKernelGGL(k_scatter_lds, dim3(nchunks), dim3(256), g.ntiles * 4, s, f, g, cursors, o, dropped);
    else
      hipLaunchKernelGGL(k_scatter_global, dim3(4096), dim3(256), 0, s, f, g, cursors, o, dropped);
  }
  return hipGetLastError();
}

}  // namespace wt
