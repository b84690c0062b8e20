// Ingest and screen-tile binning of an unordered fragment stream.
//
// The paper builds and evaluates inside a raster pipeline, where the fragments of one screen region arrive on
// the same shader core (section 2.1). A stored stream carries no such locality, and on this GPU per-fragment
// random atomics into a frame-sized coefficient buffer run at a few billion fragments per second. So the
// stream is first regrouped by screen tile with a counting sort (histogram, scan, scatter), after which every
// per-pixel update of the build and evaluate passes happens in the LDS of the compute unit that owns the tile.
//
// Kernels:
//   k_hist_lds        pixel ids (4 B/fragment) -> per-(class, tile) counts in an LDS table (in passes of tile
//                     ranges for very large frames); range drops counted.
//   k_scan            exclusive scan of the counts, tile-major over (tile, class), into segment offsets and write
//                     cursors; tile order for the tile kernels (heaviest first).
//   k_scatter_staged  one chunk (4 or 8 fragments per thread) per workgroup: vector loads into registers, LDS
//                     rank per tile, records placed in LDS in tile order in rounds, one cursor reservation per tile
//                     present in a round just before the round is written record by record with consecutive lanes
//                     on consecutive records (head array, then tail array), so each tile's run is written
//                     coalesced.
//   Frames with more than kTwoLevelTiles tiles: a chunk would touch most tiles about once, so the stream is
//   binned into super-tiles of SW x SH tiles first (k_super_counts, k_scan and k_scatter_staged over the
//   super-tile geometry), then k_split moves each super-tile's records into its tiles without atomics.
//   k_hist_global,    one global atomic per fragment (beyond kMaxLdsBins super-tiles).
//   k_scatter_global
// A chunk's class is chunk % NX in both the histogram and the scatter; with one chunk per scatter workgroup the
// class is also the XCD the workgroup runs on, so each (bin, class) run is written from a single L2.
// NaN fragments are counted as dropped and still binned; the tile kernels skip them.

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
  g.AL = (d.channels == 3) ? 6 : 4;
  g.dtype = d.coeff_dtype;
  // Largest power-of-two tile whose LDS working set fits one compute unit. Forward: FP64 endpoint masses
  // (M + 1 per channel) and three FP64 colour sums, or, where the tile would hold more pixel/channels than a
  // workgroup has threads or M > 32, FP64 coefficient sums plus FP64 accumulations. Backward: FP32 cells,
  // FP64 cell adjoints and per-pixel gradient data.
  auto tile_for = [](uint32_t per_px) {
    const uint32_t px = std::max<uint32_t>(1, kLdsBytes / per_px);
    return std::min<uint32_t>(floor_pow2(px), kMaxTilePx);
  };
  uint32_t px;
  g.ep = 0;
  g.tight = (d.flags & WT_TIGHT_DEPTH) ? 1 : 0;
  g.serial = (d.flags & WT_DETERMINISTIC) ? 1 : 0;
  const uint32_t bpx = g.tight ? 8 : 0;  // per-pixel depth bounds (two FP32) in LDS
  if (backward) {
    px = tile_for(12 * g.C * g.M + 4 * (3 + g.C) + bpx);
  } else if (d.flags & WT_TEMPORAL) {
    // one-pass render: endpoint masses, colour sums and the previous frame's FP32 cells (M <= 32 and no depth
    // bounds are checked by the API); every pixel/channel has a thread
    g.temporal = 1;
    px = std::min<uint32_t>(tile_for(8 * g.C * (g.M + 1) + 24 + 4 * g.C * g.M), floor_pow2(kTileThreads / g.C));
    g.ep = 1;
  } else {
    px = tile_for(8 * g.C * (g.M + 1) + 24 + bpx);
    // packed three-channel storage is converted on the endpoint path only: cap the tile so that every
    // pixel/channel has a thread (rank <= 4 is checked by the API)
    if (d.coeff_dtype == WT_E5B9G9R9) px = std::min<uint32_t>(px, floor_pow2(kTileThreads / g.C));
    if (g.M <= 32 && px * g.C <= kTileThreads) {
      g.ep = 1;
    } else {
      px = tile_for(8 * (g.C * g.M + g.AL) + bpx);
    }
  }
  uint32_t e = 0;
  while ((1u << e) < px) ++e;
  g.lTW = (e + 1) / 2;
  g.lTH = e / 2;
  g.TW = 1u << g.lTW;
  g.TH = 1u << g.lTH;
  g.divW = make_fastdiv(g.W);
  g.tile_px = g.TW * g.TH;
  g.tilesX = (g.W + g.TW - 1) / g.TW;
  g.tilesY = (g.H + g.TH - 1) / g.TH;
  g.ntiles = g.tilesX * g.tilesY;
  // One LDS tile table for the scatter (up to kTwoLevelTiles tiles; beyond, two levels below)
  g.lds_bins = g.ntiles <= kTwoLevelTiles ? 1 : 0;
  g.rb = g.ntiles;
  const uint32_t hnr = (g.ntiles + kMaxHistBins - 1) / kMaxHistBins;
  g.hrb = (g.ntiles + hnr - 1) / hnr;
  // Many tiles: a chunk of the stream touches each tile about chunk / ntiles times, too few for whole runs. Bin
  // into at most kMaxSupers super-tiles of SW x SH tiles first (runs as long as for a small frame), then split
  // each super-tile's records into its tiles (runs of hundreds of records, no atomics).
  g.two = 0;
  g.SW = g.SH = 1;
  if (g.ntiles > kTwoLevelTiles) {
    auto supers = [&](uint32_t sw, uint32_t sh) {
      return ((g.tilesX + sw - 1) / sw) * ((g.tilesY + sh - 1) / sh);
    };
    while (supers(g.SW, g.SH) > kMaxSupers && g.SW * g.SH < kMaxSub) {
      if (g.SW <= g.SH) g.SW *= 2;
      else g.SH *= 2;
    }
    // super-tile tables must fit the scatter's LDS; beyond that (about half a million tiles) the stream is
    // binned with one global atomic per fragment
    g.two = supers(g.SW, g.SH) <= kMaxLdsBins ? 1 : 0;
    g.lds_bins = g.two;
  }
  g.lSW = 0;
  while ((1u << g.lSW) < g.SW) ++g.lSW;
  g.lSH = 0;
  while ((1u << g.lSH) < g.SH) ++g.lSH;
  g.sX = (g.tilesX + g.SW - 1) / g.SW;
  g.sY = (g.tilesY + g.SH - 1) / g.SH;
  g.nsuper = g.sX * g.sY;
  g.NX = g.lds_bins ? kClasses : 1;
  // Scatter: two workgroups per compute unit where the tile tables (of the binning level that scatters) and a
  // 1024-record round fit half the LDS and a 4096-fragment chunk still holds two records per bin on average, so
  // that one workgroup's loads overlap the other's ranking, staging and writes: one channel, 1024 threads with 4
  // fragments each (64 registers, eight waves per SIMD); three channels, 512 threads with 8 fragments each (the
  // three-channel fragment needs about 110 registers: four waves per SIMD). Otherwise one workgroup of 1024 threads
  // with 8 fragments each per compute unit. Chunks are powers of two.
  // (Glass 3840x2160: the three-channel form took the scatter phases from 7.86 to 7.22 ms. Smoke frame at rank 4,
  // 4,080 tiles: one workgroup per compute unit, two records per bin and chunk, 2.10 -> 2.07 ms.)
  // (a one-channel record stages in at most 32 bytes, index or not, a three-channel one in at most 40: 1024 of
  // them take 32 or 40 KB)
  g.sthreads = 1024;
  g.kper = kPer;
  const uint32_t bins = g.two ? g.nsuper : g.rb;
  const bool two_wg = g.lds_bins && bins <= 2048 &&
                      8ull * bins + 1024ull * (g.C == 1 ? 32 : 40) <= kLdsBytes / 2 - 1024;
  if (two_wg && g.C == 1) g.kper = 4;
  if (two_wg && g.C == 3) g.sthreads = 512;
  g.chunk = g.sthreads * g.kper;
  return g;
}

Geom super_geom(const Geom& g) {
  Geom s = g;
  s.lTW = g.lTW + g.lSW;
  s.lTH = g.lTH + g.lSH;
  s.TW = 1u << s.lTW;
  s.TH = 1u << s.lTH;
  s.tile_px = s.TW * s.TH;
  s.tilesX = g.sX;
  s.tilesY = g.sY;
  s.ntiles = g.nsuper;
  s.rb = s.hrb = g.nsuper;
  s.two = 0;
  s.SW = s.SH = 1;
  s.lSW = s.lSH = 0;
  s.sX = s.tilesX;
  s.sY = s.tilesY;
  return s;  // NX, kper and chunk stay those of g: the first level uses the classes the histogram counted
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
  o = align256(o + 4ull * g.NX * g.ntiles * kCursorPad);
  l.order = o;
  o = align256(o + 4ull * g.ntiles);
  l.scan = o;
  o = align256(o + 4ull * 257 * ((g.NX * (uint64_t)g.ntiles + kScanRange - 1) / kScanRange));
  l.heads = o;
  o = align256(o + 4ull * head_dwords(g.C) * cap);
  l.tails = o;
  o = align256(o + 4ull * tail_dwords(true) * cap);
  l.counts1 = l.offsets1 = l.cursors1 = l.order1 = l.heads1 = l.tails1 = o;
  if (g.two) {
    l.counts1 = o;
    o = align256(o + 4ull * g.NX * g.nsuper);
    l.offsets1 = o;
    o = align256(o + 4ull * (g.NX * (uint64_t)g.nsuper + 1));
    l.cursors1 = o;
    o = align256(o + 4ull * g.NX * g.nsuper * kCursorPad);
    l.order1 = o;
    o = align256(o + 4ull * g.nsuper);
    l.heads1 = o;
    o = align256(o + 4ull * head_dwords(g.C) * cap);
    l.tails1 = o;
    o = align256(o + 4ull * tail_dwords(true) * cap);
  }
  l.total = o;
  l.cap = cap;
  return l;
}

uint64_t capacity_for(const Geom& g, size_t ws_bytes) {
  const size_t fixed = make_layout(g, 0).total;
  if (ws_bytes < fixed) return 0;
  const uint64_t per = 4ull * record_dwords(g.C, true) * (g.two ? 2 : 1);
  uint64_t cap = (ws_bytes - fixed) / per;
  while (cap > 0 && make_layout(g, cap).total > ws_bytes) --cap;
  return cap;
}

Binned binned_view(const Geom& g, const Layout& l, const void* ws, bool with_index) {
  const char* b = (const char*)ws;
  Binned v;
  v.offsets = (const uint32_t*)(b + l.offsets);
  v.order = (const uint32_t*)(b + l.order);
  v.head = (const uint32_t*)(b + l.heads);
  v.tail = (const uint32_t*)(b + l.tails);
  v.DH = head_dwords(g.C);
  v.DT = tail_dwords(with_index);
  v.hdr = (WsHeader*)(b + l.header);
  v.stamp = layout_stamp(g, l, with_index);
  v.cap = l.cap;
  return v;
}

// The stamp covers everything the tile kernels index by: frame, channels, rank, tile and super-tile geometry, write
// classes, record capacity and format, and the layout's size.
unsigned long long layout_stamp(const Geom& g, const Layout& l, bool with_index) {
  const uint32_t w[] = {0x57544c31u, g.W, g.H, g.C, g.rank, g.TW, g.TH, g.NX, g.two, g.SW, g.SH, g.lds_bins, g.serial,
                        (uint32_t)l.cap, (uint32_t)(l.cap >> 32), (uint32_t)l.total, (uint32_t)(l.total >> 32),
                        with_index ? 1u : 0u};
  return stamp_words(w, (int)(sizeof w / sizeof w[0]));
}

// A count is stamped with the layout and the stream it counted (size and the four array addresses), so that a
// scatter of another stream, or under another layout, refuses to write.
unsigned long long count_stamp(const Geom& g, const Layout& l, const wt_fragments& f) {
  const unsigned long long ls = layout_stamp(g, l, false);
  const uintptr_t a[4] = {(uintptr_t)f.pixel, (uintptr_t)f.depth, (uintptr_t)f.alpha, (uintptr_t)f.rgb};
  uint32_t w[12] = {(uint32_t)ls, (uint32_t)(ls >> 32), (uint32_t)f.count, (uint32_t)(f.count >> 32)};
  for (int i = 0; i < 4; ++i) {
    w[4 + 2 * i] = (uint32_t)a[i];
    w[5 + 2 * i] = (uint32_t)((uint64_t)a[i] >> 32);
  }
  return stamp_words(w, 12);
}

// Start of a count: no complete binning and no count in the workspace any more; the drop counter and the scatter
// fault restart. The sticky error bits stay until wt_dropped_count reports them.
__global__ void k_header_reset(WsHeader* h) {
  if (h->magic != kWsMagic) {  // a workspace the device has not written yet: no errors to keep
    h->errors = 0;
    h->magic = kWsMagic;
  }
  h->dropped = 0;
  h->fault = 0;
  h->counted = 0;
  h->binned = 0;
}

// End of a scatter: the binning is complete when the count before it was this stream's under this layout, the
// scatter did not refuse, and every write cursor reached the end of its segment (so each segment holds exactly the
// records counted for it). Then the header gets `stamp`, else 0.
// One workgroup. cursors are [NX][nt] (row stride kCursorPad words), offsets [nt * NX + 1].
__global__ __launch_bounds__(1024) void k_seal(WsHeader* h, const uint32_t* __restrict__ cursors,
                                                const uint32_t* __restrict__ offsets, uint32_t NX, uint32_t nt,
                                                unsigned long long cstamp, unsigned long long stamp) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  for (uint32_t e = threadIdx.x; e < NX * nt; e += blockDim.x) {
    const uint32_t x = e / nt, t = e - x * nt;
    mine |= cursors[(size_t)e * kCursorPad] != offsets[t * NX + x + 1];
  }
  if (mine) bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool ok = !bad && h->fault == 0 && h->counted == cstamp;
    h->binned = ok ? stamp : 0ull;
    // a scatter that did not belong to its count (another stream, arrays changed since the count, run twice)
    if (!ok) ws_raise(h, kWsErrScatter);
  }
}

// After the split of a two-level binning: complete when the first level was (the split only moves its records).
__global__ void k_seal_split(WsHeader* h, unsigned long long level1, unsigned long long stamp) {
  h->binned = h->binned == level1 ? stamp : 0ull;
}

// A first-level binning of a two-level layout carries this stamp until its split has run.
static unsigned long long level1_stamp(unsigned long long s) { return s ^ 0x9e3779b97f4a7c15ull; }

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Streaming 16-byte loads (non-temporal: each fragment is read once), defined with the scatter below.
template <bool NT>
__device__ __forceinline__ uint4 load_stream_u4(const uint32_t* p);

// ------------------------------------------------------------------------------------------------ histogram

// Workgroups of 256 threads, or of 1024 when the tile table is large (up to 144 KB of LDS leaves one workgroup per
// compute unit, which then still has sixteen waves of loads in flight). The pixel ids are read with non-temporal
// loads (smoke frame: 0.132 -> 0.121 ms for the count).

template <int kHistThreads>
__global__ __launch_bounds__(kHistThreads) void k_hist_lds(const uint32_t* __restrict__ pixel, uint32_t F, Geom g,
                                                           int vec, uint32_t* __restrict__ counts,
                                                           unsigned long long* __restrict__ dropped) {
  extern __shared__ uint32_t lh[];
  const uint32_t cls = blockIdx.x % g.NX;
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + g.chunk - 1) / g.chunk);
  uint32_t nd = 0;
  // one pass per range of g.hrb tiles (a single pass unless the frame has more tiles than the table holds)
  for (uint32_t t0 = 0; t0 < g.ntiles; t0 += g.hrb) {
  const uint32_t nt = std::min(g.hrb, g.ntiles - t0);
  const bool first = t0 == 0;
  for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) lh[t] = 0;
  __syncthreads();
  // The workgroup's whole chunks (chunk k of the workgroup is c = blockIdx.x + k gridDim.x, all of its class) as one
  // flat range of 16-byte units, so that every thread has four loads in flight whatever the chunk size; chunk sizes
  // are powers of two (threads per scatter workgroup times fragments per thread).
  const uint32_t nfull = vec ? F / g.chunk : 0;
  const uint32_t kfull = blockIdx.x < nfull ? (nfull - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const uint32_t nv = g.chunk / 4, lnv = __builtin_ctz(nv);
  const uint32_t units = kfull * nv;
  for (uint32_t u0 = 0; u0 < units; u0 += 4 * kHistThreads) {
    uint4 q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t u = u0 + v * kHistThreads + threadIdx.x;
      const uint32_t c = blockIdx.x + (u >> lnv) * gridDim.x;
      q[v] = u < units ? load_stream_u4<true>(pixel + (uint64_t)c * g.chunk + 4 * (u & (nv - 1)))
                       : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (u0 + v * kHistThreads + threadIdx.x >= units) continue;
      const uint32_t ps[4] = {q[v].x, q[v].y, q[v].z, q[v].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (ps[k] < g.P) {
          const uint32_t t = tile_of(g, ps[k]) - t0;
          if (t < nt) atomicAdd(&lh[t], 1u);
        } else if (first) {
          ++nd;
        }
      }
    }
  }
  // the rest: the partial last chunk, or every chunk of an unaligned stream
  for (uint32_t c = blockIdx.x + kfull * gridDim.x; c < nchunks; c += gridDim.x) {
    const uint32_t base = c * g.chunk;
    const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t p = pixel[base + i];
      if (p < g.P) {
        const uint32_t t = tile_of(g, p) - t0;
        if (t < nt) atomicAdd(&lh[t], 1u);
      } else if (first) {
        ++nd;
      }
    }
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) {
    const uint32_t v = lh[t];
    if (v) atomicAdd(&counts[cls * g.ntiles + t0 + t], v);
  }
  __syncthreads();
  }
  nd = wave_sum(nd);
  if ((threadIdx.x & 63) == 0 && nd) atomicAdd(dropped, (unsigned long long)nd);
}

// Fallback for very many tiles: one global atomic per fragment, one class.
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

// ------------------------------------------------------------------------------------------------ scan

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 16;
constexpr uint32_t kOrderBuckets = 256;  // size classes of the heaviest-first tile order
static_assert(kScanRange == (uint32_t)kScanThreads * kScanItems, "a scan workgroup covers one pass of k_scan");
static_assert(kScanRange % kClasses == 0, "scan ranges hold whole tiles");

// Exclusive prefix of s over the workgroup (wavefront shuffles, then the wave totals); *total receives the sum.
// wsum holds kScanThreads / 64 + 1 entries. Ends with a barrier.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t s, uint32_t* wsum, uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += v;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  if (wv == 0) {
    constexpr uint32_t NW = kScanThreads / 64;
    const uint32_t w = lane < NW ? wsum[lane] : 0u;
    uint32_t wi = w;
#pragma unroll
    for (int o = 1; o < (int)NW; o <<= 1) {
      const uint32_t v = __shfl_up(wi, o, 64);
      if (lane >= (uint32_t)o) wi += v;
    }
    if (lane < NW) wsum[lane] = wi - w;
    if (lane == NW - 1) wsum[NW] = wi;
  }
  __syncthreads();
  *total = wsum[kScanThreads / 64];
  const uint32_t r = wsum[wv] + inc - s;
  __syncthreads();  // wsum may be reused
  return r;
}

// Size class of a tile for the heaviest-first order: log-linear in the count (the leading bit's position and the
// three bits below it), monotone, 256 classes.
__device__ __forceinline__ uint32_t size_class(uint32_t c) {
  const uint32_t v = c + 1;
  const uint32_t e = 31 - __clz(v);
  const uint32_t m = e >= 3 ? (v >> (e - 3)) & 7u : (v << (3 - e)) & 7u;
  return e * 8 + m;
}

// Exclusive scan over segments in (tile, class) order (counts/cursors are class-major [NX][ntiles]), then the
// tile order for the tile kernels: heaviest first by size class (a bucket sort; ties in any order), so the last
// workgroups to start are the light ones.
__global__ __launch_bounds__(kScanThreads) void k_scan(const uint32_t* __restrict__ counts, Geom g,
                                                       uint32_t* __restrict__ offsets,
                                                       uint32_t* __restrict__ cursors,
                                                       uint32_t* __restrict__ order, int with_order,
                                                       WsHeader* hdr, unsigned long long stamp) {
  if (hdr && threadIdx.x == 0) hdr->counted = stamp;  // the last scan of a count (seen by later kernels)
  __shared__ uint32_t wsum[kScanThreads / 64 + 1];
  __shared__ uint32_t bucket[kOrderBuckets];
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
    uint32_t total;
    uint32_t run = carry + block_exclusive(s, wsum, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const uint64_t e = seg + (uint64_t)tid * kScanItems + k;
      if (e < n) {
        const uint32_t t = (uint32_t)(e / g.NX), x = (uint32_t)(e % g.NX);
        offsets[e] = run;
        cursors[(x * g.ntiles + t) * kCursorPad] = run;
      }
      run += v[k];
    }
    carry += total;
  }
  if (tid == 0) offsets[n] = carry;
  if (!with_order) return;
  // bucket sort by size class, largest class first
  for (uint32_t b = tid; b < kOrderBuckets; b += kScanThreads) bucket[b] = 0;
  __syncthreads();
  for (uint32_t t = tid; t < g.ntiles; t += kScanThreads) {
    uint32_t c = 0;
    for (uint32_t x = 0; x < g.NX; ++x) c += counts[x * g.ntiles + t];
    atomicAdd(&bucket[kOrderBuckets - 1 - size_class(c)], 1u);
  }
  __syncthreads();
  uint32_t total;
  const uint32_t bc = tid < kOrderBuckets ? bucket[tid] : 0u;
  const uint32_t start = block_exclusive(bc, wsum, &total);
  if (tid < kOrderBuckets) bucket[tid] = start;
  __syncthreads();
  for (uint32_t t = tid; t < g.ntiles; t += kScanThreads) {
    uint32_t c = 0;
    for (uint32_t x = 0; x < g.NX; ++x) c += counts[x * g.ntiles + t];
    order[atomicAdd(&bucket[kOrderBuckets - 1 - size_class(c)], 1u)] = t;
  }
}

// The same scan and tile order for frames with many segments, over several workgroups: workgroup w owns the
// segments [w R, (w + 1) R) (R = kScanRange, whole tiles since R is a multiple of NX). Pass one: each workgroup's
// segment total and the size classes of its tiles (part[w][0], part[w][1 + k] for reversed class k). Pass two:
// each workgroup adds the totals of the workgroups before it, scans its range, and places its tiles in the
// heaviest-first order after every heavier class and after its class's tiles of earlier workgroups.
__global__ __launch_bounds__(kScanThreads) void k_scan_part(const uint32_t* __restrict__ counts, Geom g,
                                                            uint32_t* __restrict__ part) {
  __shared__ uint32_t wsum[kScanThreads / 64 + 1];
  __shared__ uint32_t bucket[kOrderBuckets];
  const uint64_t n = (uint64_t)g.ntiles * g.NX;
  const uint64_t e0 = (uint64_t)blockIdx.x * kScanRange;
  const uint32_t tid = threadIdx.x;
  for (uint32_t b = tid; b < kOrderBuckets; b += kScanThreads) bucket[b] = 0;
  uint32_t s = 0;
  for (uint32_t k = tid; k < kScanRange; k += kScanThreads) {
    const uint64_t e = e0 + k;
    if (e < n) {
      const uint32_t t = (uint32_t)(e / g.NX), x = (uint32_t)(e % g.NX);
      s += counts[x * g.ntiles + t];
    }
  }
  uint32_t total;
  block_exclusive(s, wsum, &total);
  __syncthreads();
  const uint32_t t0 = (uint32_t)(e0 / g.NX), t1 = (uint32_t)std::min<uint64_t>((e0 + kScanRange) / g.NX, g.ntiles);
  for (uint32_t t = t0 + tid; t < t1; t += kScanThreads) {
    uint32_t c = 0;
    for (uint32_t x = 0; x < g.NX; ++x) c += counts[x * g.ntiles + t];
    atomicAdd(&bucket[kOrderBuckets - 1 - size_class(c)], 1u);
  }
  __syncthreads();
  uint32_t* mine = part + (size_t)blockIdx.x * (1 + kOrderBuckets);
  if (tid == 0) mine[0] = total;
  for (uint32_t b = tid; b < kOrderBuckets; b += kScanThreads) mine[1 + b] = bucket[b];
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t* __restrict__ counts, Geom g,
                                                             const uint32_t* __restrict__ part,
                                                             uint32_t* __restrict__ offsets,
                                                             uint32_t* __restrict__ cursors,
                                                             uint32_t* __restrict__ order, int with_order,
                                                             WsHeader* hdr, unsigned long long stamp) {
  __shared__ uint32_t wsum[kScanThreads / 64 + 1];
  __shared__ uint32_t start[kOrderBuckets];
  const uint64_t n = (uint64_t)g.ntiles * g.NX;
  const uint32_t G = gridDim.x, w = blockIdx.x, tid = threadIdx.x;
  const uint64_t e0 = (uint64_t)w * kScanRange;
  if (hdr && w == 0 && tid == 0) hdr->counted = stamp;
  // segments of the workgroups before this one
  uint32_t c = 0;
  for (uint32_t v = tid; v < w; v += kScanThreads) c += part[(size_t)v * (1 + kOrderBuckets)];
  uint32_t carry;
  block_exclusive(c, wsum, &carry);
  // this range's segments, kScanItems consecutive per thread
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t e = e0 + (uint64_t)tid * kScanItems + k;
    v[k] = 0;
    if (e < n) v[k] = counts[(uint32_t)(e % g.NX) * g.ntiles + (uint32_t)(e / g.NX)];
    s += v[k];
  }
  uint32_t total;
  uint32_t run = carry + block_exclusive(s, wsum, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t e = e0 + (uint64_t)tid * kScanItems + k;
    if (e < n) {
      const uint32_t t = (uint32_t)(e / g.NX), x = (uint32_t)(e % g.NX);
      offsets[e] = run;
      cursors[(x * g.ntiles + t) * kCursorPad] = run;
    }
    run += v[k];
  }
  if (w == G - 1 && tid == 0) offsets[n] = carry + total;
  if (!with_order) return;
  // start of this workgroup's tiles in each size class: all heavier classes, then earlier workgroups' tiles of
  // the same class
  uint32_t tot = 0, pre = 0;
  if (tid < kOrderBuckets) {
    for (uint32_t u = 0; u < G; ++u) {
      const uint32_t b = part[(size_t)u * (1 + kOrderBuckets) + 1 + tid];
      tot += b;
      if (u < w) pre += b;
    }
  }
  uint32_t all;
  const uint32_t base = block_exclusive(tid < kOrderBuckets ? tot : 0u, wsum, &all);
  if (tid < kOrderBuckets) start[tid] = base + pre;
  __syncthreads();
  const uint32_t t0 = (uint32_t)(e0 / g.NX), t1 = (uint32_t)std::min<uint64_t>((e0 + kScanRange) / g.NX, g.ntiles);
  for (uint32_t t = t0 + tid; t < t1; t += kScanThreads) {
    uint32_t cnt = 0;
    for (uint32_t x = 0; x < g.NX; ++x) cnt += counts[x * g.ntiles + t];
    order[atomicAdd(&start[kOrderBuckets - 1 - size_class(cnt)], 1u)] = t;
  }
}

// Per-class counts of the super-tiles (first level of two-level binning) from the per-class tile counts.
__global__ __launch_bounds__(256) void k_super_counts(const uint32_t* __restrict__ counts, Geom g,
                                                      uint32_t* __restrict__ counts1) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.NX * g.nsuper) return;
  const uint32_t x = id / g.nsuper, sidx = id - x * g.nsuper;
  const uint32_t sx = sidx % g.sX, sy = sidx / g.sX;
  uint32_t sum = 0;
  for (uint32_t j = 0; j < g.SW * g.SH; ++j) {
    const uint32_t tx = (sx << g.lSW) + (j & (g.SW - 1)), ty = (sy << g.lSH) + (j >> g.lSW);
    if (tx < g.tilesX && ty < g.tilesY) sum += counts[x * g.ntiles + ty * g.tilesX + tx];
  }
  counts1[id] = sum;
}

// ------------------------------------------------------------------------------------------------ scatter


// The fragment stream is read once. With two scatter workgroups per compute unit (PER = 4), non-temporal loads
// keep it from evicting the partly written record lines that the L2 is completing (measured on the smoke frame:
// 17% less HBM write traffic, scatter 1.96 -> 1.68 ms); with one workgroup per compute unit (PER = 8) they
// made the scatter slower (2.05 -> 2.41 ms), so there the loads stay ordinary.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 load_stream_u4(const uint32_t* p) {
  if constexpr (NT) {
    const u32x4_t v = __builtin_nontemporal_load((const u32x4_t*)p);
    return make_uint4(v.x, v.y, v.z, v.w);
  } else {
    return *(const uint4*)p;
  }
}
template <bool NT>
__device__ __forceinline__ float4 load_stream_f4(const float* p) {
  if constexpr (NT) {
    const u32x4_t v = __builtin_nontemporal_load((const u32x4_t*)p);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
  } else {
    return *(const float4*)p;
  }
}

// One chunk's fragments, held in registers by the thread that loaded them.
template <int C, int PER>
struct ChunkRegs {
  static_assert(PER % 4 == 0, "vector loads take fragments four at a time");
  uint32_t p[PER];
  float x[PER];
  float a[C * PER];
  float c[3 * PER];
};

// Loads fragments [i0, i0 + PER) of the chunk at base; out-of-range slots get pixel id 0xffffffff.
template <int C, int PER>
__device__ __forceinline__ void load_chunk(const wt_fragments& f, uint32_t base, uint32_t i0, uint32_t n, int vec,
                                           ChunkRegs<C, PER>& r) {
  constexpr uint32_t kPer = PER;
  if (vec && i0 + kPer <= n) {
    // pixel ids first: the tile count needs only them, and the other loads stay in flight meanwhile
#pragma unroll
    for (uint32_t v = 0; v < kPer / 4; ++v) {
      const uint4 p4 = load_stream_u4<PER == 4>(f.pixel + (uint64_t)base + i0 + 4 * v);
      r.p[4 * v + 0] = p4.x; r.p[4 * v + 1] = p4.y; r.p[4 * v + 2] = p4.z; r.p[4 * v + 3] = p4.w;
    }
#pragma unroll
    for (uint32_t v = 0; v < kPer / 4; ++v) {
      const uint64_t i = (uint64_t)base + i0 + 4 * v;
      const float4 x4 = load_stream_f4<PER == 4>(f.depth + i);
      r.x[4 * v + 0] = x4.x; r.x[4 * v + 1] = x4.y; r.x[4 * v + 2] = x4.z; r.x[4 * v + 3] = x4.w;
#pragma unroll
      for (int q = 0; q < C; ++q) {
        const float4 a4 = load_stream_f4<PER == 4>(f.alpha + C * i + 4 * q);
        r.a[4 * C * v + 4 * q + 0] = a4.x; r.a[4 * C * v + 4 * q + 1] = a4.y;
        r.a[4 * C * v + 4 * q + 2] = a4.z; r.a[4 * C * v + 4 * q + 3] = a4.w;
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float4 c4 = load_stream_f4<PER == 4>(f.rgb + 3 * i + 4 * q);
        r.c[12 * v + 4 * q + 0] = c4.x; r.c[12 * v + 4 * q + 1] = c4.y;
        r.c[12 * v + 4 * q + 2] = c4.z; r.c[12 * v + 4 * q + 3] = c4.w;
      }
    }
  } else {
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      const uint32_t li = i0 + k;
      r.p[k] = 0xffffffffu;
      if (li < n) {
        const uint64_t i = (uint64_t)base + li;
        r.p[k] = f.pixel[i];
        r.x[k] = f.depth[i];
#pragma unroll
        for (int q = 0; q < C; ++q) r.a[C * k + q] = f.alpha[C * i + q];
#pragma unroll
        for (int q = 0; q < 3; ++q) r.c[3 * k + q] = f.rgb[3 * i + q];
      }
    }
  }
}

template <int C, int PER>
__device__ __forceinline__ bool has_nan(const ChunkRegs<C, PER>& r, uint32_t k) {
  bool bad = isnan(r.x[k]);
#pragma unroll
  for (int q = 0; q < C; ++q) bad |= isnan(r.a[C * k + q]);
  return bad;
}

// Record dword j of fragment k (tile-local pixel `local`, stream index `src`).
// Forward binning stores each alpha as its absorbance step (binned_absorbance); records binned for the gradient
// keep alpha.
template <int C, int PER>
__device__ __forceinline__ void to_absorbance(ChunkRegs<C, PER>& r) {
#pragma unroll
  for (int i = 0; i < C * PER; ++i) r.a[i] = binned_absorbance(r.a[i]);
}

template <int C, int PER>
__device__ __forceinline__ uint32_t record_word(const ChunkRegs<C, PER>& r, uint32_t k, uint32_t local, uint32_t src,
                                                uint32_t j) {
  if (j == 0) return local;
  if (j == 1) return __float_as_uint(r.x[k]);
  if (j < 2 + C) return __float_as_uint(r.a[C * k + (j - 2)]);
  if (j < 5 + C) return __float_as_uint(r.c[3 * k + (j - 2 - C)]);
  return src;
}

// Block-wide exclusive scan of cnt[0, nt) in place; wsum holds THREADS / 64 partial sums.
template <int THREADS>
__device__ __forceinline__ void block_scan_inplace(uint32_t* cnt, uint32_t nt, uint32_t* wsum) {
  const uint32_t per = (nt + THREADS - 1) / THREADS;
  const uint32_t t0 = threadIdx.x * per, t1 = std::min(t0 + per, nt);
  uint32_t s = 0;
  for (uint32_t t = t0; t < t1; ++t) s += cnt[t];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += v;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0;
    for (uint32_t w = 0; w < THREADS / 64; ++w) {
      const uint32_t v = wsum[w];
      wsum[w] = a;
      a += v;
    }
  }
  __syncthreads();
  uint32_t run = wsum[wv] + inc - s;
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t v = cnt[t];
    cnt[t] = run;
    run += v;
  }
}

// A record as it is stored: N dwords, 4-byte aligned, so that one lane writes one record with one wide store and
// consecutive lanes write consecutive records.
template <uint32_t N>
struct Words {
  uint32_t w[N];
};

// Bytes of one record staged in LDS by the chunk scatter (its head words plus the tile, and its tail words) or by
// the split (head words plus the record's slot, and tail words), unpadded.
constexpr uint32_t staged_record_bytes(uint32_t C, bool idx) { return 4 * (head_dwords(C) + 1 + tail_dwords(idx)); }

// N words to or from LDS with the widest accesses the address allows (d holds N-word records back to back, at a
// 16-byte aligned base).
template <uint32_t N>
__device__ __forceinline__ void lds_put(uint32_t* d, const uint32_t* w) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (uint32_t u = 0; u < N / 4; ++u) ((uint4*)d)[u] = make_uint4(w[4 * u], w[4 * u + 1], w[4 * u + 2], w[4 * u + 3]);
  } else if constexpr (N % 2 == 0) {
#pragma unroll
    for (uint32_t u = 0; u < N / 2; ++u) ((uint2*)d)[u] = make_uint2(w[2 * u], w[2 * u + 1]);
  } else {
#pragma unroll
    for (uint32_t u = 0; u < N; ++u) d[u] = w[u];
  }
}

template <uint32_t N>
__device__ __forceinline__ void lds_get(const uint32_t* d, uint32_t* w) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (uint32_t u = 0; u < N / 4; ++u) {
      const uint4 v = ((const uint4*)d)[u];
      w[4 * u] = v.x; w[4 * u + 1] = v.y; w[4 * u + 2] = v.z; w[4 * u + 3] = v.w;
    }
  } else if constexpr (N % 2 == 0) {
#pragma unroll
    for (uint32_t u = 0; u < N / 2; ++u) {
      const uint2 v = ((const uint2*)d)[u];
      w[2 * u] = v.x; w[2 * u + 1] = v.y;
    }
  } else {
#pragma unroll
    for (uint32_t u = 0; u < N; ++u) w[u] = d[u];
  }
}

// LDS: srec[S][SH + ST] uint4 one round of sorted records (the slot word holds the tile until the write), cnt[nt]
// (counts, then first staged positions), gb[nt] (reserved base - run start, per round). The chunk's sorted order is
// written in
// rounds of S records (S = stage, a power of two chosen by the host to fit the LDS).
// PER = 4 is meant for two workgroups per compute unit (LDS <= 80 KB, <= 64 VGPRs at eight waves per SIMD):
// one workgroup's loads and stores overlap the other's ranking and staging.
// Refusal of a scatter that does not belong to the count before it, or whose stream puts more records in a segment
// than were counted: nothing more is written and the binning is not sealed.
__device__ __forceinline__ void scatter_refuse(WsHeader* hdr) {
  atomicOr(&hdr->fault, 1u);
  ws_raise(hdr, kWsErrScatter);
}

template <int C, bool IDX, int THREADS, int PER>
__global__ __launch_bounds__(THREADS, PER == 4 ? 8 : (THREADS == 512 ? 4 : 1)) void k_scatter_staged(wt_fragments f, Geom g, int vec,
                                                                    uint32_t stage,
                                                                    uint32_t* __restrict__ cursors,
                                                                    uint32_t* __restrict__ head,
                                                                    uint32_t* __restrict__ tail,
                                                                    WsHeader* hdr, unsigned long long cstamp,
                                                                    uint32_t cap) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX), HW = DH + 1;
  extern __shared__ uint4 sm4[];
  uint32_t* sh = (uint32_t*)sm4;               // [stage][HW]: head words, then the tile
  uint32_t* st = sh + (size_t)stage * HW;      // [stage][DT]: tail words
  uint32_t* cnt = st + (size_t)stage * DT;
  uint32_t* gb = cnt + g.ntiles;
  __shared__ uint32_t wsum[THREADS / 64];
  __shared__ uint32_t nvalid, refused;
  const uint32_t F = (uint32_t)f.count;
  const uint32_t cls = blockIdx.x % g.NX;
  const uint32_t base = blockIdx.x * g.chunk;
  const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
  for (uint32_t t = threadIdx.x; t < g.ntiles; t += blockDim.x) cnt[t] = 0;
  if (threadIdx.x == 0) nvalid = refused = 0;
  ChunkRegs<C, PER> r;
  const uint32_t i0 = threadIdx.x * PER;
  load_chunk<C, PER>(f, base, i0, n, vec, r);
  // only the stream the preceding count counted, under the same layout, is scattered into its segments (the
  // stamp is loaded behind the chunk, so the check adds no wait of its own)
  if (hdr->counted != cstamp) {
    if (threadIdx.x == 0) scatter_refuse(hdr);
    return;
  }
  if constexpr (!IDX) to_absorbance<C, PER>(r);
  __syncthreads();
  uint32_t tile[PER], rank[PER], local[PER];
  uint32_t nan_count = 0, mine = 0;
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) {
    tile[k] = 0xffffffffu;
    if (r.p[k] < g.P) {
      tile_locate(g, r.p[k], tile[k], local[k]);
      rank[k] = atomicAdd(&cnt[tile[k]], 1u);
      nan_count += has_nan<C, PER>(r, k) ? 1u : 0u;
      ++mine;
    }
  }
  mine = wave_sum(mine);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&nvalid, mine);
  __syncthreads();
  block_scan_inplace<THREADS>(cnt, g.ntiles, wsum);
  __syncthreads();
  // cnt[t] is now the chunk's first staged position of tile t (tile-major order)
  uint32_t sp[PER];
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) sp[k] = (tile[k] == 0xffffffffu) ? 0xffffffffu : cnt[tile[k]] + rank[k];
  const uint32_t total = nvalid;
  for (uint32_t r0 = 0; r0 < total; r0 += stage) {
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      if (sp[k] < r0 || sp[k] >= r0 + stage) continue;  // also skips invalid slots (0xffffffff)
      uint32_t hw[HW], tw[DT];
#pragma unroll
      for (uint32_t j = 0; j < HW; ++j) hw[j] = j < DH ? record_word<C, PER>(r, k, local[k], base + i0 + k, j) : tile[k];
#pragma unroll
      for (uint32_t j = 0; j < DT; ++j) tw[j] = record_word<C, PER>(r, k, local[k], base + i0 + k, DH + j);
      lds_put<HW>(sh + (size_t)(sp[k] - r0) * HW, hw);
      lds_put<DT>(st + (size_t)(sp[k] - r0) * DT, tw);
    }
    // Reserve this round's run of every tile it holds (one returning atomic per tile on the XCD's shared cursor)
    // just before the round is written: slots stay reserved but unwritten for one round only, so fewer partly
    // written lines wait at the frontier and more of them complete in L2 before write-back. The run of tile t is
    // [max(first_t, r0), min(end_t, r1)); gb[t] = reserved base - run start, so a record's slot is gb[t] plus its
    // staged position. (Issuing the next round's reservations during this round's writes was slower: the
    // registers that hold them push the kernel past its two-workgroup budget.)
    const uint32_t r1 = std::min(r0 + stage, total);
    for (uint32_t t = threadIdx.x; t < g.ntiles; t += THREADS) {
      const uint32_t p0 = cnt[t], p1 = t + 1 < g.ntiles ? cnt[t + 1] : total;
      const uint32_t lo = std::max(p0, r0), hi = std::min(p1, r1);
      if (hi > lo) {
        const uint32_t got = atomicAdd(&cursors[(cls * g.ntiles + t) * kCursorPad], hi - lo);
        gb[t] = got - lo;
        // writes stay inside the record arrays whatever the cursors hold; a stream that changed since its count
        // and overruns a segment into its neighbour leaves cursors off their segment ends, which the seal sees
        if (got > cap || cap - got < hi - lo) refused = 1;
      }
    }
    __syncthreads();
    if (refused) {
      if (threadIdx.x == 0) scatter_refuse(hdr);
      return;
    }
    const uint32_t ns = std::min(stage, total - r0);
    for (uint32_t sidx = threadIdx.x; sidx < ns; sidx += blockDim.x) {
      uint32_t hw[HW], tw[DT];
      lds_get<HW>(sh + (size_t)sidx * HW, hw);
      lds_get<DT>(st + (size_t)sidx * DT, tw);
      const uint64_t slot = (uint32_t)(gb[hw[DH]] + r0 + sidx);
      Words<DH> h;
#pragma unroll
      for (uint32_t j = 0; j < DH; ++j) h.w[j] = hw[j];
      Words<DT> t;
#pragma unroll
      for (uint32_t j = 0; j < DT; ++j) t.w[j] = tw[j];
      *(Words<DH>*)(head + slot * DH) = h;
      *(Words<DT>*)(tail + slot * DT) = t;
    }
    __syncthreads();
  }
  nan_count = wave_sum(nan_count);
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(&hdr->dropped, (unsigned long long)nan_count);
}

template <int C, bool IDX, int THREADS>
__global__ __launch_bounds__(THREADS) void k_scatter_global(wt_fragments f, Geom g, int vec,
                                                                    uint32_t* __restrict__ cursors,
                                                                    uint32_t* __restrict__ head,
                                                                    uint32_t* __restrict__ tail,
                                                                    WsHeader* hdr, unsigned long long cstamp,
                                                                    uint32_t cap) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX);
  if (hdr->counted != cstamp) {
    if (threadIdx.x == 0) scatter_refuse(hdr);
    return;
  }
  const uint32_t F = (uint32_t)f.count;
  const uint32_t base = blockIdx.x * g.chunk;
  const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
  ChunkRegs<C, kPer> r;
  const uint32_t i0 = threadIdx.x * kPer;
  load_chunk<C, kPer>(f, base, i0, n, vec, r);
  if constexpr (!IDX) to_absorbance<C, kPer>(r);
  uint32_t nan_count = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    if (r.p[k] >= g.P) continue;
    uint32_t tile, local;
    tile_locate(g, r.p[k], tile, local);
    nan_count += has_nan<C, kPer>(r, k) ? 1u : 0u;
    const uint64_t pos = atomicAdd(&cursors[tile * kCursorPad], 1u);
    if (pos >= cap) {  // inside the record arrays whatever the cursors hold (the seal checks the segments)
      scatter_refuse(hdr);
      continue;
    }
#pragma unroll
    for (uint32_t j = 0; j < DH; ++j) head[pos * DH + j] = record_word<C, kPer>(r, k, local, base + i0 + k, j);
#pragma unroll
    for (uint32_t j = 0; j < DT; ++j) tail[pos * DT + j] = record_word<C, kPer>(r, k, local, base + i0 + k, DH + j);
  }
  nan_count = wave_sum(nan_count);
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(&hdr->dropped, (unsigned long long)nan_count);
}

// WT_DETERMINISTIC binning: one thread copies the stream in stream order straight into the tile segments (the
// class of fragment i is that of its chunk, as in the count), so every segment holds its records in stream order.
template <int C, bool IDX>
__global__ void k_scatter_serial(wt_fragments f, Geom g, uint32_t* __restrict__ cursors,
                                 const uint32_t* __restrict__ offsets, uint32_t* __restrict__ head,
                                 uint32_t* __restrict__ tail, WsHeader* hdr, unsigned long long cstamp) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX);
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (hdr->counted != cstamp) {
    scatter_refuse(hdr);
    return;
  }
  unsigned long long nan_count = 0;
  for (uint64_t i = 0; i < f.count; ++i) {
    const uint32_t p = f.pixel[i];
    if (p >= g.P) continue;
    uint32_t tile, local;
    tile_locate(g, p, tile, local);
    const uint32_t cls = (uint32_t)((i / g.chunk) % g.NX);
    uint32_t* cur = &cursors[(cls * g.ntiles + tile) * kCursorPad];
    const uint32_t pos = *cur;
    if (pos >= offsets[tile * g.NX + cls + 1]) {
      scatter_refuse(hdr);
      return;
    }
    *cur = pos + 1;
    const float x = f.depth[i];
    bool bad = isnan(x);
    uint32_t* h = head + (uint64_t)pos * DH;
    h[0] = local;
    h[1] = __float_as_uint(x);
    for (int c = 0; c < C; ++c) {
      const float al = f.alpha[i * C + c];
      bad |= isnan(al);
      h[2 + c] = __float_as_uint(IDX ? al : binned_absorbance(al));
    }
    uint32_t* t = tail + (uint64_t)pos * DT;
    for (int q = 0; q < 3; ++q) t[q] = __float_as_uint(f.rgb[i * 3 + q]);
    if (IDX) t[3] = (uint32_t)i;
    nan_count += bad ? 1 : 0;
  }
  if (nan_count) atomicAdd(&hdr->dropped, nan_count);
}

// Second level of two-level binning: one workgroup per super-tile moves its records (all classes, contiguous in
// the first-level arrays) into the tiles' segments of the final arrays. Rounds of split_per(C, IDX) records per
// thread: rank by tile in LDS, place in tile order in LDS (head words plus the record's slot, then the tail words,
// unpadded), write with consecutive lanes on consecutive records. The workgroup owns its tiles, so their write
// cursors live in LDS; runs are about kSplitThreads * split_per / (SW SH) records long, so each round takes as many
// records as the LDS holds (glass 3840x2160, 32 tiles per super-tile: two records per thread 3.35 ms, three 3.28,
// four 3.18).
constexpr uint32_t kSplitThreads = 1024;
constexpr uint32_t split_per(uint32_t C, bool idx) {
  return (kLdsBytes - 2048) / (kSplitThreads * staged_record_bytes(C, idx));
}

template <int C, bool IDX>
__global__ __launch_bounds__(kSplitThreads) void k_split(Geom g, const uint32_t* __restrict__ offsets1,
                                                         const uint32_t* __restrict__ offsets,
                                                         const uint32_t* __restrict__ head1,
                                                         const uint32_t* __restrict__ tail1,
                                                         uint32_t* __restrict__ head, uint32_t* __restrict__ tail,
                                                         const WsHeader* hdr, unsigned long long level1) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX), HW = DH + 1;
  constexpr uint32_t PER = split_per(C, IDX), RECS = kSplitThreads * PER;
  // only a complete first level is split (its records then hold valid super-tile-local pixels)
  if (hdr->binned != level1) return;
  extern __shared__ uint4 sm4[];
  uint32_t* sh = (uint32_t*)sm4;  // [RECS][HW]: head words, then the record's slot
  uint32_t* st = sh + RECS * HW;  // [RECS][DT]: tail words
  __shared__ uint32_t cur[kMaxSub], cnt[kMaxSub], pre[kMaxSub];
  const uint32_t sidx = blockIdx.x;
  const uint32_t sx = sidx % g.sX, sy = sidx / g.sX;
  const uint32_t nsub = g.SW * g.SH;
  const uint32_t beg = offsets1[sidx * g.NX], end = offsets1[(sidx + 1) * g.NX];
  const uint32_t lTWs = g.lTW + g.lSW;  // super-tile width in pixels is 2^lTWs
  if (threadIdx.x < nsub) {
    const uint32_t j = threadIdx.x;
    const uint32_t tx = (sx << g.lSW) + (j & (g.SW - 1)), ty = (sy << g.lSH) + (j >> g.lSW);
    cur[j] = (tx < g.tilesX && ty < g.tilesY) ? offsets[(ty * g.tilesX + tx) * g.NX] : 0u;
  }
  for (uint32_t c0 = beg; c0 < end; c0 += RECS) {
    if (threadIdx.x < nsub) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t hw[PER][HW], tw[PER][DT], sub[PER], rank[PER];
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      const uint32_t i = c0 + k * kSplitThreads + threadIdx.x;
      sub[k] = 0xffffffffu;
      if (i < end) {
#pragma unroll
        for (uint32_t w = 0; w < DH; ++w) hw[k][w] = head1[(uint64_t)i * DH + w];
#pragma unroll
        for (uint32_t w = 0; w < DT; ++w) tw[k][w] = tail1[(uint64_t)i * DT + w];
        const uint32_t loc = hw[k][0];  // pixel within the super-tile
        const uint32_t lx = loc & ((1u << lTWs) - 1), ly = loc >> lTWs;
        sub[k] = ((ly >> g.lTH) << g.lSW) + (lx >> g.lTW);
        hw[k][0] = ((ly & (g.TH - 1)) << g.lTW) + (lx & (g.TW - 1));  // pixel within the tile
        rank[k] = atomicAdd(&cnt[sub[k]], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t run = 0;
      for (uint32_t j = 0; j < nsub; ++j) {
        pre[j] = run;
        run += cnt[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      if (sub[k] == 0xffffffffu) continue;
      hw[k][DH] = cur[sub[k]] + rank[k];
      const uint32_t pos = pre[sub[k]] + rank[k];
      lds_put<HW>(sh + (size_t)pos * HW, hw[k]);
      lds_put<DT>(st + (size_t)pos * DT, tw[k]);
    }
    __syncthreads();
    const uint32_t ns = std::min(RECS, end - c0);
    for (uint32_t q = threadIdx.x; q < ns; q += kSplitThreads) {
      uint32_t h[HW], t[DT];
      lds_get<HW>(sh + (size_t)q * HW, h);
      lds_get<DT>(st + (size_t)q * DT, t);
      const uint64_t slot = h[DH];
      Words<DH> hh;
#pragma unroll
      for (uint32_t w = 0; w < DH; ++w) hh.w[w] = h[w];
      Words<DT> tt;
#pragma unroll
      for (uint32_t w = 0; w < DT; ++w) tt.w[w] = t[w];
      *(Words<DH>*)(head + slot * DH) = hh;
      *(Words<DT>*)(tail + slot * DT) = tt;
    }
    __syncthreads();
    if (threadIdx.x < nsub) cur[threadIdx.x] += cnt[threadIdx.x];
  }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Largest staging round with two workgroups per compute unit. A round's slots are reserved when it is staged and
// stay partly written until it is, so longer rounds leave more partial lines at the frontier: on the smoke frame
// rounds of 2048 records took 1.93 ms against 1.69 ms for 1024 (and shorter rounds expose the reservations' latency
// more often: 512, 2.07 ms).
constexpr uint32_t kStageTwoWg = 1024;

template <int C, bool IDX, int PER, int THREADS>
static hipError_t launch_scatter_t(const Geom& g, const wt_fragments& f, int vec, uint32_t* cursors,
                                   uint32_t* head, uint32_t* tail, WsHeader* hdr,
                                   unsigned long long cstamp, uint32_t cap, uint32_t nchunks, hipStream_t s) {
  if (g.lds_bins) {
    constexpr uint32_t RB = staged_record_bytes(C, IDX);
    // largest power-of-two round beside the tile tables (1 KB left for static LDS), within half the LDS when two
    // workgroups share a compute unit
    constexpr bool kTwoWg = PER == 4 || THREADS == 512;
    const size_t budget = (kTwoWg ? kLdsBytes / 2 : kLdsBytes) - 1024;
    uint32_t stage = std::min<uint32_t>(g.chunk, kTwoWg ? kStageTwoWg : g.chunk);
    while (stage > 256 && (size_t)stage * RB + 8ull * g.rb > budget) stage >>= 1;
    const size_t lds = (size_t)stage * RB + 8ull * g.rb;
    auto k = k_scatter_staged<C, IDX, THREADS, PER>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(nchunks), dim3(THREADS), lds, s, f, g, vec, stage, cursors, head, tail, hdr, cstamp,
                       cap);
  } else {
    hipLaunchKernelGGL((k_scatter_global<C, IDX, THREADS>), dim3(nchunks), dim3(THREADS), 0, s, f, g, vec, cursors,
                       head, tail, hdr, cstamp, cap);
  }
  return hipGetLastError();
}

template <int C, bool IDX>
static hipError_t launch_scatter(const Geom& g, const wt_fragments& f, int vec, uint32_t* cursors,
                                 uint32_t* head, uint32_t* tail, WsHeader* hdr,
                                 unsigned long long cstamp, uint32_t cap, uint32_t nchunks, hipStream_t s) {
  if (g.kper == 4)
    return launch_scatter_t<C, IDX, 4, 1024>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s);
  if (g.sthreads == 512)
    return launch_scatter_t<C, IDX, kPer, 512>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s);
  return launch_scatter_t<C, IDX, kPer, 1024>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s);
}

hipError_t launch_bin_count(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, hipStream_t s) {
  char* b = (char*)ws;
  uint32_t* counts = (uint32_t*)(b + l.counts);
  uint32_t* offsets = (uint32_t*)(b + l.offsets);
  uint32_t* cursors = (uint32_t*)(b + l.cursors);
  WsHeader* hdr = (WsHeader*)(b + l.header);
  unsigned long long* dropped = &hdr->dropped;
  const uint64_t ncount = (uint64_t)g.NX * g.ntiles;
  // reset the header and zero the tile counts (kernels, not memsets: safe inside captured graphs)
  hipLaunchKernelGGL(k_header_reset, dim3(1), dim3(1), 0, s, hdr);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((ncount + 255) / 256, 4096)), dim3(256), 0, s,
                     counts, ncount, 0u);
  const uint32_t F = (uint32_t)f.count;
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + g.chunk - 1) / g.chunk);
  const int vec = aligned16(f.pixel);
  if (F > 0) {
    if (g.lds_bins) {
      // at most 1024 workgroups (four per compute unit with 256 threads): each counts about 32 chunks of its class
      // and then adds its table to the global counts once (half the global adds of 2048 workgroups; the smoke
      // frame's histogram measured 0.111 -> 0.101 ms)
      const uint32_t grid = std::min<uint32_t>(((nchunks + g.NX - 1) / g.NX) * g.NX, 1024);
      const size_t lds = 4ull * g.hrb;
      if (lds <= 32768) {
        hipLaunchKernelGGL(k_hist_lds<256>, dim3(grid), dim3(256), lds, s, f.pixel, F, g, vec, counts, dropped);
      } else {
        auto k = k_hist_lds<1024>;
        if (lds > 65536) {
          hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k, dim3(grid), dim3(1024), lds, s, f.pixel, F, g, vec, counts, dropped);
      }
    } else {
      hipLaunchKernelGGL(k_hist_global, dim3(2048), dim3(256), 0, s, f.pixel, F, g, counts, dropped);
    }
  }
  const unsigned long long cstamp = count_stamp(g, l, f);
  const uint64_t nseg = (uint64_t)g.NX * g.ntiles;
  if (nseg <= 2 * (uint64_t)kScanRange) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts, g, offsets, cursors,
                       (uint32_t*)(b + l.order), 1, g.two ? nullptr : hdr, cstamp);
  } else {
    // many segments (two-level and global-atomic binnings): the scan over several workgroups
    uint32_t* part = (uint32_t*)(b + l.scan);
    const uint32_t G = (uint32_t)((nseg + kScanRange - 1) / kScanRange);
    hipLaunchKernelGGL(k_scan_part, dim3(G), dim3(kScanThreads), 0, s, counts, g, part);
    hipLaunchKernelGGL(k_scan_apply, dim3(G), dim3(kScanThreads), 0, s, counts, g, part, offsets, cursors,
                       (uint32_t*)(b + l.order), 1, g.two ? nullptr : hdr, cstamp);
  }
  if (g.two) {
    // first level: per-class super-tile counts, and their segments and cursors
    const Geom gs = super_geom(g);
    uint32_t* counts1 = (uint32_t*)(b + l.counts1);
    const uint32_t n1 = g.NX * g.nsuper;
    hipLaunchKernelGGL(k_super_counts, dim3((n1 + 255) / 256), dim3(256), 0, s, counts, g, counts1);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts1, gs, (uint32_t*)(b + l.offsets1),
                       (uint32_t*)(b + l.cursors1), (uint32_t*)(b + l.order1), 0, hdr, cstamp);
  }
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                              hipStream_t s) {
  char* b = (char*)ws;
  uint32_t* cursors = (uint32_t*)(b + l.cursors);
  const uint32_t* offsets = (const uint32_t*)(b + l.offsets);
  uint32_t* head = (uint32_t*)(b + l.heads);
  uint32_t* tail = (uint32_t*)(b + l.tails);
  WsHeader* hdr = (WsHeader*)(b + l.header);
  const unsigned long long cstamp = count_stamp(g, l, f);
  const unsigned long long stamp = layout_stamp(g, l, record_index);
  const uint32_t cap = (uint32_t)std::min<uint64_t>(l.cap, 0xffffffffull);  // records each array holds
  const uint32_t F = (uint32_t)f.count;
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + g.chunk - 1) / g.chunk);
  const int vec = aligned16(f.pixel) && aligned16(f.depth) && aligned16(f.alpha) && aligned16(f.rgb);
  hipError_t e = hipSuccess;
  if (g.serial) {
    // deterministic: straight into the tile segments, whatever the number of levels
    auto k = g.C == 1 ? (record_index ? k_scatter_serial<1, true> : k_scatter_serial<1, false>)
                      : (record_index ? k_scatter_serial<3, true> : k_scatter_serial<3, false>);
    hipLaunchKernelGGL(k, dim3(1), dim3(64), 0, s, f, g, cursors, offsets, head, tail, hdr, cstamp);
    hipLaunchKernelGGL(k_seal, dim3(1), dim3(1024), 0, s, hdr, cursors, offsets, g.NX, g.ntiles, cstamp, stamp);
    return hipGetLastError();
  }
  if (!g.two) {
    if (F > 0) {
      if (g.C == 1)
        e = record_index ? launch_scatter<1, true>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s)
                         : launch_scatter<1, false>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s);
      else
        e = record_index ? launch_scatter<3, true>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s)
                         : launch_scatter<3, false>(g, f, vec, cursors, head, tail, hdr, cstamp, cap, nchunks, s);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_seal, dim3(1), dim3(1024), 0, s, hdr, cursors, offsets, g.NX, g.ntiles, cstamp, stamp);
    return hipGetLastError();
  }
  // two levels: the stream into super-tiles (first-level arrays), then each super-tile into its tiles
  const Geom gs = super_geom(g);
  uint32_t* cursors1 = (uint32_t*)(b + l.cursors1);
  uint32_t* head1 = (uint32_t*)(b + l.heads1);
  uint32_t* tail1 = (uint32_t*)(b + l.tails1);
  const uint32_t* offsets1 = (const uint32_t*)(b + l.offsets1);
  const unsigned long long stamp1 = level1_stamp(stamp);
  if (F > 0) {
    if (g.C == 1)
      e = record_index ? launch_scatter<1, true>(gs, f, vec, cursors1, head1, tail1, hdr, cstamp, cap, nchunks, s)
                       : launch_scatter<1, false>(gs, f, vec, cursors1, head1, tail1, hdr, cstamp, cap, nchunks, s);
    else
      e = record_index ? launch_scatter<3, true>(gs, f, vec, cursors1, head1, tail1, hdr, cstamp, cap, nchunks, s)
                       : launch_scatter<3, false>(gs, f, vec, cursors1, head1, tail1, hdr, cstamp, cap, nchunks, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_seal, dim3(1), dim3(1024), 0, s, hdr, cursors1, offsets1, gs.NX, g.nsuper, cstamp, stamp1);
  auto split = [&](auto kern, uint32_t rb, uint32_t per) -> hipError_t {
    const size_t lds = (size_t)kSplitThreads * per * rb;
    if (lds > 65536) {
      hipError_t e2 = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e2 != hipSuccess) return e2;
    }
    hipLaunchKernelGGL(kern, dim3(g.nsuper), dim3(kSplitThreads), lds, s, g, offsets1, offsets, head1, tail1, head,
                       tail, hdr, stamp1);
    return hipGetLastError();
  };
  if (g.C == 1)
    e = record_index ? split(k_split<1, true>, staged_record_bytes(1, true), split_per(1, true))
                     : split(k_split<1, false>, staged_record_bytes(1, false), split_per(1, false));
  else
    e = record_index ? split(k_split<3, true>, staged_record_bytes(3, true), split_per(3, true))
                     : split(k_split<3, false>, staged_record_bytes(3, false), split_per(3, false));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seal_split, dim3(1), dim3(1), 0, s, hdr, stamp1, stamp);
  return hipGetLastError();
}

hipError_t launch_bin(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                      hipStream_t s) {
  hipError_t e = launch_bin_count(g, f, ws, l, s);
  if (e != hipSuccess) return e;
  return launch_bin_scatter(g, f, ws, l, record_index, s);
}

}  // namespace wt
