// Ingest and screen-tile binning of an unordered fragment stream.
//
// The paper builds and evaluates inside a raster pipeline, where the fragments of one screen region arrive on
// the same shader core (section 2.1). A stored stream carries no such locality, and on this GPU per-fragment
// random atomics into a frame-sized coefficient buffer run at a few billion fragments per second. So the
// stream is first regrouped by screen tile with a counting sort (histogram, scan, scatter), after which every
// per-pixel update of the build and evaluate passes happens in the LDS of the compute unit that owns the tile.
//
// Kernels:
//   k_hist            pixel ids (4 B/fragment) -> per-(class, tile) counts; range drops counted.
//   k_scan            exclusive scan of the counts, tile-major, into segment offsets and write cursors.
//   k_scatter_staged  one chunk (kPer fragments per thread) per workgroup: vector loads into registers, LDS count
//                     per tile, one cursor reservation per touched tile, records placed in LDS in tile order,
//                     then written as flat runs of dwords (head array, then tail array) so that consecutive
//                     lanes store consecutive addresses inside each tile's run.
//   k_scatter_global  one cursor atomic per fragment (very many tiles).
// A chunk's class is chunk % NX in both k_hist and the scatter; with one chunk per scatter workgroup the class
// is also the XCD the workgroup runs on, so each (tile, class) run is written from a single L2.
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
  const uint32_t bpx = g.tight ? 8 : 0;  // per-pixel depth bounds (two FP32) in LDS
  if (backward) {
    px = tile_for(12 * g.C * g.M + 4 * (3 + g.C) + bpx);
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
  // LDS tile tables of at most kMaxLdsBins tiles: one range, or several passes of balanced ranges
  const uint32_t nr = (g.ntiles + kMaxLdsBins - 1) / kMaxLdsBins;
  g.lds_bins = nr <= kMaxRanges ? 1 : 0;
  g.rb = (g.ntiles + nr - 1) / nr;
  const uint32_t hnr = (g.ntiles + kMaxHistBins - 1) / kMaxHistBins;
  g.hrb = (g.ntiles + hnr - 1) / hnr;
  g.NX = g.lds_bins ? kClasses : 1;
  // scatter workgroup: 1024 threads (one per CU, larger chunks) by default; WT_SCATTER_WG=512 selects two
  // 512-thread workgroups per CU (tuning override) where their tile tables fit half the LDS
  // Scatter: 1024 threads, 8 fragments per thread (one workgroup per compute unit), or 4 per thread where the
  // tile tables and a 1024-record round fit half the LDS, so that two workgroups share a compute unit.
  g.sthreads = 1024;
  g.kper = (g.lds_bins && 8ull * g.rb + 1024ull * 48 <= kLdsBytes / 2 - 1024) ? 4 : kPer;
  g.chunk = g.sthreads * g.kper;
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
  l.order = o;
  o = align256(o + 4ull * g.ntiles);
  l.heads = o;
  o = align256(o + 4ull * head_dwords(g.C) * cap);
  l.tails = o;
  o = align256(o + 4ull * tail_dwords(true) * cap);
  l.total = o;
  l.cap = cap;
  return l;
}

uint64_t capacity_for(const Geom& g, size_t ws_bytes) {
  const size_t fixed = make_layout(g, 0).total;
  if (ws_bytes < fixed) return 0;
  const uint64_t per = 4ull * record_dwords(g.C, true);
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
  return v;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------------------------------------------------ histogram

// Workgroups of 256 threads, or of 1024 when the tile table is large (up to 144 KB of LDS leaves one workgroup per
// compute unit, which then still has sixteen waves of loads in flight).

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
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint32_t base = c * g.chunk;
    const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
    if (vec && n == g.chunk) {
      // chunk / 4 uint4 per chunk; up to four per thread in flight at a time
      const uint4* q4 = (const uint4*)(pixel + base);
      const uint32_t nv = g.chunk / 4;
      for (uint32_t v0 = 0; v0 < nv; v0 += 4 * kHistThreads) {
        uint4 q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t iv = v0 + v * kHistThreads + threadIdx.x;
          q[v] = iv < nv ? q4[iv] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (v0 + v * kHistThreads + threadIdx.x >= nv) continue;
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
    } else {
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
constexpr uint32_t kOrderMax = 4096;  // tile counts up to this are ordered by size; beyond, raster order

// Exclusive scan over segments in (tile, class) order (counts/cursors are class-major [NX][ntiles]), then the
// tile order for the tile kernels: heaviest tile first, so the last workgroups to start are the light ones.
__global__ __launch_bounds__(kScanThreads) void k_scan(const uint32_t* __restrict__ counts, Geom g,
                                                       uint32_t* __restrict__ offsets,
                                                       uint32_t* __restrict__ cursors,
                                                       uint32_t* __restrict__ order) {
  __shared__ uint32_t sums[kScanThreads];
  __shared__ unsigned long long keys[kOrderMax];
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
  if (g.ntiles > kOrderMax) {
    for (uint32_t t = tid; t < g.ntiles; t += kScanThreads) order[t] = t;
    return;
  }
  // bitonic sort of (~count, tile) ascending over the next power of two >= ntiles
  uint32_t N = 1;
  while (N < g.ntiles) N <<= 1;
  for (uint32_t t = tid; t < N; t += kScanThreads) {
    unsigned long long key = ~0ull;
    if (t < g.ntiles) {
      uint32_t c = 0;
      for (uint32_t x = 0; x < g.NX; ++x) c += counts[x * g.ntiles + t];
      key = ((unsigned long long)(~c) << 32) | t;
    }
    keys[t] = key;
  }
  __syncthreads();
  for (uint32_t size = 2; size <= N; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = tid; i < N / 2; i += kScanThreads) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long a = keys[lo], b = keys[hi];
        if ((a > b) == up) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t t = tid; t < g.ntiles; t += kScanThreads) order[t] = (uint32_t)(keys[t] & 0xffffffffu);
}

// ------------------------------------------------------------------------------------------------ scatter


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
      const uint4 p4 = *(const uint4*)(f.pixel + (uint64_t)base + i0 + 4 * v);
      r.p[4 * v + 0] = p4.x; r.p[4 * v + 1] = p4.y; r.p[4 * v + 2] = p4.z; r.p[4 * v + 3] = p4.w;
    }
#pragma unroll
    for (uint32_t v = 0; v < kPer / 4; ++v) {
      const uint64_t i = (uint64_t)base + i0 + 4 * v;
      const float4 x4 = *(const float4*)(f.depth + i);
      r.x[4 * v + 0] = x4.x; r.x[4 * v + 1] = x4.y; r.x[4 * v + 2] = x4.z; r.x[4 * v + 3] = x4.w;
#pragma unroll
      for (int q = 0; q < C; ++q) {
        const float4 a4 = *(const float4*)(f.alpha + C * i + 4 * q);
        r.a[4 * C * v + 4 * q + 0] = a4.x; r.a[4 * C * v + 4 * q + 1] = a4.y;
        r.a[4 * C * v + 4 * q + 2] = a4.z; r.a[4 * C * v + 4 * q + 3] = a4.w;
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float4 c4 = *(const float4*)(f.rgb + 3 * i + 4 * q);
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

// Staged record in LDS: the head dwords followed by the record's global slot, padded to whole 16-byte units
// (SH of them), then the tail dwords padded likewise (ST units).
constexpr uint32_t staged_head_units(uint32_t C) { return (head_dwords(C) + 1 + 3) / 4; }
constexpr uint32_t staged_tail_units(bool idx) { return (tail_dwords(idx) + 3) / 4; }

// LDS: srec[S][SH + ST] uint4 one round of sorted records, cnt[nt], gb[nt]. The chunk's sorted order is written in
// rounds of S records (S = stage, a power of two chosen by the host to fit the LDS).
// PER = 4 is meant for two workgroups per compute unit (LDS <= 80 KB, <= 64 VGPRs at eight waves per SIMD):
// one workgroup's loads and stores overlap the other's ranking and staging.
template <int C, bool IDX, int THREADS, int PER>
__global__ __launch_bounds__(THREADS, PER == 4 ? 8 : 1) void k_scatter_staged(wt_fragments f, Geom g, int vec,
                                                                    uint32_t stage,
                                                                    uint32_t* __restrict__ cursors,
                                                                    uint32_t* __restrict__ head,
                                                                    uint32_t* __restrict__ tail,
                                                                    unsigned long long* __restrict__ dropped) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX);
  constexpr uint32_t SH = staged_head_units(C), ST = staged_tail_units(IDX), SU = SH + ST;
  extern __shared__ uint4 sm4[];
  uint4* srec = sm4;
  uint32_t* cnt = (uint32_t*)(srec + (size_t)stage * SU);
  uint32_t* gb = cnt + g.ntiles;
  __shared__ uint32_t wsum[THREADS / 64];
  __shared__ uint32_t nvalid;
  const uint32_t F = (uint32_t)f.count;
  const uint32_t cls = blockIdx.x % g.NX;
  const uint32_t base = blockIdx.x * g.chunk;
  const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
  for (uint32_t t = threadIdx.x; t < g.ntiles; t += blockDim.x) cnt[t] = 0;
  if (threadIdx.x == 0) nvalid = 0;
  ChunkRegs<C, PER> r;
  const uint32_t i0 = threadIdx.x * PER;
  load_chunk<C, PER>(f, base, i0, n, vec, r);
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
  // Reserve this chunk's run in every touched tile. The first kResv tiles of each thread keep their returned
  // slots in registers until after the block scan, so the round trip of the atomics overlaps the scan.
  constexpr uint32_t kResv = 4;
  uint32_t resv[kResv];
#pragma unroll
  for (uint32_t j = 0; j < kResv; ++j) {
    const uint32_t t = threadIdx.x + j * THREADS;
    const uint32_t v = t < g.ntiles ? cnt[t] : 0u;
    resv[j] = v ? atomicAdd(&cursors[cls * g.ntiles + t], v) : 0u;
  }
  for (uint32_t t = threadIdx.x + kResv * THREADS; t < g.ntiles; t += THREADS) {
    const uint32_t v = cnt[t];
    gb[t] = v ? atomicAdd(&cursors[cls * g.ntiles + t], v) : 0u;
  }
  block_scan_inplace<THREADS>(cnt, g.ntiles, wsum);
#pragma unroll
  for (uint32_t j = 0; j < kResv; ++j) {
    const uint32_t t = threadIdx.x + j * THREADS;
    if (t < g.ntiles) gb[t] = resv[j];
  }
  __syncthreads();
  uint32_t sp[PER];
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) sp[k] = (tile[k] == 0xffffffffu) ? 0xffffffffu : cnt[tile[k]] + rank[k];
  const uint32_t total = nvalid;
  for (uint32_t r0 = 0; r0 < total; r0 += stage) {
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      if (sp[k] < r0 || sp[k] >= r0 + stage) continue;  // also skips invalid slots (0xffffffff)
      uint32_t hw[4 * SH], tw[4 * ST];
#pragma unroll
      for (uint32_t j = 0; j < 4 * SH; ++j)
        hw[j] = j < DH ? record_word<C, PER>(r, k, local[k], base + i0 + k, j) : gb[tile[k]] + rank[k];
#pragma unroll
      for (uint32_t j = 0; j < 4 * ST; ++j) tw[j] = j < DT ? record_word<C, PER>(r, k, local[k], base + i0 + k, DH + j) : 0u;
      uint4* d = srec + (size_t)(sp[k] - r0) * SU;
#pragma unroll
      for (uint32_t u = 0; u < SH; ++u) d[u] = make_uint4(hw[4 * u], hw[4 * u + 1], hw[4 * u + 2], hw[4 * u + 3]);
#pragma unroll
      for (uint32_t u = 0; u < ST; ++u)
        d[SH + u] = make_uint4(tw[4 * u], tw[4 * u + 1], tw[4 * u + 2], tw[4 * u + 3]);
    }
    __syncthreads();
    const uint32_t ns = std::min(stage, total - r0);
    for (uint32_t sidx = threadIdx.x; sidx < ns; sidx += blockDim.x) {
      const uint4* q = srec + (size_t)sidx * SU;
      uint32_t hw[4 * SH], tw[4 * ST];
#pragma unroll
      for (uint32_t u = 0; u < SH; ++u) {
        const uint4 v = q[u];
        hw[4 * u] = v.x; hw[4 * u + 1] = v.y; hw[4 * u + 2] = v.z; hw[4 * u + 3] = v.w;
      }
#pragma unroll
      for (uint32_t u = 0; u < ST; ++u) {
        const uint4 v = q[SH + u];
        tw[4 * u] = v.x; tw[4 * u + 1] = v.y; tw[4 * u + 2] = v.z; tw[4 * u + 3] = v.w;
      }
      const uint64_t slot = hw[DH];
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
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(dropped, (unsigned long long)nan_count);
}

// The same for frames with more tiles than one LDS table holds: the chunk stays in registers and is placed in one
// pass per range of g.rb tiles.
template <int C, bool IDX, int THREADS, int PER>
__global__ __launch_bounds__(THREADS, PER == 4 ? 8 : 1) void k_scatter_ranged(wt_fragments f, Geom g, int vec,
                                                                    uint32_t stage,
                                                                    uint32_t* __restrict__ cursors,
                                                                    uint32_t* __restrict__ head,
                                                                    uint32_t* __restrict__ tail,
                                                                    unsigned long long* __restrict__ dropped) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX);
  constexpr uint32_t SH = staged_head_units(C), ST = staged_tail_units(IDX), SU = SH + ST;
  extern __shared__ uint4 sm4[];
  uint4* srec = sm4;
  uint32_t* cnt = (uint32_t*)(srec + (size_t)stage * SU);
  uint32_t* gb = cnt + g.rb;
  __shared__ uint32_t wsum[THREADS / 64];
  __shared__ uint32_t nvalid;
  const uint32_t F = (uint32_t)f.count;
  const uint32_t cls = blockIdx.x % g.NX;
  const uint32_t base = blockIdx.x * g.chunk;
  const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
  ChunkRegs<C, PER> r;
  const uint32_t i0 = threadIdx.x * PER;
  load_chunk<C, PER>(f, base, i0, n, vec, r);
  uint32_t tile[PER], local[PER];
  uint32_t nan_count = 0;
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) {
    tile[k] = 0xffffffffu;
    if (r.p[k] < g.P) {
      tile_locate(g, r.p[k], tile[k], local[k]);
      nan_count += has_nan<C, PER>(r, k) ? 1u : 0u;
    }
  }
  // The tile tables cover g.rb tiles at a time: one pass per range of tiles [t0, t0 + nt) (one pass unless the
  // frame has more tiles than a table holds); every fragment is placed in the pass of its tile's range.
  for (uint32_t t0 = 0; t0 < g.ntiles; t0 += g.rb) {
  const uint32_t nt = std::min(g.rb, g.ntiles - t0);
  for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) cnt[t] = 0;
  if (threadIdx.x == 0) nvalid = 0;
  __syncthreads();
  uint32_t rank[PER];
  uint32_t mine = 0;
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) {
    if (tile[k] - t0 < nt) {  // unsigned: also false for invalid slots
      rank[k] = atomicAdd(&cnt[tile[k] - t0], 1u);
      ++mine;
    }
  }
  mine = wave_sum(mine);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&nvalid, mine);
  __syncthreads();
  // Reserve this chunk's run in every touched tile. The first kResv tiles of each thread keep their returned
  // slots in registers until after the block scan, so the round trip of the atomics overlaps the scan.
  constexpr uint32_t kResv = 4;
  uint32_t* cur = cursors + cls * g.ntiles + t0;
  uint32_t resv[kResv];
#pragma unroll
  for (uint32_t j = 0; j < kResv; ++j) {
    const uint32_t t = threadIdx.x + j * THREADS;
    const uint32_t v = t < nt ? cnt[t] : 0u;
    resv[j] = v ? atomicAdd(&cur[t], v) : 0u;
  }
  for (uint32_t t = threadIdx.x + kResv * THREADS; t < nt; t += THREADS) {
    const uint32_t v = cnt[t];
    gb[t] = v ? atomicAdd(&cur[t], v) : 0u;
  }
  block_scan_inplace<THREADS>(cnt, nt, wsum);
#pragma unroll
  for (uint32_t j = 0; j < kResv; ++j) {
    const uint32_t t = threadIdx.x + j * THREADS;
    if (t < nt) gb[t] = resv[j];
  }
  __syncthreads();
  uint32_t sp[PER];
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) sp[k] = (tile[k] - t0 < nt) ? cnt[tile[k] - t0] + rank[k] : 0xffffffffu;
  const uint32_t total = nvalid;
  for (uint32_t r0 = 0; r0 < total; r0 += stage) {
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      if (sp[k] < r0 || sp[k] >= r0 + stage) continue;  // also skips invalid slots (0xffffffff)
      uint32_t hw[4 * SH], tw[4 * ST];
#pragma unroll
      for (uint32_t j = 0; j < 4 * SH; ++j)
        hw[j] = j < DH ? record_word<C, PER>(r, k, local[k], base + i0 + k, j) : gb[tile[k] - t0] + rank[k];
#pragma unroll
      for (uint32_t j = 0; j < 4 * ST; ++j) tw[j] = j < DT ? record_word<C, PER>(r, k, local[k], base + i0 + k, DH + j) : 0u;
      uint4* d = srec + (size_t)(sp[k] - r0) * SU;
#pragma unroll
      for (uint32_t u = 0; u < SH; ++u) d[u] = make_uint4(hw[4 * u], hw[4 * u + 1], hw[4 * u + 2], hw[4 * u + 3]);
#pragma unroll
      for (uint32_t u = 0; u < ST; ++u)
        d[SH + u] = make_uint4(tw[4 * u], tw[4 * u + 1], tw[4 * u + 2], tw[4 * u + 3]);
    }
    __syncthreads();
    const uint32_t ns = std::min(stage, total - r0);
    for (uint32_t sidx = threadIdx.x; sidx < ns; sidx += blockDim.x) {
      const uint4* q = srec + (size_t)sidx * SU;
      uint32_t hw[4 * SH], tw[4 * ST];
#pragma unroll
      for (uint32_t u = 0; u < SH; ++u) {
        const uint4 v = q[u];
        hw[4 * u] = v.x; hw[4 * u + 1] = v.y; hw[4 * u + 2] = v.z; hw[4 * u + 3] = v.w;
      }
#pragma unroll
      for (uint32_t u = 0; u < ST; ++u) {
        const uint4 v = q[SH + u];
        tw[4 * u] = v.x; tw[4 * u + 1] = v.y; tw[4 * u + 2] = v.z; tw[4 * u + 3] = v.w;
      }
      const uint64_t slot = hw[DH];
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
  }
  nan_count = wave_sum(nan_count);
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(dropped, (unsigned long long)nan_count);
}

template <int C, bool IDX, int THREADS>
__global__ __launch_bounds__(THREADS) void k_scatter_global(wt_fragments f, Geom g, int vec,
                                                                    uint32_t* __restrict__ cursors,
                                                                    uint32_t* __restrict__ head,
                                                                    uint32_t* __restrict__ tail,
                                                                    unsigned long long* __restrict__ dropped) {
  constexpr uint32_t DH = head_dwords(C), DT = tail_dwords(IDX);
  const uint32_t F = (uint32_t)f.count;
  const uint32_t base = blockIdx.x * g.chunk;
  const uint32_t n = std::min<uint32_t>(g.chunk, F - base);
  ChunkRegs<C, kPer> r;
  const uint32_t i0 = threadIdx.x * kPer;
  load_chunk<C, kPer>(f, base, i0, n, vec, r);
  uint32_t nan_count = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    if (r.p[k] >= g.P) continue;
    uint32_t tile, local;
    tile_locate(g, r.p[k], tile, local);
    nan_count += has_nan<C, kPer>(r, k) ? 1u : 0u;
    const uint64_t pos = atomicAdd(&cursors[tile], 1u);
#pragma unroll
    for (uint32_t j = 0; j < DH; ++j) head[pos * DH + j] = record_word<C, kPer>(r, k, local, base + i0 + k, j);
#pragma unroll
    for (uint32_t j = 0; j < DT; ++j) tail[pos * DT + j] = record_word<C, kPer>(r, k, local, base + i0 + k, DH + j);
  }
  nan_count = wave_sum(nan_count);
  if ((threadIdx.x & 63) == 0 && nan_count) atomicAdd(dropped, (unsigned long long)nan_count);
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <int C, bool IDX, int PER>
static hipError_t launch_scatter_t(const Geom& g, const wt_fragments& f, int vec, uint32_t* cursors, uint32_t* head,
                                   uint32_t* tail, unsigned long long* dropped, uint32_t nchunks, hipStream_t s) {
  constexpr int THREADS = 1024;
  if (g.lds_bins) {
    constexpr uint32_t SU = staged_head_units(C) + staged_tail_units(IDX);
    // largest power-of-two round beside the tile tables (1 KB left for static LDS), within half the LDS when two
    // workgroups share a compute unit
    const size_t budget = (PER == 4 ? kLdsBytes / 2 : kLdsBytes) - 1024;
    uint32_t stage = g.chunk;
    while (stage > 256 && (size_t)stage * SU * 16 + 8ull * g.rb > budget) stage >>= 1;
    const size_t lds = (size_t)stage * SU * 16 + 8ull * g.rb;
    auto k = g.rb < g.ntiles ? k_scatter_ranged<C, IDX, THREADS, PER> : k_scatter_staged<C, IDX, THREADS, PER>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(nchunks), dim3(THREADS), lds, s, f, g, vec, stage, cursors, head, tail, dropped);
  } else {
    hipLaunchKernelGGL((k_scatter_global<C, IDX, THREADS>), dim3(nchunks), dim3(THREADS), 0, s, f, g, vec, cursors,
                       head, tail, dropped);
  }
  return hipGetLastError();
}

template <int C, bool IDX>
static hipError_t launch_scatter(const Geom& g, const wt_fragments& f, int vec, uint32_t* cursors, uint32_t* head,
                                 uint32_t* tail, unsigned long long* dropped, uint32_t nchunks, hipStream_t s) {
  if (g.kper == 4) return launch_scatter_t<C, IDX, 4>(g, f, vec, cursors, head, tail, dropped, nchunks, s);
  return launch_scatter_t<C, IDX, 8>(g, f, vec, cursors, head, tail, dropped, nchunks, s);
}

hipError_t launch_bin_count(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, hipStream_t s) {
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
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + g.chunk - 1) / g.chunk);
  const int vec = aligned16(f.pixel);
  if (F > 0) {
    if (g.lds_bins) {
      const uint32_t grid = std::min<uint32_t>(((nchunks + g.NX - 1) / g.NX) * g.NX, 2048);
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
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts, g, offsets, cursors,
                     (uint32_t*)(b + l.order));
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                              hipStream_t s) {
  char* b = (char*)ws;
  uint32_t* cursors = (uint32_t*)(b + l.cursors);
  uint32_t* head = (uint32_t*)(b + l.heads);
  uint32_t* tail = (uint32_t*)(b + l.tails);
  unsigned long long* dropped = (unsigned long long*)(b + l.header);
  const uint32_t F = (uint32_t)f.count;
  if (F == 0) return hipSuccess;
  const uint32_t nchunks = (uint32_t)(((uint64_t)F + g.chunk - 1) / g.chunk);
  const int vec = aligned16(f.pixel) && aligned16(f.depth) && aligned16(f.alpha) && aligned16(f.rgb);
  if (g.C == 1)
    return record_index ? launch_scatter<1, true>(g, f, vec, cursors, head, tail, dropped, nchunks, s)
                        : launch_scatter<1, false>(g, f, vec, cursors, head, tail, dropped, nchunks, s);
  return record_index ? launch_scatter<3, true>(g, f, vec, cursors, head, tail, dropped, nchunks, s)
                      : launch_scatter<3, false>(g, f, vec, cursors, head, tail, dropped, nchunks, s);
}

hipError_t launch_bin(const Geom& g, const wt_fragments& f, void* ws, const Layout& l, bool record_index,
                      hipStream_t s) {
  hipError_t e = launch_bin_count(g, f, ws, l, s);
  if (e != hipSuccess) return e;
  return launch_bin_scatter(g, f, ws, l, record_index, s);
}

}  // namespace wt
