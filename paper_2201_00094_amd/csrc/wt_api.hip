// C ABI of libwt: argument validation, workspace layout and the order of kernel launches. Every call only
// enqueues work on the caller's stream; nothing here allocates device memory.
#include <stdarg.h>
#include <stdio.h>

#include <cmath>
#include <mutex>
#include <string>

#include "wt_internal.h"

// Workspace of wt_render_noalloc: one copy per GPU, held until the process ends. Host code reaches it only through
// the device address that hipGetSymbolAddress returns for the current device (scratch_here below).
static __device__ __align__(256) unsigned char scratch[WT_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

wt_status fail(wt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

wt_status hip_fail(hipError_t e, const char* where) {
  return fail(WT_ERR_HIP, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

wt_status check_desc(const wt_frame_desc* d) {
  if (!d) return fail(WT_ERR_INVALID, "desc is NULL");
  if (d->width == 0 || d->height == 0) return fail(WT_ERR_INVALID, "frame size %ux%u is empty", d->width, d->height);
  if ((uint64_t)d->width * d->height >= (1ull << 32))
    return fail(WT_ERR_RANGE, "frame %ux%u has 2^32 or more pixels", d->width, d->height);
  if (d->rank > 10) return fail(WT_ERR_RANGE, "rank %u exceeds 10", d->rank);
  if (d->channels != 1 && d->channels != 3) return fail(WT_ERR_INVALID, "channels must be 1 or 3, got %u", d->channels);
  if (d->coeff_dtype > WT_E5B9G9R9) return fail(WT_ERR_INVALID, "unknown coefficient dtype %u", d->coeff_dtype);
  if (d->coeff_dtype == WT_E5B9G9R9 && d->channels != 3)
    return fail(WT_ERR_INVALID, "E5B9G9R9 storage packs three channels (channels = %u)", d->channels);
  if (d->coeff_dtype == WT_E5B9G9R9 && d->rank > 4)
    return fail(WT_ERR_UNSUPPORTED, "E5B9G9R9 storage supports rank <= 4 (rank = %u)", d->rank);
  if (d->flags & ~(WT_TIGHT_DEPTH | WT_TEMPORAL | WT_DETERMINISTIC))
    return fail(WT_ERR_INVALID, "unknown flags 0x%x", d->flags);
  if ((d->flags & WT_TEMPORAL) && (d->flags & WT_TIGHT_DEPTH))
    return fail(WT_ERR_UNSUPPORTED, "WT_TEMPORAL excludes WT_TIGHT_DEPTH");
  if ((d->flags & WT_TEMPORAL) && d->rank > 4)
    return fail(WT_ERR_UNSUPPORTED, "WT_TEMPORAL supports rank <= 4 (rank = %u)", d->rank);
  return WT_OK;
}

wt_status check_temporal(const wt_frame_desc* d, const void* prev, const uint32_t* map, const void* coeffs,
                         const float* bg, const float* out) {
  if (!(d->flags & WT_TEMPORAL)) return fail(WT_ERR_INVALID, "the one-pass render needs a WT_TEMPORAL description");
  if (!bg || !out) return fail(WT_ERR_INVALID, "bg_rgb or out is NULL");
  if (map && prev && prev == coeffs)
    return fail(WT_ERR_INVALID, "prev_coeffs and coeffs are one buffer, which needs prev_pixel == NULL");
  return WT_OK;
}

static_assert(WT_MAX_FRAGMENTS == (1ull << 32) - (1ull << 20), "fragment limit");

wt_status check_frags(const wt_fragments* f) {
  if (!f) return fail(WT_ERR_INVALID, "frags is NULL");
  if (f->count > WT_MAX_FRAGMENTS)
    return fail(WT_ERR_RANGE, "fragment count %llu is above WT_MAX_FRAGMENTS (2^32 - 2^20)",
                (unsigned long long)f->count);
  if (f->count && (!f->pixel || !f->depth || !f->alpha || !f->rgb))
    return fail(WT_ERR_INVALID, "a fragment array pointer is NULL");
  return WT_OK;
}

wt_status check_ws(const wt::Geom& g, const void* ws, size_t ws_bytes, uint64_t need_cap, wt::Layout* l) {
  if (!ws) return fail(WT_ERR_INVALID, "workspace is NULL");
  const uint64_t cap = wt::capacity_for(g, ws_bytes);
  if (cap < need_cap || ws_bytes < wt::make_layout(g, 0).total)
    return fail(WT_ERR_RANGE, "workspace of %zu bytes holds %llu fragments, %llu needed (wt_workspace_bytes)", ws_bytes,
                (unsigned long long)cap, (unsigned long long)need_cap);
  *l = wt::make_layout(g, cap);
  return WT_OK;
}

wt_status check_lds(const wt::Geom& g) {
  if (wt::lds_tile_bytes(g, true) > wt::kLdsBytes)
    return fail(WT_ERR_UNSUPPORTED, "tile of %u pixels needs %zu bytes of LDS", g.tile_px, wt::lds_tile_bytes(g, true));
  return WT_OK;
}

#define WT_TRY(expr)                 \
  do {                               \
    wt_status st_ = (expr);          \
    if (st_ != WT_OK) return st_;    \
  } while (0)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices];  // device address of scratch on device d, once looked up

// Device address of the current device's scratch array, looked up with hipGetSymbolAddress on the first call per
// device (with that device current) and kept.
wt_status scratch_here(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "wt_render_noalloc (hipGetDevice)");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(WT_ERR_UNSUPPORTED, "wt_render_noalloc: device %d is beyond the %d devices tracked", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "wt_render_noalloc (hipGetSymbolAddress)");
    if (!p) return fail(WT_ERR_HIP, "wt_render_noalloc: hipGetSymbolAddress gave a null address");
    g_scratch_at[dev] = p;
  }
  *ptr = g_scratch_at[dev];
  return WT_OK;
}

}  // namespace

extern "C" {

int wt_abi_version(void) { return 2; }

const char* wt_last_error(void) { return g_last_error.c_str(); }

size_t wt_workspace_bytes(const wt_frame_desc* desc, uint64_t max_fragments) {
  if (check_desc(desc) != WT_OK || max_fragments > WT_MAX_FRAGMENTS) return 0;
  // the gradient uses smaller tiles (more tile-table entries), so size for whichever layout is larger
  const size_t fwd = wt::make_layout(wt::make_geom(*desc), max_fragments).total;
  const size_t bwd = wt::make_layout(wt::make_geom(*desc, true), max_fragments).total;
  return fwd > bwd ? fwd : bwd;
}

wt_status wt_bin(const wt_frame_desc* desc, const wt_fragments* frags, void* ws, size_t ws_bytes, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, frags->count, &l));
  hipError_t e = wt::launch_bin(g, *frags, ws, l, false, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_bin");
  return WT_OK;
}

wt_status wt_bin_count(const wt_frame_desc* desc, const wt_fragments* frags, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, frags->count, &l));
  hipError_t e = wt::launch_bin_count(g, *frags, ws, l, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_bin_count");
  return WT_OK;
}

wt_status wt_bin_scatter(const wt_frame_desc* desc, const wt_fragments* frags, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, frags->count, &l));
  hipError_t e = wt::launch_bin_scatter(g, *frags, ws, l, false, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_bin_scatter");
  return WT_OK;
}

wt_status wt_build_binned(const wt_frame_desc* desc, void* coeffs, const void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  WT_TRY(check_desc(desc));
  if (!coeffs) return fail(WT_ERR_INVALID, "coeffs is NULL");
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, 0, &l));
  hipError_t e = wt::launch_build(g, wt::binned_view(g, l, ws, false), coeffs, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_build");
  return WT_OK;
}

wt_status wt_evaluate_binned(const wt_frame_desc* desc, const void* coeffs, float* accum, const void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  if (!coeffs || !accum) return fail(WT_ERR_INVALID, "coeffs or accum is NULL");
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, 0, &l));
  hipError_t e = wt::launch_evaluate(g, wt::binned_view(g, l, ws, false), coeffs, accum, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_evaluate");
  return WT_OK;
}

wt_status wt_build(const wt_frame_desc* desc, const wt_fragments* frags, void* coeffs, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
  if (!coeffs) return fail(WT_ERR_INVALID, "coeffs is NULL");
  WT_TRY(wt_bin(desc, frags, ws, ws_bytes, stream));
  return wt_build_binned(desc, coeffs, ws, ws_bytes, stream);
}

wt_status wt_evaluate(const wt_frame_desc* desc, const wt_fragments* frags, const void* coeffs, float* accum,
                      void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!coeffs || !accum) return fail(WT_ERR_INVALID, "coeffs or accum is NULL");
  WT_TRY(wt_bin(desc, frags, ws, ws_bytes, stream));
  return wt_evaluate_binned(desc, coeffs, accum, ws, ws_bytes, stream);
}

wt_status wt_resolve(const wt_frame_desc* desc, const float* accum, const float* bg_rgb, float* out,
                     hipStream_t stream) {
  WT_TRY(check_desc(desc));
  if (!accum || !bg_rgb || !out) return fail(WT_ERR_INVALID, "accum, bg_rgb or out is NULL");
  const wt::Geom g = wt::make_geom(*desc);
  hipError_t e = wt::launch_resolve(g, accum, bg_rgb, out, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_resolve");
  return WT_OK;
}

wt_status wt_resolve_chromatic(const wt_frame_desc* desc, const float* accum, const float* background,
                               const float* offset, float dispersion, uint32_t taps, float* out, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  if (!accum || !background || !offset || !out) return fail(WT_ERR_INVALID, "accum, background, offset or out is NULL");
  if (taps < 3 || taps > 63 || !(taps & 1)) return fail(WT_ERR_INVALID, "taps must be odd and in 3..63, got %u", taps);
  if (!std::isfinite(dispersion)) return fail(WT_ERR_INVALID, "dispersion is not finite");
  if ((uintptr_t)accum % 16 || (uintptr_t)offset % 8)
    return fail(WT_ERR_INVALID, "accum must be 16-byte and offset 8-byte aligned");
  const wt::Geom g = wt::make_geom(*desc);
  hipError_t e = wt::launch_resolve_chromatic(g, accum, background, offset, dispersion, taps, out, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_resolve_chromatic");
  return WT_OK;
}

wt_status wt_render(const wt_frame_desc* desc, const wt_fragments* frags, const float* bg_rgb, void* coeffs,
                    float* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  if (!bg_rgb || !out) return fail(WT_ERR_INVALID, "bg_rgb or out is NULL");
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, frags->count, &l));
  hipError_t e = wt::launch_bin(g, *frags, ws, l, false, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_render (bin)");
  e = wt::launch_render(g, wt::binned_view(g, l, ws, false), bg_rgb, coeffs, out, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_render");
  return WT_OK;
}

wt_status wt_render_noalloc(const wt_frame_desc* desc, const wt_fragments* frags, const float* bg_rgb, void* coeffs,
                            float* out, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  if (!bg_rgb || !out) return fail(WT_ERR_INVALID, "bg_rgb or out is NULL");
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  const size_t need = wt::make_layout(g, frags->count).total;
  if (need > WT_SCRATCH_BYTES)
    return fail(WT_ERR_RANGE, "wt_render_noalloc: %llu fragments need %zu bytes of scratch, the static array holds %zu",
                (unsigned long long)frags->count, need, (size_t)WT_SCRATCH_BYTES);
  void* ws = nullptr;
  WT_TRY(scratch_here(&ws));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, WT_SCRATCH_BYTES, frags->count, &l));
  hipError_t e = wt::launch_bin(g, *frags, ws, l, false, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_render_noalloc (bin)");
  e = wt::launch_render(g, wt::binned_view(g, l, ws, false), bg_rgb, coeffs, out, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_render_noalloc");
  return WT_OK;
}

wt_status wt_render_binned(const wt_frame_desc* desc, const void* ws, size_t ws_bytes, const float* bg_rgb,
                           void* coeffs, float* out, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  if (!bg_rgb || !out) return fail(WT_ERR_INVALID, "bg_rgb or out is NULL");
  const wt::Geom g = wt::make_geom(*desc);
  WT_TRY(check_lds(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, 0, &l));
  hipError_t e = wt::launch_render(g, wt::binned_view(g, l, ws, false), bg_rgb, coeffs, out, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_render_binned");
  return WT_OK;
}

wt_status wt_render_temporal_binned(const wt_frame_desc* desc, const void* ws, size_t ws_bytes, const float* bg_rgb,
                                    const void* prev_coeffs, const uint32_t* prev_pixel, void* coeffs, float* out,
                                    hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_temporal(desc, prev_coeffs, prev_pixel, coeffs, bg_rgb, out));
  const wt::Geom g = wt::make_geom(*desc);
  if (wt::lds_temporal_bytes(g) > wt::kLdsBytes)
    return fail(WT_ERR_UNSUPPORTED, "one-pass tile of %u pixels needs %zu bytes of LDS", g.tile_px,
                wt::lds_temporal_bytes(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, 0, &l));
  hipError_t e = wt::launch_render_temporal(g, wt::binned_view(g, l, ws, false), bg_rgb, prev_coeffs, prev_pixel,
                                            coeffs, out, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_render_temporal");
  return WT_OK;
}

wt_status wt_render_temporal(const wt_frame_desc* desc, const wt_fragments* frags, const float* bg_rgb,
                             const void* prev_coeffs, const uint32_t* prev_pixel, void* coeffs, float* out, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  WT_TRY(check_temporal(desc, prev_coeffs, prev_pixel, coeffs, bg_rgb, out));
  WT_TRY(wt_bin(desc, frags, ws, ws_bytes, stream));
  return wt_render_temporal_binned(desc, ws, ws_bytes, bg_rgb, prev_coeffs, prev_pixel, coeffs, out, stream);
}

wt_status wt_backward(const wt_frame_desc* desc, const wt_fragments* frags, const void* coeffs, const float* accum,
                      const float* bg_rgb, const float* grad_out, float* grad_alpha, float* grad_rgb, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  WT_TRY(check_desc(desc));
  WT_TRY(check_frags(frags));
  if (!coeffs || !accum || !bg_rgb || !grad_out || (frags->count && (!grad_alpha || !grad_rgb)))
    return fail(WT_ERR_INVALID, "a backward array pointer is NULL");
  const wt::Geom g = wt::make_geom(*desc, true);
  if (wt::lds_backward_bytes(g) > wt::kLdsBytes)
    return fail(WT_ERR_UNSUPPORTED, "gradient tile of %u pixels needs %zu bytes of LDS", g.tile_px,
                wt::lds_backward_bytes(g));
  wt::Layout l;
  WT_TRY(check_ws(g, ws, ws_bytes, frags->count, &l));
  hipError_t e = wt::launch_bin(g, *frags, ws, l, true, stream);
  if (e != hipSuccess) return hip_fail(e, "wt_backward (bin)");
  e = wt::launch_backward(g, wt::binned_view(g, l, ws, true), coeffs, accum, bg_rgb, grad_out, grad_alpha, grad_rgb,
                          frags->count, stream);
  if (e == hipErrorNotSupported) return fail(WT_ERR_UNSUPPORTED, "wt_backward: not available for this frame");
  if (e != hipSuccess) return hip_fail(e, "wt_backward");
  return WT_OK;
}

wt_status wt_dropped_count(const void* ws, size_t ws_bytes, uint64_t* count, hipStream_t stream) {
  if (!ws || !count) return fail(WT_ERR_INVALID, "ws or count is NULL");
  if (ws_bytes < 256) return fail(WT_ERR_RANGE, "workspace of %zu bytes has no header", ws_bytes);
  wt::WsHeader h{};
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "wt_dropped_count");
  if (h.magic != wt::kWsMagic) {  // nothing has been binned into this workspace yet
    *count = 0;
    return WT_OK;
  }
  *count = h.dropped;
  if (h.errors) {
    wt::WsHeader* dh = (wt::WsHeader*)const_cast<void*>(ws);
    e = wt::launch_fill_u32(&dh->errors, 1, 0u, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "wt_dropped_count (clearing the error bits)");
    return fail(WT_ERR_INVALID, "workspace misuse detected on the device since the last report (bits 0x%x):%s%s",
                h.errors,
                (h.errors & wt::kWsErrMismatch)
                    ? " a call over the binned stream found no complete binning for its description and workspace "
                      "size, and computed nothing;"
                    : "",
                (h.errors & wt::kWsErrScatter)
                    ? " a scatter did not follow a count of the same stream under the same layout, or its stream held "
                      "more fragments for a tile than were counted, and nothing was binned;"
                    : "");
  }
  return WT_OK;
}

}  // extern "C"
