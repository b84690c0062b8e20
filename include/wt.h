/*
 * wt.h -- C ABI of libwt, the MI355X (gfx950) wavelet-transparency resolve.
 *
 * Method: M. Aizenshtein, N. Smal, M. McGuire, "Wavelet Transparency" (2021).
 *   Build pass     (section 2.1 step 2; closed forms of section 2.3.1): every transparent fragment adds its
 *                  Haar coefficients of absorbance a = -ln(1 - alpha) over normalised depth into a fixed-size
 *                  per-pixel array, in any order.
 *   Evaluate pass  (section 2.1 step 3; compositing sum of section 2.2; interpolation of section 2.3.2):
 *                  visibility v = exp(-A~(x)) is reconstructed at each fragment's depth and the
 *                  visibility-weighted colour alpha * rgb * v is accumulated, together with sum(a).
 *   Resolve        (section 2.1 step 4): out = accumulated colour + background * exp(-sum(a)).
 *
 * Conventions shared by every entry point
 *   - All pointers to per-frame data are DEVICE pointers (HIP device memory of the current device) unless a
 *     parameter says "host". The library never allocates persistent memory and never frees caller memory;
 *     scratch comes from a caller-provided device workspace sized by wt_workspace_bytes(), except for
 *     wt_render_noalloc, which uses a static per-GPU device array instead.
 *   - Every call is asynchronous on the given HIP stream (0 = the null stream) and returns once the work is
 *     enqueued. The return code reports host-side validation and launch failures only.
 *   - Errors: WT_ERR_INVALID (null pointer, bad enum, zero size), WT_ERR_RANGE (size limits: rank > 10,
 *     pixel count >= 2^32, fragment count > WT_MAX_FRAGMENTS, workspace too small), WT_ERR_HIP (a HIP runtime
 *     error; the HIP error string is in wt_last_error()). Nothing is enqueued when validation fails.
 *   - Device-side bad fragments are dropped, not faulted: a pixel id >= width*height, a NaN depth or a NaN
 *     alpha. Their number is read back with wt_dropped_count(). Depth is clamped to [0, 1]; alpha to
 *     [0, 1 - 2^-24].
 *   - The library is stateless and re-entrant; calls that share a workspace must be ordered on one stream.
 *   - A workspace records on the device what was binned into it. A call over a binned stream (wt_*_binned, and
 *     the passes inside wt_build, wt_evaluate, wt_render, wt_backward) checks, before it reads a table or a record,
 *     that the workspace holds a complete binning made under the same description and ws_bytes, with the record
 *     format it reads; otherwise it computes nothing and leaves its outputs untouched. wt_bin_scatter writes only
 *     after a wt_bin_count of the same stream (count and the four array addresses) under the same description
 *     and ws_bytes, and stops writing if a tile would receive more fragments than were counted (the stream's
 *     contents changed in between). Such refusals happen on the device; wt_dropped_count reports them.
 *
 * Data layout (row-major, little endian)
 *   fragments  structure of arrays, F = count entries:
 *                pixel[F] uint32 = y * width + x;  depth[F] float;  alpha[F * channels] float
 *                (channel-minor);  rgb[F * 3] float, straight (not premultiplied) colour.
 *   coeffs     [P][channels][M] of the storage type (M = 2^(rank+1)); element m = 0 holds the scaling
 *              coefficient chi_00, element m = 2^n + k holds 2^(n/2) X_{n,k} (level n = 0..rank).
 *   accum      float [P][4] for channels = 1: (sum alpha r v, sum alpha g v, sum alpha b v, sum a);
 *              float [P][8] for channels = 3: (sum alpha_r r v_r, .._g, .._b, 0, sum a_r, sum a_g, sum a_b, 0).
 *   out        float [P][3] linear RGB, no clamp.
 */
#ifndef WT_H
#define WT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

/* Largest fragment count a call takes: 2^32 - 2^20. Binned records are addressed by 32-bit indices, and a kernel's
 * loop over a tile's records may step up to 8,192 records past its last one before it stops, so counts stop well
 * short of 2^32 (larger counts are refused with WT_ERR_RANGE, and wt_workspace_bytes returns 0 for them). */
#define WT_MAX_FRAGMENTS 4293918720ull

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WT_OK = 0,
  WT_ERR_INVALID = -1,
  WT_ERR_RANGE = -2,
  WT_ERR_NOMEM = -3,
  WT_ERR_HIP = -4,
  WT_ERR_UNSUPPORTED = -5
} wt_status;

/* Storage type of the coefficient array. On-chip sums are FP64; FP32, FP16 and BF16 round once, to nearest
 * even, when a coefficient tile is stored, and widen exactly when it is loaded.
 * WT_E5B9G9R9 is the packed storage of section 2.1 for three channels: coefficient m of the three channels
 * shares one 32-bit word, a 5-bit exponent e (bits 27-31, bias 15) and three 9-bit mantissas without an
 * implicit one (B bits 18-26, G 9-17, R 0-8), value = mantissa * 2^(e - 24). Only magnitudes are stored: the
 * closed forms of section 2.3.1 fix the signs (coefficient 0 is >= 0, every other one <= 0). The encoding is
 * the shared-exponent texture format: values clamp to [0, 65408], the exponent is the smallest that holds the
 * largest of the three in 9 bits after rounding half up, each mantissa rounds half up. Requires channels == 3
 * and rank <= 4; the coefficient array is then P * M words ([P][M]). */
typedef enum { WT_F32 = 0, WT_F16 = 1, WT_BF16 = 2, WT_E5B9G9R9 = 3 } wt_dtype;

/* wt_frame_desc.flags.
 * WT_TIGHT_DEPTH: per-pixel depth bounds (section 2.1, step 1). Before the build, each pixel's clamped depths are
 * mapped onto its own range, x' = (x - zmin) / (zmax - zmin) (0 when every fragment of the pixel has the same
 * depth), and the build, evaluate and gradient use x'. zmin and zmax are taken over the fragments one call sees,
 * so with this flag a frame's stream is passed whole to each call (no chunked accumulation). */
#define WT_TIGHT_DEPTH 1u
/* WT_TEMPORAL: the frame is rendered in one pass against the previous frame's coefficients
 * (wt_render_temporal). Screen tiles are sized for that kernel's working set, so a stream binned under a
 * WT_TEMPORAL description serves wt_render_temporal_binned; the other entry points accept the flag as well (smaller
 * tiles, same results). Requires rank <= 4 and excludes WT_TIGHT_DEPTH (WT_ERR_UNSUPPORTED). */
#define WT_TEMPORAL 2u
/* WT_DETERMINISTIC: a debug mode whose results are bit-identical from run to run for the same stream. The binning
 * copies the stream in stream order with a single thread, and each tile's fragments are applied one after another,
 * in that order, by a single thread of the tile's workgroup (no two updates of a sum race). Much slower than the
 * default; meant for tests and for telling a race from rounding (results differ from the default mode only in the
 * order of the FP64 on-chip sums). Combines with the other flags. */
#define WT_DETERMINISTIC 4u

typedef struct {
  uint32_t width;       /* pixels per row, >= 1 */
  uint32_t height;      /* rows, >= 1; width * height < 2^32 */
  uint32_t rank;        /* N in 0..10: levels n = 0..N, M = 2^(N+1) coefficients per channel */
  uint32_t channels;    /* 1 (one visibility for r, g, b) or 3 (per-channel transmittance) */
  uint32_t coeff_dtype; /* wt_dtype */
  uint32_t flags;       /* 0 or WT_TIGHT_DEPTH or WT_TEMPORAL, optionally with WT_DETERMINISTIC */
} wt_frame_desc;

typedef struct {
  uint64_t count;       /* F <= WT_MAX_FRAGMENTS */
  const uint32_t* pixel;
  const float* depth;
  const float* alpha;
  const float* rgb;
} wt_fragments;

/* Bytes of device workspace needed for frames of this description with up to max_fragments fragments.
 * Returns 0 for an invalid description. */
size_t wt_workspace_bytes(const wt_frame_desc* desc, uint64_t max_fragments);

/* Ingest and screen-tile binning (a device-side regrouping of the stream so that each pixel's fragments
 * are processed on one compute unit; it stands in for the screen locality of a raster pipeline). Copies the
 * stream into the workspace grouped by screen tile, dropping and counting bad fragments. The binned copy
 * stays valid until the workspace is reused and serves any number of wt_*_binned calls with the same desc
 * and ws_bytes. */
wt_status wt_bin(const wt_frame_desc* desc, const wt_fragments* frags, void* ws, size_t ws_bytes,
                 hipStream_t stream);

/* The two halves of wt_bin, for callers that time or schedule them separately: wt_bin_count zeroes the
 * drop counter, counts fragments per screen tile and lays out the tile segments; wt_bin_scatter then copies
 * the stream into them. wt_bin_scatter must follow wt_bin_count on the same stream with the same arguments and
 * unchanged fragment arrays (checked on the device, see the conventions above). */
wt_status wt_bin_count(const wt_frame_desc* desc, const wt_fragments* frags, void* ws, size_t ws_bytes,
                       hipStream_t stream);
wt_status wt_bin_scatter(const wt_frame_desc* desc, const wt_fragments* frags, void* ws, size_t ws_bytes,
                         hipStream_t stream);

/* Build pass over a binned stream (section 2.3.1): coeffs += the coefficients of every binned fragment.
 * coeffs must hold P * channels * M elements of desc->coeff_dtype; the caller zeroes it before the first
 * contribution of a frame. */
wt_status wt_build_binned(const wt_frame_desc* desc, void* coeffs, const void* ws, size_t ws_bytes,
                          hipStream_t stream);

/* Evaluate pass over a binned stream (sections 2.2, 2.3.2): accum += the visibility-weighted colour and
 * absorbance of every binned fragment, reconstructed from complete coefficients. */
wt_status wt_evaluate_binned(const wt_frame_desc* desc, const void* coeffs, float* accum, const void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* wt_bin followed by wt_build_binned. Calls accumulate, so a long stream can be built in chunks. */
wt_status wt_build(const wt_frame_desc* desc, const wt_fragments* frags, void* coeffs, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/* wt_bin followed by wt_evaluate_binned. */
wt_status wt_evaluate(const wt_frame_desc* desc, const wt_fragments* frags, const void* coeffs, float* accum,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/* Composite (section 2.1 step 4): out[p] = accum colour + bg * exp(-sum a); bg_rgb is a HOST array of 3. */
wt_status wt_resolve(const wt_frame_desc* desc, const float* accum, const float* bg_rgb, float* out,
                     hipStream_t stream);

/* Composite over a background IMAGE with the chromatic-aberration gather of section 3 (instead of wt_resolve's
 * constant colour). Each pixel's background is gathered along its screen-space refraction offset (accumulated by
 * the renderer's shading): `taps` bilinear samples (clamp-to-edge addressing; pixel (x, y) has its centre at
 * (x + 0.5, y + 0.5)) at the centre plus s_i * offset, s_i = 1 + dispersion * (t_i - 1/2), t_i = i / (taps - 1),
 * so the segment is centred on the single refracted sample and spans dispersion times the offset. Channel q takes
 * the mean of the taps under its spectral weight: red = smoothstep formula u^2 (3 - 2u), u = clamp((t - 1/2) /
 * (1/3 - 1/2), 0, 1) (1 for t <= 1/3, 0 for t >= 1/2), blue the same with edges 1/2 and 2/3 (0 for t <= 1/2,
 * 1 for t >= 2/3), green = 1 - red - blue; red samples the least displaced end, blue the most.
 * out[p][q] = accum colour + exp(-sum a) * sum_i w_q(t_i) sample_i[q] / sum_i w_q(t_i). With a zero offset, or
 * dispersion 0 and a constant image, this is wt_resolve over that background.
 *   accum       [P][4] or [P][8] as written by wt_evaluate; 16-byte aligned.
 *   background  float [P][3] device image, row-major like out.
 *   offset      float [P][2] device, (dx, dy) in pixels; 8-byte aligned.
 *   dispersion  finite; taps odd, 3..63 (WT_ERR_INVALID otherwise; odd counts sample t = 1/2, where green
 *               has its weight). out [P][3] is overwritten. */
wt_status wt_resolve_chromatic(const wt_frame_desc* desc, const float* accum, const float* background,
                               const float* offset, float dispersion, uint32_t taps, float* out, hipStream_t stream);

/* The whole path for one frame in one pass over the binned stream: bin, build, evaluate and resolve, with
 * the per-pixel state held on chip. Writes out[P][3] (overwritten) and, if coeffs is not NULL, the frame's
 * coefficients (overwritten). The evaluation sees the coefficients at storage precision, exactly as a
 * build/evaluate pair through a stored coefficient array would. bg_rgb is a HOST array of 3. */
wt_status wt_render(const wt_frame_desc* desc, const wt_fragments* frags, const float* bg_rgb, void* coeffs,
                    float* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of the per-GPU device array that wt_render_noalloc bins into (256 MiB). */
#define WT_SCRATCH_BYTES ((size_t)256 << 20)

/* wt_render for callers that cannot allocate device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc. Same arguments, kernels and results as wt_render, without the workspace: the
 * binned stream and the tile tables go to a static device array of WT_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends (its address is looked up once per device, on the first call with that
 * device current). Nothing is allocated or freed, by the library or by any routine it calls.
 *   Limit: a frame whose workspace (wt_workspace_bytes(desc, frags->count) without the gradient's layout) exceeds
 *   WT_SCRATCH_BYTES is refused with WT_ERR_RANGE before anything is enqueued: about 9.5 million fragments at one
 *   channel (28 bytes per binned fragment) and 7.4 million at three (36 bytes), half as many for frames of more than
 *   4096 screen tiles (binned in two levels, each with its own copy).
 *   Sharing: every call on one GPU uses that GPU's one array, which keeps the last call's contents (each call clears
 *   what it needs zeroed with its own fill kernels). Calls that overlap in time on one GPU (on different streams, or
 *   from different threads without ordering) race on the array: the caller serialises them, for example on one
 *   stream. The drop count of such a call is not reported (wt_dropped_count reads a caller's workspace). */
wt_status wt_render_noalloc(const wt_frame_desc* desc, const wt_fragments* frags, const float* bg_rgb, void* coeffs,
                            float* out, hipStream_t stream);

/* The build, evaluate and resolve of wt_render over a stream already binned into ws by wt_bin (same desc and
 * ws_bytes). Writes out[P][3] and, if coeffs is not NULL, the coefficients (both overwritten). */
wt_status wt_render_binned(const wt_frame_desc* desc, const void* ws, size_t ws_bytes, const float* bg_rgb,
                           void* coeffs, float* out, hipStream_t stream);

/* One-pass render against the previous frame's coefficients: the single-pass variant proposed as future work
 * in the paper's closing section. The frame's coefficients are built in the same pass that shades its fragments,
 * so the shading cannot see them: each fragment's visibility is reconstructed (sections 2.3, 2.3.2) from the
 * PREVIOUS frame's coefficients, read at the pixel's reprojected position. Every binned record is read once
 * instead of twice.
 *   desc         must carry WT_TEMPORAL (WT_ERR_INVALID otherwise); rank <= 4.
 *   prev_coeffs  the previous frame's coefficients, same layout and storage type as coeffs ([P][C][M], or [P][M]
 *                words for WT_E5B9G9R9), or NULL for a first frame (no history anywhere).
 *   prev_pixel   uint32 [P] or NULL: pixel p reads the previous buffer at prev_pixel[p] (a reprojection computed
 *                by the caller); NULL reads p itself. An entry >= P means that p has no history.
 *   coeffs       this frame's coefficients (overwritten), for the next frame; may be NULL. It may be the same
 *                buffer as prev_coeffs when prev_pixel is NULL (each tile reads the previous coefficients of its
 *                own pixels before it writes them); with a map the two must not overlap (WT_ERR_INVALID when
 *                they are equal).
 *   out          [P][3] (overwritten): sum of alpha rgb exp(-A~_prev(x)) + bg * exp(-sum a), with sum a over this
 *                frame's fragments. A pixel with no history sees nothing in front of its fragments (v = 1).
 *   bg_rgb is a HOST array of 3. Depth is used as given (no per-pixel bounds: the previous coefficients were
 *   built over the previous frame's range). */
wt_status wt_render_temporal(const wt_frame_desc* desc, const wt_fragments* frags, const float* bg_rgb,
                             const void* prev_coeffs, const uint32_t* prev_pixel, void* coeffs, float* out, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* wt_render_temporal over a stream already binned into ws by wt_bin (same WT_TEMPORAL desc and ws_bytes). */
wt_status wt_render_temporal_binned(const wt_frame_desc* desc, const void* ws, size_t ws_bytes, const float* bg_rgb,
                                    const void* prev_coeffs, const uint32_t* prev_pixel, void* coeffs, float* out,
                                    hipStream_t stream);

/* Gradient of a scalar loss through wt_render with respect to alpha and colour. grad_out is dL/dout
 * [P][3]; coeffs are the frame's complete coefficients and accum its accumulation (as written by wt_build
 * and wt_evaluate, or recomputed). Writes grad_alpha[F * channels] and grad_rgb[F * 3] (overwritten, in
 * stream order). Depth is not differentiated (A~ has kinks on the subdivision grid). The clamp of alpha has
 * zero slope outside (0, 1 - 2^-24); dropped fragments get zero gradients. bg_rgb is a HOST array of 3.
 * It bins frags into ws in the gradient's own layout (smaller tiles, records that keep alpha), so a stream binned
 * there before for wt_*_binned calls is gone: bin again before the next such call. */
wt_status wt_backward(const wt_frame_desc* desc, const wt_fragments* frags, const void* coeffs, const float* accum,
                      const float* bg_rgb, const float* grad_out, float* grad_alpha, float* grad_rgb, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* Number of fragments dropped by the last binning in this workspace. Synchronises the given stream. Returns
 * WT_ERR_INVALID (with *count still written) when a call on this workspace was refused on the device since the last
 * report: a call over the binned stream that found no complete binning for its description and ws_bytes, or a
 * scatter that did not belong to the count before it; wt_last_error() names which, and the report is cleared. */
wt_status wt_dropped_count(const void* ws, size_t ws_bytes, uint64_t* count, hipStream_t stream);

/* Thread-local message describing the last non-OK status returned on this thread ("" if none). */
const char* wt_last_error(void);

/* ABI version of this header: increments on any incompatible change. */
int wt_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WT_H */
