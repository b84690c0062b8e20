/*
 * wt_oracle.c -- FP64 CPU oracle for the wavelet-transparency resolve.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this
 * library. It shares no code, header, table or helper with the HIP path and must never be used to produce
 * a product result.
 *
 * Source: M. Aizenshtein, N. Smal, M. McGuire, "Wavelet Transparency" (2021).
 *   section 1.2  (The Visibility Function)  -- v(x), the single 25%-opaque layer example
 *   section 2.1  (Overview)                 -- build pass, shade pass weighted by v, composite
 *   section 2.2  (Derivation)               -- L = sum_i L_i r_i v(x_i); A = -log v; A = sum a_i theta(x - x_i)
 *   section 2.3  (Wavelet approximation)    -- A ~ chi_00 phi_00 + sum X_nk psi_nk
 *   section 2.3.1 (Coefficients)            -- chi_00 = sum a_i (1 - x_i); X_nk = -sum a_i Psi_nk(x_i)
 *   section 2.3.2 (Interpolation)           -- linear interpolation between the subdivision points
 *
 * Readings taken where the paper is silent or garbled (each is listed in the design notes):
 *   - The step of A at an interface is a_i = -ln(1 - alpha_i): the worked example of section 1.2 (v = 0.75
 *     behind a 25%-opaque plane) requires it, and A = -log v makes the log natural.
 *   - "Rank N" keeps the scaling function and wavelet levels n = 0..N: 2^(N+1) coefficients per channel,
 *     matching the storage count of section 2.1.
 *   - Depth lives on [0,1] (the integration range of section 2.3.1); inputs are clamped to it.
 *   - Interpolation: the subdivision point (j+1)/M carries the average of cell j and the point 0 carries 0;
 *     A~ is the piecewise-linear curve through (0,0), (1/M, Abar_0), ..., (1, Abar_{M-1}).
 *   - Background transmittance is exp(-sum_i a_i) (the exact net coverage product).
 *   - Each fragment contributes alpha_i * c_i * v(x_i) with straight (not premultiplied) colour c_i.
 *   - alpha is clamped to [0, 1 - 2^-24]; fragments with a pixel id >= W*H or a NaN depth/alpha are dropped.
 *   - Exact A-buffer: equal depths do not occlude each other (strict inequality).
 *
 * Stored coefficient layout per pixel and channel (M = 2^(N+1) doubles):
 *   m = 0          : chi_{0,0}
 *   m = 2^n + k    : d_{n,k} = 2^(n/2) X_{n,k}   (level-scaled, so that synthesis is plain +/- sums)
 *
 * Every per-pixel sum runs over that pixel's fragments in a canonical order (depth, alpha, colour, stream
 * index), so the result does not depend on the order of the input stream, bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)

/* ------------------------------------------------------------------------------------------------ */
/* Scalars                                                                                          */
/* ------------------------------------------------------------------------------------------------ */

static const double ALPHA_MAX = 1.0 - 1.0 / 16777216.0; /* 1 - 2^-24 */

/* alpha as used by the method: clamped to [0, 1 - 2^-24] (a NaN never reaches here). */
double orc_alpha_used(double alpha) {
  if (!(alpha > 0.0)) return 0.0;
  if (alpha > ALPHA_MAX) return ALPHA_MAX;
  return alpha;
}

/* Absorbance step of one interface, a = -ln(1 - alpha) (section 2.2, A = -log v, with the section 1.2
 * example fixing the step size). */
double orc_absorbance(double alpha) { return -log1p(-orc_alpha_used(alpha)); }

static double clamp_depth(double x) {
  if (!(x > 0.0)) return 0.0;
  if (x > 1.0) return 1.0;
  return x;
}

/* Depths of one pixel's fragments as the method uses them. With tight bounds (section 2.1, step 1: a depth
 * buffer pass records each pixel's nearest and farthest transparent depth before the coefficients are built),
 * the clamped depths are mapped affinely so that the pixel's range [zmin, zmax] becomes [0, 1]:
 * x' = (x - zmin) / (zmax - zmin). Reading: the paper names the bounds but not the mapping; linear depth
 * (section 2.3's choice) makes the affine map the natural one, and a pixel whose fragments share one depth
 * maps them to 0. */
static void pixel_depths(const float* depth, const uint32_t* order, uint64_t k, int tight, double* xs) {
  double lo = 1.0, hi = 0.0;
  for (uint64_t r = 0; r < k; ++r) {
    xs[r] = clamp_depth(depth[order[r]]);
    if (xs[r] < lo) lo = xs[r];
    if (xs[r] > hi) hi = xs[r];
  }
  if (!tight) return;
  for (uint64_t r = 0; r < k; ++r) xs[r] = hi > lo ? (xs[r] - lo) / (hi - lo) : 0.0;
}

/* 2^(e/2) for integer e, the level normalisation of the orthonormal Haar basis (2^(n/2) psi(2^n x - k)). */
static double half_pow2(int e) {
  double r = ldexp(1.0, e / 2 - (e < 0 && (e & 1) ? 1 : 0)); /* 2^floor(e/2) */
  if (e & 1) r *= 1.4142135623730951;                          /* times sqrt(2) for odd e */
  return r;
}

/* Psi_{n,k}(x) of section 2.3.1: the antiderivative of the orthonormal Haar wavelet psi_{n,k}, a tent of
 * height 2^(-n/2) / 2 on [k/2^n, (k+1)/2^n]. */
double orc_Psi(int n, int k, double x) {
  double s = ldexp(1.0, n); /* 2^n */
  double u = s * x - (double)k;
  double scale = half_pow2(-n);
  if (u >= 0.0 && u < 0.5) return scale * u;
  if (u >= 0.5 && u <= 1.0) return scale * (1.0 + (double)k - s * x);
  return 0.0;
}

/* psi_{n,k}(z): orthonormal Haar wavelet, +2^(n/2) on the first half of its support, -2^(n/2) on the second. */
double orc_psi(int n, int k, double z) {
  double s = ldexp(1.0, n);
  double u = s * z - (double)k;
  double h = half_pow2(n);
  if (u >= 0.0 && u < 0.5) return h;
  if (u >= 0.5 && u < 1.0) return -h;
  return 0.0;
}

/* Round to a binary format with `mbits` fraction bits and minimum normal exponent `emin`, to nearest with
 * ties to even (IEEE 754 roundTiesToEven). mbits = 10, emin = -14, emax = 15: binary16 (FP16);
 * mbits = 7, emin = -126, emax = 127: bfloat16. Values beyond the largest finite number become infinite. */
static double round_format(double v, int mbits, int emin, int emax) {
  if (v == 0.0 || isnan(v) || isinf(v)) return v;
  int e;
  frexp(fabs(v), &e); /* |v| = f 2^e, f in [0.5, 1): exponent of the leading bit is e - 1 */
  int lead = e - 1;
  if (lead < emin) lead = emin; /* subnormal range: fixed spacing */
  double ulp = ldexp(1.0, lead - mbits);
  double r = nearbyint(v / ulp) * ulp; /* default rounding mode: to nearest, ties to even */
  double maxfin = ldexp(2.0 - ldexp(1.0, -mbits), emax);
  if (fabs(r) > maxfin) return v > 0 ? INFINITY : -INFINITY;
  return r;
}

/* Coefficient storage precision: 0 = exact (FP64 here), 1 = FP16, 2 = BF16. (3, the shared-exponent packing
 * below, works on coefficient triples and is applied by orc_round_triple.) */
double orc_round_storage(double v, int storage) {
  if (storage == 1) return round_format(v, 10, -14, 15);
  if (storage == 2) return round_format(v, 7, -126, 127);
  return v;
}

/* Shared-exponent packing of three non-negative values into 32 bits, the E5B9G9R9 coefficient storage of
 * section 2.1: a 5-bit exponent in the top bits, then three 9-bit mantissas (B, G, R from high to low bits)
 * without an implicit leading one. The encoding is the published shared-exponent texture format (exponent
 * bias 15, 9 mantissa bits): clamp each value to [0, 511/512 * 2^16] (NaN to 0); take the shared exponent from
 * the largest, e' = max(-16, floor(log2 max)) + 1 + 15; if max rounds to 512 at that exponent, use e' + 1;
 * each mantissa is floor(value / 2^(e - 24) + 1/2). Reading: the paper names the packing and defers its bit
 * layout to a code supplement that is not available; the inputs are FP32 values (the precision in which the
 * GPU path forms them), and every step below is exact in FP64. */
uint32_t orc_pack_e5b9g9r9(float r, float g, float b) {
  const double vmax = 511.0 / 512.0 * 65536.0;
  double v[3] = {r, g, b};
  double mx = 0.0;
  for (int q = 0; q < 3; ++q) {
    if (!(v[q] > 0.0)) v[q] = 0.0; /* negative and NaN */
    if (v[q] > vmax) v[q] = vmax;
    if (v[q] > mx) mx = v[q];
  }
  int lead = -16;
  if (mx > 0.0) {
    int e;
    frexp(mx, &e); /* mx = f 2^e, f in [0.5, 1): floor(log2 mx) = e - 1 */
    if (e - 1 > lead) lead = e - 1;
  }
  int es = lead + 1 + 15;
  if (floor(ldexp(mx, 24 - es) + 0.5) == 512.0) es += 1;
  uint32_t w = (uint32_t)es << 27;
  for (int q = 0; q < 3; ++q) {
    uint32_t m = (uint32_t)floor(ldexp(v[q], 24 - es) + 0.5);
    w |= m << (9 * q); /* R in bits 0-8, G in 9-17, B in 18-26 */
  }
  return w;
}

void orc_unpack_e5b9g9r9(uint32_t w, double out[3]) {
  const int es = (int)(w >> 27);
  for (int q = 0; q < 3; ++q) out[q] = ldexp((double)((w >> (9 * q)) & 511u), es - 24);
}

/* Storage 3 for one coefficient of three channels: magnitudes packed and unpacked, signs restored (chi >= 0 and
 * d <= 0 are fixed by the closed forms of section 2.3.1, so only magnitudes are stored). */
void orc_round_triple(double* c0, double* c1, double* c2, int negative) {
  const double sg = negative ? -1.0 : 1.0;
  double out[3];
  orc_unpack_e5b9g9r9(orc_pack_e5b9g9r9((float)(sg * *c0), (float)(sg * *c1), (float)(sg * *c2)), out);
  *c0 = sg * out[0];
  *c1 = sg * out[1];
  *c2 = sg * out[2];
}

/* ------------------------------------------------------------------------------------------------ */
/* One pixel, one channel: coefficients, cell averages, reconstruction                              */
/* ------------------------------------------------------------------------------------------------ */

/* Section 2.3.1 closed forms. x[] are clamped depths, a[] absorbance steps; coef[] receives the stored
 * layout described at the top of the file (M = 2^(rank+1) entries). The sums run in array order. */
void orc_coeffs_one(int rank, int nfr, const double* x, const double* a, double* coef) {
  int M = 1 << (rank + 1);
  memset(coef, 0, sizeof(double) * (size_t)M);
  for (int i = 0; i < nfr; ++i) {
    /* chi_{0,0} = sum a_i (1 - x_i) */
    coef[0] += a[i] * (1.0 - x[i]);
    /* X_{n,k} = -sum a_i Psi_{n,k}(x_i); only the one k whose support holds x_i is non-zero (the last
     * support is closed at x = 1). Stored as 2^(n/2) X_{n,k}. */
    for (int n = 0; n <= rank; ++n) {
      int s = 1 << n;
      int k = (int)floor(s * x[i]);
      if (k > s - 1) k = s - 1;
      double X = -a[i] * orc_Psi(n, k, x[i]);
      coef[s + k] += half_pow2(n) * X;
    }
  }
}

/* The Haar expansion of section 2.3, chi phi_00 + sum X_nk psi_nk, is constant on each of the M cells of
 * width 1/M; its value there (evaluated at the cell centre) is the cell average Abar_j. */
void orc_cells_one(int rank, const double* coef, double* cells) {
  int M = 1 << (rank + 1);
  for (int j = 0; j < M; ++j) {
    double z = ((double)j + 0.5) / (double)M;
    double A = coef[0]; /* phi_00 = 1 on [0,1] */
    for (int n = 0; n <= rank; ++n) {
      int s = 1 << n;
      int k = (int)floor(s * z); /* the only wavelet of level n whose support holds z */
      double X = half_pow2(-n) * coef[s + k];
      A += X * orc_psi(n, k, z);
    }
    cells[j] = A;
  }
}

/* Section 2.3.2 interpolation: piecewise linear through (0, 0) and ((j+1)/M, Abar_j). */
double orc_reconstruct(int rank, const double* cells, double z) {
  int M = 1 << (rank + 1);
  double u = (double)M * z;
  int j = (int)floor(u);
  if (j > M - 1) j = M - 1;
  if (j < 0) j = 0;
  double t = u - (double)j;
  double lo = (j == 0) ? 0.0 : cells[j - 1];
  return (1.0 - t) * lo + t * cells[j];
}

/* ------------------------------------------------------------------------------------------------ */
/* Frame-level helpers                                                                              */
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
  uint32_t width, height, rank, channels;
  uint64_t count;
  const uint32_t* pixel;
  const float* depth;
  const float* alpha; /* [count * channels] */
  const float* rgb;   /* [count * 3] */
} orc_stream;

static int frag_valid(const orc_stream* s, uint64_t i) {
  uint64_t P = (uint64_t)s->width * s->height;
  if (s->pixel[i] >= P) return 0;
  if (isnan(s->depth[i])) return 0;
  for (uint32_t c = 0; c < s->channels; ++c)
    if (isnan(s->alpha[i * s->channels + c])) return 0;
  return 1;
}

/* Canonical order inside a pixel: depth, then alpha, then colour, then stream index. */
static const orc_stream* g_sort_stream; /* set per call; comparator context (qsort has none) */
#ifdef _OPENMP
#pragma omp threadprivate(g_sort_stream)
#endif
static int cmp_frag(const void* pa, const void* pb) {
  const orc_stream* s = g_sort_stream;
  uint32_t ia = *(const uint32_t*)pa, ib = *(const uint32_t*)pb;
  double xa = clamp_depth(s->depth[ia]), xb = clamp_depth(s->depth[ib]);
  if (xa != xb) return xa < xb ? -1 : 1;
  for (uint32_t c = 0; c < s->channels; ++c) {
    double aa = s->alpha[(uint64_t)ia * s->channels + c], ab = s->alpha[(uint64_t)ib * s->channels + c];
    if (aa != ab) return aa < ab ? -1 : 1;
  }
  for (int c = 0; c < 3; ++c) {
    double ca = s->rgb[(uint64_t)ia * 3 + c], cb = s->rgb[(uint64_t)ib * 3 + c];
    if (ca != cb) return ca < cb ? -1 : 1;
  }
  return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* Group fragment indices by pixel (counting sort). start has P+1 entries. Pixels with mask[p] == 0 are
 * skipped when a mask is given. Returns the number of dropped fragments via *dropped. */
static int group_by_pixel(const orc_stream* s, const uint8_t* mask, uint64_t** start_out, uint32_t** idx_out,
                          uint64_t* dropped) {
  uint64_t P = (uint64_t)s->width * s->height;
  uint64_t* start = (uint64_t*)calloc(P + 1, sizeof(uint64_t));
  if (!start) return ORC_ENOMEM;
  uint64_t nd = 0;
  for (uint64_t i = 0; i < s->count; ++i) {
    if (!frag_valid(s, i)) { ++nd; continue; }
    uint32_t p = s->pixel[i];
    if (mask && !mask[p]) continue;
    start[p + 1]++;
  }
  for (uint64_t p = 0; p < P; ++p) start[p + 1] += start[p];
  uint32_t* idx = (uint32_t*)malloc(sizeof(uint32_t) * (start[P] ? start[P] : 1));
  uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * (P ? P : 1));
  if (!idx || !fill) { free(start); free(idx); free(fill); return ORC_ENOMEM; }
  memcpy(fill, start, sizeof(uint64_t) * P);
  for (uint64_t i = 0; i < s->count; ++i) {
    if (!frag_valid(s, i)) continue;
    uint32_t p = s->pixel[i];
    if (mask && !mask[p]) continue;
    idx[fill[p]++] = (uint32_t)i;
  }
  free(fill);
  *start_out = start;
  *idx_out = idx;
  *dropped = nd;
  return ORC_OK;
}

static uint64_t max_run(const uint64_t* start, uint64_t P) {
  uint64_t m = 0;
  for (uint64_t p = 0; p < P; ++p) if (start[p + 1] - start[p] > m) m = start[p + 1] - start[p];
  return m;
}

/* ------------------------------------------------------------------------------------------------ */
/* The wavelet resolve of a whole frame                                                             */
/* ------------------------------------------------------------------------------------------------ */

/*
 * orc_resolve: build (section 2.3.1), cell averages and interpolation (2.3, 2.3.2), shading weighted by
 * visibility (2.1 step 3, 2.2 compositing sum), composite over a constant background (2.1 step 4).
 *
 *   coeffs [P][C][M]  stored coefficients (may be NULL)
 *   cells  [P][C][M]  cell averages Abar_j (may be NULL)
 *   accum  [P][3]     S_q = sum_i alpha_{i,c(q)} c_{i,q} v_{i,c(q)}     (may be NULL)
 *   suma   [P][C]     sum_i a_{i,c}                                      (may be NULL)
 *   out    [P][3]     S_q + bg_q exp(-suma_{c(q)})                        (may be NULL)
 *   vis    [F][C]     v_{i,c} = exp(-A~_c(x_i)); NaN for dropped fragments (may be NULL)
 * with c(q) = q when C = 3 and 0 when C = 1. storage != 0 rounds every coefficient to FP16 (1) or BF16 (2), or
 * packs the three channels' coefficient m into one E5B9G9R9 word (3, C = 3 only), before the cell averages are
 * formed (the method with coefficients kept at that precision). tight != 0 maps every pixel's depths onto its
 * own [zmin, zmax] first (pixel_depths).
 * mask (uint8 [P], may be NULL) restricts the pixels computed;
 * outputs of unmasked pixels are left untouched. threads <= 0 keeps the OpenMP default.
 */
int orc_resolve(uint32_t width, uint32_t height, uint32_t rank, uint32_t channels, uint64_t count,
                const uint32_t* pixel, const float* depth, const float* alpha, const float* rgb, const double* bg,
                const uint8_t* mask, int storage, int tight, double* coeffs, double* cells, double* accum, double* suma,
                double* out, double* vis, uint64_t* dropped, int threads) {
  if (rank > 12 || (channels != 1 && channels != 3) || (count && (!pixel || !depth || !alpha || !rgb)) || !bg ||
      storage < 0 || storage > 3 || (storage == 3 && channels != 3))
    return ORC_EINVAL;
  orc_stream s = {width, height, rank, channels, count, pixel, depth, alpha, rgb};
  uint64_t P = (uint64_t)width * height;
  int M = 1 << (rank + 1);
  int C = (int)channels;
  uint64_t* start;
  uint32_t* idx;
  uint64_t nd;
  int rc = group_by_pixel(&s, mask, &start, &idx, &nd);
  if (rc) return rc;
  if (dropped) *dropped = nd;
  if (vis)
    for (uint64_t i = 0; i < count; ++i)
      if (!frag_valid(&s, i))
        for (int c = 0; c < C; ++c) vis[i * C + c] = NAN;
  uint64_t kmax = max_run(start, P);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int fail = 0;
#pragma omp parallel
  {
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (kmax ? kmax : 1));
    double* xs = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    double* as = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    double* cfa = (double*)malloc(sizeof(double) * M * 3);
    double* ce = (double*)malloc(sizeof(double) * M);
    if (!order || !xs || !as || !cfa || !ce) {
#pragma omp atomic write
      fail = 1;
    } else {
      g_sort_stream = &s;
#pragma omp for schedule(dynamic, 256)
      for (int64_t p = 0; p < (int64_t)P; ++p) {
        if (mask && !mask[p]) continue;
        uint64_t k = start[p + 1] - start[p];
        memcpy(order, idx + start[p], sizeof(uint32_t) * k);
        qsort(order, k, sizeof(uint32_t), cmp_frag);
        double S[3] = {0.0, 0.0, 0.0};
        double sa[3] = {0.0, 0.0, 0.0};
        pixel_depths(depth, order, k, tight, xs);
        for (int c = 0; c < C; ++c) {
          for (uint64_t r = 0; r < k; ++r) as[r] = orc_absorbance(alpha[(uint64_t)order[r] * C + c]);
          orc_coeffs_one((int)rank, (int)k, xs, as, cfa + c * M);
          for (int m = 0; m < M; ++m) cfa[c * M + m] = orc_round_storage(cfa[c * M + m], storage);
        }
        if (storage == 3)
          for (int m = 0; m < M; ++m) orc_round_triple(cfa + m, cfa + M + m, cfa + 2 * M + m, m > 0);
        for (int c = 0; c < C; ++c) {
          for (uint64_t r = 0; r < k; ++r) as[r] = orc_absorbance(alpha[(uint64_t)order[r] * C + c]);
          double* cf = cfa + c * M;
          orc_cells_one((int)rank, cf, ce);
          if (coeffs) memcpy(coeffs + ((uint64_t)p * C + c) * M, cf, sizeof(double) * M);
          if (cells) memcpy(cells + ((uint64_t)p * C + c) * M, ce, sizeof(double) * M);
          for (uint64_t r = 0; r < k; ++r) {
            uint32_t i = order[r];
            double v = exp(-orc_reconstruct((int)rank, ce, xs[r]));
            double au = orc_alpha_used(alpha[(uint64_t)i * C + c]);
            if (vis) vis[(uint64_t)i * C + c] = v;
            sa[c] += as[r];
            if (C == 3) {
              S[c] += au * rgb[(uint64_t)i * 3 + c] * v;
            } else {
              for (int q = 0; q < 3; ++q) S[q] += au * rgb[(uint64_t)i * 3 + q] * v;
            }
          }
        }
        for (int q = 0; q < 3; ++q) {
          int c = (C == 3) ? q : 0;
          if (accum) accum[p * 3 + q] = S[q];
          if (out) out[p * 3 + q] = S[q] + bg[q] * exp(-sa[c]);
        }
        if (suma)
          for (int c = 0; c < C; ++c) suma[p * C + c] = sa[c];
      }
    }
    free(order); free(xs); free(as); free(cfa); free(ce);
  }
  free(start);
  free(idx);
  return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* Single pass against the previous frame's coefficients                                            */
/* ------------------------------------------------------------------------------------------------ */

/*
 * orc_shade_prev: the one-pass variant proposed as future work in the paper's closing section: the frame's
 * fragments are shaded in the same pass that builds its coefficients, so the visibility they see is
 * reconstructed from the PREVIOUS frame's coefficient buffer, read at each pixel's reprojected position.
 *
 *   prev        [Pp][C][M] the previous frame's stored coefficients (values as stored), or NULL: no history
 *   prev_pixel  [P] pixel of the previous buffer that pixel p reads (NULL: p itself); an entry >= Pp means
 *               that p has no history
 *   out, accum, suma, vis as in orc_resolve.
 *
 * Per pixel: cells of the previous coefficients (section 2.3; all zero without history), then for every
 * fragment v = exp(-A~_prev(x)) by the interpolation of section 2.3.2 and S += alpha c v (2.1 step 3). The
 * background weight uses this frame's own absorbance total, exp(-sum a) (2.1 step 4 with the reading taken in
 * orc_resolve): a plain sum over the frame's fragments that the single pass has in hand. Readings: the paper
 * leaves the reprojection to the renderer (here an integer pixel map supplied by the caller, identity by
 * default), and a pixel with no history (outside the guard band, disoccluded) sees nothing in front of it.
 * Depth is used as given (no per-pixel bounds: the previous buffer was built over the previous frame's range).
 */
int orc_shade_prev(uint32_t width, uint32_t height, uint32_t rank, uint32_t channels, uint64_t count,
                   const uint32_t* pixel, const float* depth, const float* alpha, const float* rgb, const double* bg,
                   const uint8_t* mask, const double* prev, const uint32_t* prev_pixel, uint64_t prev_pixels,
                   double* accum, double* suma, double* out, double* vis, uint64_t* dropped, int threads) {
  if (rank > 12 || (channels != 1 && channels != 3) || (count && (!pixel || !depth || !alpha || !rgb)) || !bg)
    return ORC_EINVAL;
  orc_stream s = {width, height, rank, channels, count, pixel, depth, alpha, rgb};
  uint64_t P = (uint64_t)width * height;
  int M = 1 << (rank + 1);
  int C = (int)channels;
  uint64_t* start;
  uint32_t* idx;
  uint64_t nd;
  int rc = group_by_pixel(&s, mask, &start, &idx, &nd);
  if (rc) return rc;
  if (dropped) *dropped = nd;
  if (vis)
    for (uint64_t i = 0; i < count; ++i)
      if (!frag_valid(&s, i))
        for (int c = 0; c < C; ++c) vis[i * C + c] = NAN;
  uint64_t kmax = max_run(start, P);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int fail = 0;
#pragma omp parallel
  {
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (kmax ? kmax : 1));
    double* xs = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    double* ce = (double*)malloc(sizeof(double) * M);
    if (!order || !xs || !ce) {
#pragma omp atomic write
      fail = 1;
    } else {
      g_sort_stream = &s;
#pragma omp for schedule(dynamic, 256)
      for (int64_t p = 0; p < (int64_t)P; ++p) {
        if (mask && !mask[p]) continue;
        uint64_t k = start[p + 1] - start[p];
        memcpy(order, idx + start[p], sizeof(uint32_t) * k);
        qsort(order, k, sizeof(uint32_t), cmp_frag);
        pixel_depths(depth, order, k, 0, xs);
        const uint64_t src = prev_pixel ? prev_pixel[p] : (uint64_t)p;
        const int history = prev != NULL && src < prev_pixels;
        double S[3] = {0.0, 0.0, 0.0};
        double sa[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < C; ++c) {
          if (history)
            orc_cells_one((int)rank, prev + (src * C + c) * M, ce);
          else
            memset(ce, 0, sizeof(double) * M);
          for (uint64_t r = 0; r < k; ++r) {
            uint32_t i = order[r];
            double v = exp(-orc_reconstruct((int)rank, ce, xs[r]));
            double al = alpha[(uint64_t)i * C + c];
            double au = orc_alpha_used(al);
            if (vis) vis[(uint64_t)i * C + c] = v;
            sa[c] += orc_absorbance(al);
            if (C == 3) {
              S[c] += au * rgb[(uint64_t)i * 3 + c] * v;
            } else {
              for (int q = 0; q < 3; ++q) S[q] += au * rgb[(uint64_t)i * 3 + q] * v;
            }
          }
        }
        for (int q = 0; q < 3; ++q) {
          int c = (C == 3) ? q : 0;
          if (accum) accum[p * 3 + q] = S[q];
          if (out) out[p * 3 + q] = S[q] + bg[q] * exp(-sa[c]);
        }
        if (suma)
          for (int c = 0; c < C; ++c) suma[p * C + c] = sa[c];
      }
    }
    free(order); free(xs); free(ce);
  }
  free(start);
  free(idx);
  return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* Composite with the chromatic-aberration gather (section 3)                                       */
/* ------------------------------------------------------------------------------------------------ */

/* GLSL smoothstep as a formula: u = clamp((x - e0) / (e1 - e0), 0, 1), u^2 (3 - 2u). With e0 > e1 (as printed
 * for the red weight) the formula is a falling step, 1 below e1 and 0 above e0. */
static double smoothstep_formula(double e0, double e1, double x) {
  double u = (x - e0) / (e1 - e0);
  if (u < 0.0) u = 0.0;
  if (u > 1.0) u = 1.0;
  return u * u * (3.0 - 2.0 * u);
}

/* Per-channel weight of gather tap i of k (section 3, the spectral weight of the compositing step). Reading of
 * the garbled listing: the tap parameter is t = i / (k - 1) in [0, 1] (the printed "0.5 + 2i/(k-1)" read as
 * "0.5 * 2i/(k-1)": with the printed sum every t >= 0.5 and red would never be sampled), and the smoothstep calls
 * are the formula above with the printed edges: red 1 for t <= 1/3 falling to 0 at t = 1/2, blue rising from 0 at
 * t = 1/2 to 1 at t >= 2/3, green the remainder 1 - red - blue. */
void orc_spectral_weight(int i, int k, double w[3]) {
  double t = (double)i / (double)(k - 1);
  w[0] = smoothstep_formula(0.5, 1.0 / 3.0, t);
  w[2] = smoothstep_formula(0.5, 2.0 / 3.0, t);
  w[1] = 1.0 - w[0] - w[2];
}

/* Bilinear sample of channel q of an image [H][W][3] at a position in pixel units (pixel (x, y) covers
 * [x, x+1) x [y, y+1), its centre at (x + 0.5, y + 0.5)), addresses clamped to the edge. */
static double bilinear(const float* img, uint32_t W, uint32_t H, double X, double Y, int q) {
  double u = X - 0.5, v = Y - 0.5;
  double fx0 = floor(u), fy0 = floor(v);
  double fx = u - fx0, fy = v - fy0;
  long x0 = (long)fx0, y0 = (long)fy0;
  long xs[2] = {x0, x0 + 1}, ys[2] = {y0, y0 + 1};
  for (int e = 0; e < 2; ++e) {
    if (xs[e] < 0) xs[e] = 0;
    if (xs[e] > (long)W - 1) xs[e] = (long)W - 1;
    if (ys[e] < 0) ys[e] = 0;
    if (ys[e] > (long)H - 1) ys[e] = (long)H - 1;
  }
  double a = img[((uint64_t)ys[0] * W + xs[0]) * 3 + q], b = img[((uint64_t)ys[0] * W + xs[1]) * 3 + q];
  double c = img[((uint64_t)ys[1] * W + xs[0]) * 3 + q], d = img[((uint64_t)ys[1] * W + xs[1]) * 3 + q];
  return (1.0 - fy) * ((1.0 - fx) * a + fx * b) + fy * ((1.0 - fx) * c + fx * d);
}

/*
 * orc_resolve_chromatic: the composite of section 2.1 step 4 with the background taken from an image through the
 * refraction offset and the chromatic-aberration gather of section 3. Per pixel p with centre c_p and refraction
 * offset delta_p (pixels; accumulated by the renderer's shading): k taps at c_p + s_i delta_p along the offset,
 * s_i = 1 + dispersion (t_i - 1/2), each a bilinear sample of the background; channel q of the background term is
 * the spectral-weighted mean sum_i w_q(t_i) sample_i[q] / sum_i w_q(t_i); out_q = S_q + T_q * that, with
 * T_q = exp(-suma_{c(q)}). Reading: the paper places the segment along the refraction offset, its length scaling
 * with the offset's; here it is centred on the single-sample position (s = 1) and spans dispersion x delta,
 * red (t = 0) displaced least and blue (t = 1) most, as normal dispersion bends shorter wavelengths more; the
 * weights of a channel are normalised so that a uniform background is unchanged. k must be odd and >= 3 (the
 * centre tap t = 1/2 is the one green tap for k = 3 .. 7).
 *   S [P][3], suma [P][C] (FP64), background [P][3], offset [P][2] (float), out [P][3].
 */
int orc_resolve_chromatic(uint32_t width, uint32_t height, uint32_t channels, const double* S, const double* suma,
                          const float* background, const float* offset, double dispersion, int taps, double* out) {
  if ((channels != 1 && channels != 3) || taps < 3 || !(taps & 1) || !S || !suma || !background || !offset || !out)
    return ORC_EINVAL;
  uint64_t P = (uint64_t)width * height;
  int C = (int)channels;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < (int64_t)P; ++p) {
    double cx = (double)(p % width) + 0.5, cy = (double)(p / width) + 0.5;
    double dx = offset[p * 2], dy = offset[p * 2 + 1];
    double num[3] = {0.0, 0.0, 0.0}, den[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < taps; ++i) {
      double w[3];
      orc_spectral_weight(i, taps, w);
      double s = 1.0 + dispersion * ((double)i / (double)(taps - 1) - 0.5);
      for (int q = 0; q < 3; ++q) {
        num[q] += w[q] * bilinear(background, width, height, cx + s * dx, cy + s * dy, q);
        den[q] += w[q];
      }
    }
    for (int q = 0; q < 3; ++q) {
      int c = (C == 3) ? q : 0;
      out[p * 3 + q] = S[p * 3 + q] + exp(-suma[p * C + c]) * num[q] / den[q];
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* Exact A-buffer (the reference the method approximates)                                           */
/* ------------------------------------------------------------------------------------------------ */

/*
 * orc_abuffer: per pixel and channel, V_i = prod_{j : x_j < x_i} (1 - alpha_j) (section 1.2 visibility,
 * strict inequality), out_q = sum_i alpha_{i,c(q)} c_{i,q} V_{i,c(q)} + bg_q prod_j (1 - alpha_{j,c(q)}).
 * brute != 0 evaluates every V_i by the O(k^2) product; otherwise fragments are walked in depth order with
 * a running product over groups of equal depth. vis [F][C] (may be NULL) receives V_i.
 */
int orc_abuffer(uint32_t width, uint32_t height, uint32_t channels, uint64_t count, const uint32_t* pixel,
                const float* depth, const float* alpha, const float* rgb, const double* bg, const uint8_t* mask,
                int brute, double* out, double* vis, uint64_t* dropped, int threads) {
  if ((channels != 1 && channels != 3) || (count && (!pixel || !depth || !alpha || !rgb)) || !bg || !out)
    return ORC_EINVAL;
  orc_stream s = {width, height, 0, channels, count, pixel, depth, alpha, rgb};
  uint64_t P = (uint64_t)width * height;
  int C = (int)channels;
  uint64_t* start;
  uint32_t* idx;
  uint64_t nd;
  int rc = group_by_pixel(&s, mask, &start, &idx, &nd);
  if (rc) return rc;
  if (dropped) *dropped = nd;
  if (vis)
    for (uint64_t i = 0; i < count; ++i)
      if (!frag_valid(&s, i))
        for (int c = 0; c < C; ++c) vis[i * C + c] = NAN;
  uint64_t kmax = max_run(start, P);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int fail = 0;
#pragma omp parallel
  {
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (kmax ? kmax : 1));
    double* V = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    if (!order || !V) {
#pragma omp atomic write
      fail = 1;
    } else {
      g_sort_stream = &s;
#pragma omp for schedule(dynamic, 256)
      for (int64_t p = 0; p < (int64_t)P; ++p) {
        if (mask && !mask[p]) continue;
        uint64_t k = start[p + 1] - start[p];
        memcpy(order, idx + start[p], sizeof(uint32_t) * k);
        qsort(order, k, sizeof(uint32_t), cmp_frag); /* depth-major order */
        double S[3] = {0.0, 0.0, 0.0}, T[3] = {1.0, 1.0, 1.0};
        for (int c = 0; c < C; ++c) {
          if (brute) {
            for (uint64_t r = 0; r < k; ++r) {
              double xr = clamp_depth(depth[order[r]]);
              double prod = 1.0;
              for (uint64_t q = 0; q < k; ++q)
                if (clamp_depth(depth[order[q]]) < xr) prod *= 1.0 - orc_alpha_used(alpha[(uint64_t)order[q] * C + c]);
              V[r] = prod;
            }
          } else {
            double run = 1.0;
            uint64_t r = 0;
            while (r < k) {
              uint64_t e = r;
              double xr = clamp_depth(depth[order[r]]);
              while (e < k && clamp_depth(depth[order[e]]) == xr) ++e;
              double grp = 1.0;
              for (uint64_t q = r; q < e; ++q) {
                V[q] = run;
                grp *= 1.0 - orc_alpha_used(alpha[(uint64_t)order[q] * C + c]);
              }
              run *= grp;
              r = e;
            }
          }
          double tot = 1.0;
          for (uint64_t r = 0; r < k; ++r) {
            uint32_t i = order[r];
            double au = orc_alpha_used(alpha[(uint64_t)i * C + c]);
            tot *= 1.0 - au;
            if (vis) vis[(uint64_t)i * C + c] = V[r];
            if (C == 3) {
              S[c] += au * rgb[(uint64_t)i * 3 + c] * V[r];
            } else {
              for (int q = 0; q < 3; ++q) S[q] += au * rgb[(uint64_t)i * 3 + q] * V[r];
            }
          }
          T[c] = tot;
        }
        for (int q = 0; q < 3; ++q) out[p * 3 + q] = S[q] + bg[q] * T[(C == 3) ? q : 0];
      }
    }
    free(order); free(V);
  }
  free(start);
  free(idx);
  return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* Gradient of the resolve with respect to alpha and colour                                         */
/* ------------------------------------------------------------------------------------------------ */

/*
 * orc_backward: the chain rule through the forward steps above, for a loss whose gradient with respect to
 * out is grad_out [P][3]. Depth is not differentiated. With g_q = grad_out_q and c(q) as in orc_resolve:
 *   d/dc_{i,q}      = g_q alpha_{i,c(q)} v_{i,c(q)}
 *   d/dalpha_{i,c}  = sum_{q: c(q)=c} g_q c_{i,q} v_{i,c}
 *                   + (1 / (1 - alpha_{i,c})) * dL/da_{i,c},
 *   dL/da_{i,c}     = - sum_{q: c(q)=c} g_q [ sum_k alpha_{k,c} c_{k,q} v_{k,c} K(x_i, x_k) + bg_q T_c ],
 * where K(x_i, z) = dA~(z)/da_i is found by running the build of section 2.3.1 for a lone unit step at x_i,
 * synthesising its cell averages and interpolating at z. The clamp of alpha has zero slope outside
 * (0, 1 - 2^-24); dropped fragments get zero gradients.
 */
int orc_backward(uint32_t width, uint32_t height, uint32_t rank, uint32_t channels, uint64_t count,
                 const uint32_t* pixel, const float* depth, const float* alpha, const float* rgb, const double* bg,
                 const double* grad_out, const uint8_t* mask, int tight, double* grad_alpha, double* grad_rgb,
                 int threads) {
  if (rank > 12 || (channels != 1 && channels != 3) || (count && (!pixel || !depth || !alpha || !rgb)) || !bg ||
      !grad_out || !grad_alpha || !grad_rgb)
    return ORC_EINVAL;
  orc_stream s = {width, height, rank, channels, count, pixel, depth, alpha, rgb};
  uint64_t P = (uint64_t)width * height;
  int M = 1 << (rank + 1);
  int C = (int)channels;
  uint64_t* start;
  uint32_t* idx;
  uint64_t nd;
  int rc = group_by_pixel(&s, mask, &start, &idx, &nd);
  if (rc) return rc;
  for (uint64_t i = 0; i < count; ++i) {
    if (frag_valid(&s, i) && !(mask && !mask[pixel[i]])) continue;
    for (int c = 0; c < C; ++c) grad_alpha[i * C + c] = 0.0;
    for (int q = 0; q < 3; ++q) grad_rgb[i * 3 + q] = 0.0;
  }
  uint64_t kmax = max_run(start, P);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int fail = 0;
#pragma omp parallel
  {
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (kmax ? kmax : 1));
    double* xs = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    double* as = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    double* v = (double*)malloc(sizeof(double) * (kmax ? kmax : 1));
    double* cf = (double*)malloc(sizeof(double) * M);
    double* ce = (double*)malloc(sizeof(double) * M);
    double* uc = (double*)malloc(sizeof(double) * M);
    double* ue = (double*)malloc(sizeof(double) * M);
    if (!order || !xs || !as || !v || !cf || !ce || !uc || !ue) {
#pragma omp atomic write
      fail = 1;
    } else {
      g_sort_stream = &s;
#pragma omp for schedule(dynamic, 256)
      for (int64_t p = 0; p < (int64_t)P; ++p) {
        if (mask && !mask[p]) continue;
        uint64_t k = start[p + 1] - start[p];
        memcpy(order, idx + start[p], sizeof(uint32_t) * k);
        qsort(order, k, sizeof(uint32_t), cmp_frag);
        const double* g = grad_out + p * 3;
        pixel_depths(depth, order, k, tight, xs);
        for (int c = 0; c < C; ++c) {
          double suma = 0.0;
          for (uint64_t r = 0; r < k; ++r) {
            as[r] = orc_absorbance(alpha[(uint64_t)order[r] * C + c]);
            suma += as[r];
          }
          orc_coeffs_one((int)rank, (int)k, xs, as, cf);
          orc_cells_one((int)rank, cf, ce);
          for (uint64_t r = 0; r < k; ++r) v[r] = exp(-orc_reconstruct((int)rank, ce, xs[r]));
          double T = exp(-suma);
          for (uint64_t r = 0; r < k; ++r) {
            uint32_t i = order[r];
            double araw = alpha[(uint64_t)i * C + c];
            double au = orc_alpha_used(araw);
            /* K(x_i, .): the forward steps applied to a lone unit step at x_i */
            double one = 1.0;
            orc_coeffs_one((int)rank, 1, &xs[r], &one, uc);
            orc_cells_one((int)rank, uc, ue);
            double dLda = 0.0, direct = 0.0;
            for (int q = 0; q < 3; ++q) {
              if (C == 3 && q != c) continue;
              double inner = bg[q] * T;
              for (uint64_t m = 0; m < k; ++m) {
                uint32_t j = order[m];
                double am = orc_alpha_used(alpha[(uint64_t)j * C + c]);
                inner += am * rgb[(uint64_t)j * 3 + q] * v[m] * orc_reconstruct((int)rank, ue, xs[m]);
              }
              dLda -= g[q] * inner;
              direct += g[q] * rgb[(uint64_t)i * 3 + q] * v[r];
              grad_rgb[(uint64_t)i * 3 + q] = g[q] * au * v[r];
            }
            int inside = (araw > 0.0) && (araw < ALPHA_MAX);
            grad_alpha[(uint64_t)i * C + c] = inside ? direct + dLda / (1.0 - au) : 0.0;
          }
        }
      }
    }
    free(order); free(xs); free(as); free(v); free(cf); free(ce); free(uc); free(ue);
  }
  free(start);
  free(idx);
  return fail ? ORC_ENOMEM : ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
