/*
 * fpsz_oracle.c -- plain, slow, single-threaded CPU oracle of fixed-PSNR
 * SZ-style compression.
 *
 * TEST INFRASTRUCTURE. This file exists only to check the GPU library
 * against. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it. It shares no code, header, table or constant
 * generator with the GPU library; the format constants below are written out
 * here independently from the format description.
 *
 * Paper: D. Tao, S. Di, X. Liang, Z. Chen, F. Cappello, "Fixed-PSNR Lossy
 * Compression for Scientific Data", arXiv:1805.07384.
 *
 * What the oracle computes, in the paper's order:
 *   1. the value range vr of the original data (Sec. IV, definition under
 *      Eq. 4; Eq. 6 and the remark after it: eb_abs / vr = eb_rel);
 *   2. the value-range-relative bound from the target PSNR,
 *      eb_rel = sqrt(3) * 10^(-PSNR/20) (Eq. 7), then eb_abs = eb_rel * vr;
 *   3. uniform quantization with bin size 2*eb_abs and midpoint
 *      reconstruction (Sec. IV: bins of equal length, midpoint m_i of each
 *      bin; Eq. 5 and Eq. 6 with delta = 2*eb_abs).  The field is
 *      prequantized, q = rint(x / (2 eb)), so the prediction of Sec. III runs
 *      on integers and the decompressor repeats it exactly (Eq. 1);
 *   4. Lorenzo prediction from the preceding neighbours (Sec. II-A step (1),
 *      Sec. III), giving integer residuals delta;
 *   5. Huffman coding of the residual symbols (Sec. II-A step (2));
 *   6. decompression: decode, undo the prediction (inclusive prefix sums),
 *      reconstruct bin midpoints (Sec. III, Eq. 1);
 *   7. MSE / PSNR of the reconstruction (Eq. 4, first two lines).
 *
 * Readings where the paper is silent (all are fixed format choices):
 *   - rounding of the bin index is round-half-to-even (rint);
 *   - the Lorenzo predictor pads with zero outside the field (GLOBAL domain)
 *     or outside each tile (TILE domain); both reconstruct identically
 *     (Theorem 1 / Theorem 3: the error is that of the quantizer alone);
 *   - residual symbols: |d| <= 511 coded directly, 512 <= |d| < 2^15 coded
 *     as one of 12 magnitude classes plus raw bits, |d| >= 2^15 is an
 *     outlier kept in a sparse exception list;
 *   - points whose float32 reconstruction lands just outside eb are kept
 *     exactly in the same exception list ("patches");
 *   - Huffman: two-queue construction with leaves ordered by (count, symbol)
 *     and leaf-first ties; code lengths limited to 18 bits by rebalancing
 *     the per-length code counts (see or_code_lengths); canonical codes in
 *     (length, symbol) order;
 *   - GZIP (step (3) of SZ) is omitted.
 *
 * Built with -O2 -ffp-contract=off, no fast-math, no SIMD intrinsics.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ---- format constants (written out independently of the GPU library) --- */
#define OR_MAGIC 0x5A535046u /* "FPSZ" little-endian */
#define OR_VERSION 1
#define OR_HDR_BYTES 256
#define OR_NSYM 1036      /* 1 outlier + 1023 direct + 12 escape classes */
#define OR_DIRECT_MAX 511 /* |d| <= 511 coded directly */
#define OR_ESC_LOG_MIN 9  /* escape classes k = 9..14 */
#define OR_ESC_LOG_MAX 14
#define OR_OUTLIER_MIN 32768 /* |d| >= 2^15 -> outlier */
#define OR_LMAX 18
#define OR_CHUNK 128
#define OR_FLAG_CONST 1u
#define OR_FLAG_TILE 2u
#define OR_FLAG_CLOSED 4u /* bound rescaled by the closed-loop step */
#define OR_FLAG_INLOOP 8u /* in-loop prediction from reconstructed values (TILE) */
#define OR_FLAG_XFORM 16u /* orthonormal block transform of the coefficients (TILE) */
#define OR_TAG_PATCH 0x80000000u

/* status codes */
enum {
  OR_OK = 0,
  OR_E_INVALID_ARG = 1,
  OR_E_NONFINITE = 2,
  OR_E_RANGE = 3,
  OR_E_CORRUPT = 4,
  OR_E_CAPACITY = 5,
  OR_E_NOMEM = 6
};

/* optional intermediates; every non-NULL array is filled */
typedef struct {
  int32_t *q;         /* [n] field order: prequantized bin index */
  int32_t *delta;     /* [n] field order: Lorenzo residual */
  int16_t *code16;    /* [n] stream order: delta, or -32768 for outliers */
  uint32_t *hist;     /* [1036] */
  uint8_t *code_len;  /* [1036] */
  uint32_t *code;     /* [1036] canonical codewords (right-aligned) */
  double scalars[8];  /* vr, eb_rel, eb, e2, r, e2_f, r_f, maxabs */
  double minmax[2];
  uint64_t counts[6]; /* n_tiles, n_chunks, n_words, n_exc, n_outliers, n_patches */
} or_trace;

/* ------------------------------------------------------------------------ */
/* small helpers                                                           */
/* ------------------------------------------------------------------------ */
/* Wall-clock seconds of the stages of the last call (for the CPU baseline of
 * the benchmark; no effect on any result).  Slots: 0 range, 1 prequantization,
 * 2 Lorenzo, 3 symbols + histogram + exception list, 4 Huffman code,
 * 5 encode, 6 blob assembly; 8 parse + tables, 9 decode, 10 prefix sums,
 * 11 reconstruction; 12 statistics. */
static double g_stage[16];
static double g_mark;
static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}
static void stage_begin(void) { g_mark = now_s(); }
static void stage_end(int k) {
  const double t = now_s();
  g_stage[k] += t - g_mark;
  g_mark = t;
}
void or_stage_times(double *out) { memcpy(out, g_stage, sizeof(g_stage)); }

static uint64_t rd_u64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static uint32_t rd_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint16_t rd_u16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
static double rd_f64(const uint8_t *p) { double v; memcpy(&v, p, 8); return v; }
static void wr_u64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static void wr_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void wr_u16(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }
static void wr_f64(uint8_t *p, double v) { memcpy(p, &v, 8); }
static uint64_t align8(uint64_t v) { return (v + 7) & ~(uint64_t)7; }

/* value of element i as double (exact for both dtypes) */
static double elem(const void *x, int dtype, uint64_t i) {
  return dtype == 0 ? (double)((const float *)x)[i] : ((const double *)x)[i];
}

/* Field shape normalized to (nz, ny, nx), and the fixed tile shape per
 * dimensionality: 1D 8192, 2D 64 x 128, 3D 16 x 16 x 32 (all 8192 points). */
typedef struct {
  uint64_t nz, ny, nx, n;
  uint64_t tz, ty, tx;    /* tile extents */
  uint64_t gz, gy, gx;    /* tile grid */
  uint64_t n_tiles, n_chunks;
} or_shape;

static int make_shape(int ndim, const uint64_t *dims, or_shape *s) {
  if (ndim < 1 || ndim > 3) return OR_E_INVALID_ARG;
  uint64_t d[3] = {1, 1, 1};
  for (int i = 0; i < ndim; i++) {
    if (dims[i] == 0) return OR_E_INVALID_ARG;
    d[3 - ndim + i] = dims[i];
  }
  s->nz = d[0]; s->ny = d[1]; s->nx = d[2];
  s->n = d[0] * d[1] * d[2];
  if (s->n >= ((uint64_t)1 << 31)) return OR_E_INVALID_ARG;
  if (ndim == 1) { s->tz = 1; s->ty = 1; s->tx = 8192; }
  else if (ndim == 2) { s->tz = 1; s->ty = 64; s->tx = 128; }
  else { s->tz = 16; s->ty = 16; s->tx = 32; }
  s->gz = (s->nz + s->tz - 1) / s->tz;
  s->gy = (s->ny + s->ty - 1) / s->ty;
  s->gx = (s->nx + s->tx - 1) / s->tx;
  s->n_tiles = s->gz * s->gy * s->gx;
  /* chunks are counted per tile: ceil(points_in_tile / 128) */
  s->n_chunks = 0;
  for (uint64_t a = 0; a < s->gz; a++)
    for (uint64_t b = 0; b < s->gy; b++)
      for (uint64_t c = 0; c < s->gx; c++) {
        uint64_t ez = (a + 1) * s->tz <= s->nz ? s->tz : s->nz - a * s->tz;
        uint64_t ey = (b + 1) * s->ty <= s->ny ? s->ty : s->ny - b * s->ty;
        uint64_t ex = (c + 1) * s->tx <= s->nx ? s->tx : s->nx - c * s->tx;
        s->n_chunks += (ez * ey * ex + OR_CHUNK - 1) / OR_CHUNK;
      }
  return OR_OK;
}

/* Walk the stream: tiles in row-major order over the tile grid, points in
 * row-major order inside the (edge-clipped) tile.  Fills perm[p] = field
 * index of stream position p. */
static void stream_order(const or_shape *s, uint64_t *perm) {
  uint64_t p = 0;
  for (uint64_t a = 0; a < s->gz; a++)
    for (uint64_t b = 0; b < s->gy; b++)
      for (uint64_t c = 0; c < s->gx; c++) {
        uint64_t z0 = a * s->tz, y0 = b * s->ty, x0 = c * s->tx;
        uint64_t z1 = z0 + s->tz < s->nz ? z0 + s->tz : s->nz;
        uint64_t y1 = y0 + s->ty < s->ny ? y0 + s->ty : s->ny;
        uint64_t x1 = x0 + s->tx < s->nx ? x0 + s->tx : s->nx;
        for (uint64_t z = z0; z < z1; z++)
          for (uint64_t y = y0; y < y1; y++)
            for (uint64_t x = x0; x < x1; x++) perm[p++] = (z * s->ny + y) * s->nx + x;
      }
}

/* ------------------------------------------------------------------------ */
/* In-loop prediction (SZ 1.4's scheme, Sec. II-A step (1) and Sec. III,     */
/* Eq. 1): the Lorenzo predictor of a point reads the RECONSTRUCTED values   */
/* of its preceding neighbours, as the decompressor will see them; outside   */
/* the point's tile it reads zero.  The seven terms are summed in the field's */
/* precision in this fixed order (zero for a neighbour outside the tile):     */
/*   (z,y,x-1) + (z,y-1,x) + (z-1,y,x) - (z,y-1,x-1) - (z-1,y,x-1)            */
/*   - (z-1,y-1,x) + (z-1,y-1,x-1)                                            */
/* ------------------------------------------------------------------------ */
static double il_nb(const void *xr, int dtype, const or_shape *S, uint64_t z, uint64_t y,
                    uint64_t x, uint64_t z0, uint64_t y0, uint64_t x0, int dz, int dy, int dx) {
  if ((dz && z == z0) || (dy && y == y0) || (dx && x == x0)) return 0.0;
  uint64_t i = ((z - dz) * S->ny + (y - dy)) * S->nx + (x - dx);
  return dtype == 0 ? (double)((const float *)xr)[i] : ((const double *)xr)[i];
}

static float il_pred_f(const float *xr, const or_shape *S, uint64_t z, uint64_t y, uint64_t x,
                       uint64_t z0, uint64_t y0, uint64_t x0) {
  float p = (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 0, 0, 1);
  p = p + (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 0, 1, 0);
  p = p + (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 1, 0, 0);
  p = p - (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 0, 1, 1);
  p = p - (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 1, 0, 1);
  p = p - (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 1, 1, 0);
  p = p + (float)il_nb(xr, 0, S, z, y, x, z0, y0, x0, 1, 1, 1);
  return p;
}

static double il_pred_d(const double *xr, const or_shape *S, uint64_t z, uint64_t y, uint64_t x,
                        uint64_t z0, uint64_t y0, uint64_t x0) {
  double p = il_nb(xr, 1, S, z, y, x, z0, y0, x0, 0, 0, 1);
  p = p + il_nb(xr, 1, S, z, y, x, z0, y0, x0, 0, 1, 0);
  p = p + il_nb(xr, 1, S, z, y, x, z0, y0, x0, 1, 0, 0);
  p = p - il_nb(xr, 1, S, z, y, x, z0, y0, x0, 0, 1, 1);
  p = p - il_nb(xr, 1, S, z, y, x, z0, y0, x0, 1, 0, 1);
  p = p - il_nb(xr, 1, S, z, y, x, z0, y0, x0, 1, 1, 0);
  p = p + il_nb(xr, 1, S, z, y, x, z0, y0, x0, 1, 1, 1);
  return p;
}

/* ------------------------------------------------------------------------ */
/* Orthogonal-transform variant (Sec. III Theorem 2, Sec. IV Theorem 3): the */
/* field is cut into blocks of 4 (1D), 4 x 4 (2D) or 4 x 4 x 4 (3D) points,   */
/* each block transformed by the orthonormal 4-point Walsh-Hadamard matrix    */
/*   H = 1/2 [[1,1,1,1], [1,1,-1,-1], [1,-1,-1,1], [1,-1,1,-1]]               */
/* along x, then y, then z, and the coefficients quantized with bin 2 eb.     */
/* H is symmetric and H H = I, so the inverse applies H along the same axes.  */
/* An orthonormal transform keeps the squared error, so the MSE of the data   */
/* is that of the coefficients (Theorem 2) and Eq. 7 sets the PSNR as for     */
/* the prediction-based scheme (Theorem 3); there is no pointwise bound.      */
/* The sums run in the field's precision in the order written below.          */
/* ------------------------------------------------------------------------ */
static void wht4_f(float *v, int st) {
  float a = v[0], b = v[st], c = v[2 * st], d = v[3 * st];
  float w0 = ((a + b) + c) + d, w1 = ((a + b) - c) - d;
  float w2 = ((a - b) - c) + d, w3 = ((a - b) + c) - d;
  v[0] = 0.5f * w0; v[st] = 0.5f * w1; v[2 * st] = 0.5f * w2; v[3 * st] = 0.5f * w3;
}
static void wht4_d(double *v, int st) {
  double a = v[0], b = v[st], c = v[2 * st], d = v[3 * st];
  double w0 = ((a + b) + c) + d, w1 = ((a + b) - c) - d;
  double w2 = ((a - b) - c) + d, w3 = ((a - b) + c) - d;
  v[0] = 0.5 * w0; v[st] = 0.5 * w1; v[2 * st] = 0.5 * w2; v[3 * st] = 0.5 * w3;
}
/* a block of 4^ndim values laid out [kz][ky][kx] (strides 16, 4, 1) */
static void wht_block_f(float *blk, int ndim) {
  for (int r = 0; r < (ndim == 3 ? 16 : ndim == 2 ? 4 : 1); r++) wht4_f(blk + 4 * r, 1);
  if (ndim >= 2)
    for (int kz = 0; kz < (ndim == 3 ? 4 : 1); kz++)
      for (int kx = 0; kx < 4; kx++) wht4_f(blk + 16 * kz + kx, 4);
  if (ndim == 3)
    for (int r = 0; r < 16; r++) wht4_f(blk + r, 16);
}
static void wht_block_d(double *blk, int ndim) {
  for (int r = 0; r < (ndim == 3 ? 16 : ndim == 2 ? 4 : 1); r++) wht4_d(blk + 4 * r, 1);
  if (ndim >= 2)
    for (int kz = 0; kz < (ndim == 3 ? 4 : 1); kz++)
      for (int kx = 0; kx < 4; kx++) wht4_d(blk + 16 * kz + kx, 4);
  if (ndim == 3)
    for (int r = 0; r < 16; r++) wht4_d(blk + r, 16);
}

/* Codes of the transform variant in stream order: tile by tile, blocks in
 * row-major order over the tile's block grid, a block's 4^ndim coefficient
 * codes row-major; a block's first (DC) code is its difference from the
 * previous block's DC bin in the tile (the first block's from zero). */
static void xform_codes(const void *x, int dtype, int ndim, const or_shape *S, double r,
                        float r_f, int32_t *code) {
  const int bs = ndim == 3 ? 64 : ndim == 2 ? 16 : 4;
  const int bz = ndim == 3 ? 4 : 1, by = ndim >= 2 ? 4 : 1;
  uint64_t p = 0;
  for (uint64_t t = 0; t < S->n_tiles; t++) {
    uint64_t a = t / (S->gy * S->gx), b = (t / S->gx) % S->gy, c = t % S->gx;
    uint64_t z0 = a * S->tz, y0 = b * S->ty, x0 = c * S->tx;
    uint64_t ez = z0 + S->tz <= S->nz ? S->tz : S->nz - z0;
    uint64_t ey = y0 + S->ty <= S->ny ? S->ty : S->ny - y0;
    uint64_t ex = x0 + S->tx <= S->nx ? S->tx : S->nx - x0;
    int32_t prev_dc = 0;
    for (uint64_t kz = 0; kz < ez; kz += bz)
      for (uint64_t ky = 0; ky < ey; ky += by)
        for (uint64_t kx = 0; kx < ex; kx += 4) {
          float bf[64];
          double bd[64];
          for (int u = 0; u < bs; u++) {
            int uz = u / 16, uy = (u / 4) % 4, ux = u % 4;
            if (ndim == 2) { uz = 0; uy = u / 4; }
            if (ndim == 1) { uz = 0; uy = 0; }
            uint64_t i = ((z0 + kz + uz) * S->ny + (y0 + ky + uy)) * S->nx + (x0 + kx + ux);
            if (dtype == 0) bf[u] = ((const float *)x)[i];
            else bd[u] = ((const double *)x)[i];
          }
          if (dtype == 0) wht_block_f(bf, ndim);
          else wht_block_d(bd, ndim);
          for (int u = 0; u < bs; u++) {
            int32_t q = dtype == 0 ? (int32_t)rintf(bf[u] * r_f) : (int32_t)rint(bd[u] * r);
            if (u == 0) {
              code[p + u] = (int32_t)((uint32_t)q - (uint32_t)prev_dc); /* modulo 2^32 */
              prev_dc = q;
            } else {
              code[p + u] = q;
            }
          }
          p += (uint64_t)bs;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Eq. 7: eb_rel = sqrt(3) * 10^(-PSNR/20)                                  */
/* ------------------------------------------------------------------------ */
double or_eb_rel(double psnr) { return sqrt(3.0) * pow(10.0, -psnr / 20.0); }

/* ------------------------------------------------------------------------ */
/* Symbol map of a Lorenzo residual (format reading; the paper only says   */
/* "customized Huffman coding", Sec. II-A).                                  */
/* ------------------------------------------------------------------------ */
/* returns symbol; *nextra / *extra receive the raw bits of escape classes */
int or_symbol(int32_t d, int *nextra, uint32_t *extra) {
  int64_t a = d < 0 ? -(int64_t)d : (int64_t)d;
  *nextra = 0;
  *extra = 0;
  if (a <= OR_DIRECT_MAX) return (int)(d + 512);
  if (a >= OR_OUTLIER_MIN) return 0;
  int k = 0;
  while (((int64_t)1 << (k + 1)) <= a) k++; /* k = floor(log2 a) */
  *nextra = k;
  *extra = (uint32_t)(a - ((int64_t)1 << k));
  return 1024 + 2 * (k - OR_ESC_LOG_MIN) + (d < 0 ? 1 : 0);
}

/* inverse: residual from symbol and raw bits (outlier symbol 0 not handled) */
int32_t or_unsymbol(int s, uint32_t extra) {
  if (s >= 1 && s <= 1023) return (int32_t)s - 512;
  int k = (s - 1024) / 2 + OR_ESC_LOG_MIN;
  int32_t mag = (int32_t)((1u << k) + extra);
  return ((s - 1024) & 1) ? -mag : mag;
}

static int sym_extra_bits(int s) {
  if (s >= 1024 && s < OR_NSYM) return (s - 1024) / 2 + OR_ESC_LOG_MIN;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Huffman code lengths: textbook two-queue construction.                   */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t w; int sym; } leaf_t;

static int leaf_cmp(const void *a, const void *b) {
  const leaf_t *x = (const leaf_t *)a, *y = (const leaf_t *)b;
  if (x->w != y->w) return x->w < y->w ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym ? 1 : 0);
}

/* Unlimited Huffman lengths for counts w[0..nsym) (zero counts get length 0).
 * Leaves sorted by (count, symbol); each step takes the two smallest fronts of
 * the leaf queue and the FIFO of merged nodes, preferring the leaf on equal
 * weight.  A single used symbol gets length 1.  Returns the maximum length. */
static int huffman_lengths(const uint64_t *w, int nsym, uint8_t *len) {
  leaf_t *L = (leaf_t *)malloc(sizeof(leaf_t) * (size_t)nsym);
  int n = 0;
  for (int s = 0; s < nsym; s++) {
    len[s] = 0;
    if (w[s] > 0) { L[n].w = w[s]; L[n].sym = s; n++; }
  }
  if (n == 0) { free(L); return 0; }
  if (n == 1) { len[L[0].sym] = 1; free(L); return 1; }
  qsort(L, (size_t)n, sizeof(leaf_t), leaf_cmp);
  uint64_t *Iw = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  int *parent = (int *)malloc(sizeof(int) * (size_t)(2 * n)); /* leaves 0..n-1, internals n.. */
  int li = 0, ii = 0, ni = 0;
  while (ni < n - 1) {
    int pick[2];
    uint64_t pw[2];
    for (int k = 0; k < 2; k++) {
      if (li < n && (ii >= ni || L[li].w <= Iw[ii])) {
        pw[k] = L[li].w; pick[k] = li; li++;
      } else {
        pw[k] = Iw[ii]; pick[k] = n + ii; ii++;
      }
    }
    Iw[ni] = pw[0] + pw[1];
    parent[pick[0]] = n + ni;
    parent[pick[1]] = n + ni;
    ni++;
  }
  /* depths: the root is the last internal node; parents come later */
  int *depth = (int *)malloc(sizeof(int) * (size_t)(2 * n));
  depth[n + ni - 1] = 0;
  for (int v = n + ni - 2; v >= 0; v--) depth[v] = depth[parent[v]] + 1;
  int maxl = 0;
  for (int j = 0; j < n; j++) {
    len[L[j].sym] = (uint8_t)depth[j];
    if (depth[j] > maxl) maxl = depth[j];
  }
  free(L); free(Iw); free(parent); free(depth);
  return maxl;
}

/* Length-limited variant used by the format.  Build the optimal lengths
 * once.  If some code is longer than 18 bits, rebalance the number of codes
 * per length: repeatedly take two codes at the deepest level d (siblings)
 * and move them up to one code at d - 1, and split one code at the deepest
 * level j < d - 1 that has any into two codes at j + 1.  The number of codes
 * and the Kraft sum stay the same.  Then hand the resulting lengths out again
 * in frequency order: leaves ordered by (count, symbol) get the lengths
 * sorted from longest to shortest, so the rarest symbol gets the longest
 * code. */
typedef struct { uint32_t c; int sym; } cnt_t;

static int cnt_cmp(const void *a, const void *b) {
  const cnt_t *x = (const cnt_t *)a, *y = (const cnt_t *)b;
  if (x->c != y->c) return x->c < y->c ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym ? 1 : 0);
}

void or_code_lengths_limited(const uint32_t *hist, int nsym, int lmax, uint8_t *len) {
  uint64_t *w = (uint64_t *)calloc((size_t)nsym + 1, sizeof(uint64_t));
  for (int s = 0; s < nsym; s++) w[s] = hist[s];
  int maxl = huffman_lengths(w, nsym, len);
  free(w);
  if (maxl <= lmax) return;
  uint32_t bits[64];
  memset(bits, 0, sizeof(bits));
  for (int s = 0; s < nsym; s++)
    if (len[s]) bits[len[s]]++;
  for (int d = maxl; d > lmax; d--) {
    while (bits[d] > 0) {
      int j = d - 2;
      while (bits[j] == 0) j--;
      bits[d] -= 2;
      bits[d - 1] += 1;
      bits[j + 1] += 2;
      bits[j] -= 1;
    }
  }
  /* leaves in (count, symbol) order take lengths longest first */
  cnt_t *L = (cnt_t *)malloc(sizeof(cnt_t) * (size_t)nsym);
  int n = 0;
  for (int s = 0; s < nsym; s++)
    if (hist[s] > 0) { L[n].c = hist[s]; L[n].sym = s; n++; }
  qsort(L, (size_t)n, sizeof(cnt_t), cnt_cmp);
  int l = lmax, j = 0;
  while (j < n) {
    while (bits[l] == 0) l--;
    len[L[j].sym] = (uint8_t)l;
    bits[l]--;
    j++;
  }
  free(L);
}

void or_code_lengths(const uint32_t *hist, int nsym, uint8_t *len) {
  or_code_lengths_limited(hist, nsym, OR_LMAX, len);
}

/* exposed for the Huffman pins: unlimited lengths */
int or_huffman_unlimited(const uint64_t *w, int nsym, uint8_t *len) {
  return huffman_lengths(w, nsym, len);
}

/* Canonical codes: symbols in (length, symbol) order get consecutive codes;
 * moving to a longer length shifts left by the length difference. */
void or_canonical_codes(const uint8_t *len, int nsym, uint32_t *code) {
  uint32_t next = 0;
  int prev_len = 0;
  int first = 1;
  for (int l = 1; l <= 32; l++) {
    for (int s = 0; s < nsym; s++) {
      if (len[s] != l) continue;
      if (first) { next = 0; prev_len = l; first = 0; }
      else { next = (next + 1) << (l - prev_len); prev_len = l; }
      code[s] = next;
    }
  }
  for (int s = 0; s < nsym; s++)
    if (len[s] == 0) code[s] = 0;
}

/* ------------------------------------------------------------------------ */
/* bit writer / reader, MSB-first in little-endian 32-bit words             */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t *w; uint64_t nbits; } bitw_t;

static void put_bits(bitw_t *bw, uint32_t v, int n) {
  for (int i = n - 1; i >= 0; i--) {
    uint32_t bit = (v >> i) & 1u;
    uint64_t pos = bw->nbits++;
    if (bit) bw->w[pos >> 5] |= 1u << (31 - (pos & 31));
  }
}

static uint32_t get_bit(const uint32_t *w, uint64_t pos) {
  return (w[pos >> 5] >> (31 - (pos & 31))) & 1u;
}

/* ------------------------------------------------------------------------ */
/* checksum of the blob (format definition): sum over little-endian 32-bit  */
/* words w_j of mix(w_j, j), mod 2^64; the checksum field reads as zero.    */
/* ------------------------------------------------------------------------ */
static uint64_t mix64(uint32_t w, uint64_t j) {
  uint64_t h = (uint64_t)w * 0x9E3779B97F4A7C15ull + j * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  return h;
}

uint64_t or_checksum(const uint8_t *blob, uint64_t bytes) {
  uint64_t s = 0;
  for (uint64_t j = 0; j < bytes / 4; j++) {
    uint32_t w = (j == 50 || j == 51) ? 0u : rd_u32(blob + 4 * j); /* bytes 200..207 */
    s += mix64(w, j);
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* header field offsets                                                     */
/* ------------------------------------------------------------------------ */
enum {
  H_MAGIC = 0, H_VERSION = 4, H_FLAGS = 6, H_DTYPE = 8, H_NDIM = 9, H_LOG2D = 10,
  H_LOG2R = 11, H_LMAX = 12, H_DIMS = 16, H_TILE = 40, H_CHUNK = 52,
  H_PSNR = 56, H_EBREL = 64, H_VR = 72, H_EB = 80, H_E2 = 88, H_R = 96,
  H_E2T = 104, H_RT = 112, H_MIN = 120, H_MAX = 128, H_N = 136,
  H_NTILES = 144, H_NCHUNKS = 152, H_NWORDS = 160, H_NEXC = 168,
  H_NOUT = 176, H_NPATCH = 184, H_BYTES = 192, H_CSUM = 200, H_CONST = 208,
  H_SCALE = 216 /* closed loop: the factor applied to eb_rel (raw float64) */
};

/* section layout after the header */
typedef struct {
  uint64_t off_len, off_two, off_teo, off_cb, off_exc, off_words, total;
} or_layout;

static void layout(uint64_t n_tiles, uint64_t n_chunks, uint64_t n_exc, uint64_t n_words,
                   or_layout *L) {
  uint64_t o = OR_HDR_BYTES;
  L->off_len = o; o = align8(o + OR_NSYM);
  L->off_two = o; o = align8(o + 8 * (n_tiles + 1));
  L->off_teo = o; o = align8(o + 8 * (n_tiles + 1));
  L->off_cb = o; o = align8(o + 2 * n_chunks);
  L->off_exc = o; o = align8(o + 8 * n_exc);
  L->off_words = o; o = align8(o + 4 * n_words);
  L->total = o;
}

/* ------------------------------------------------------------------------ */
/* compression                                                              */
/* ------------------------------------------------------------------------ */
/* dtype: 0 float32, 1 float64.  domain: 0 GLOBAL, 1 TILE.                  */
/* scale: factor applied to eb_rel; closed: the blob records the factor (flag
 * CLOSED and the float64 at H_SCALE).  Plain compression is scale 1, closed 0. */
static int compress_impl(const void *x, int dtype, int ndim, const uint64_t *dims, double psnr,
                         int domain, double scale, int closed, int variant,
                         uint8_t **blob_out, uint64_t *bytes_out, or_trace *tr) {
  const int inloop = variant == 1, xform = variant == 2;
  if (variant) domain = 1; /* in-loop prediction and block transforms run per tile */
  *blob_out = NULL;
  *bytes_out = 0;
  if (dtype != 0 && dtype != 1) return OR_E_INVALID_ARG;
  if (domain != 0 && domain != 1) return OR_E_INVALID_ARG;
  if (!isfinite(psnr)) return OR_E_INVALID_ARG;
  or_shape S;
  int st = make_shape(ndim, dims, &S);
  if (st != OR_OK) return st;
  const uint64_t n = S.n;
  memset(g_stage, 0, sizeof(g_stage));
  stage_begin();

  /* 1. value range of the original data (vr, definition under Eq. 4) */
  double mn = 0, mx = 0;
  for (uint64_t i = 0; i < n; i++) {
    double v = elem(x, dtype, i);
    if (!isfinite(v)) return OR_E_NONFINITE;
    if (i == 0 || v < mn) mn = v;
    if (i == 0 || v > mx) mx = v;
  }
  mn = mn + 0.0; /* -0 reads as +0 */
  mx = mx + 0.0;
  double vr = mx - mn;
  stage_end(0);

  /* 2. Eq. 7 and eb_abs = eb_rel * vr (remark after Eq. 6); bin size 2 eb */
  double eb_rel = or_eb_rel(psnr);
  if (closed) eb_rel = eb_rel * scale;
  double eb = vr * eb_rel;
  double e2 = 2.0 * eb;
  double r = 1.0 / e2;
  float e2_f = (float)e2, r_f = (float)r;
  double maxabs = fabs(mn) > fabs(mx) ? fabs(mn) : fabs(mx);
  if (tr) {
    tr->scalars[0] = vr; tr->scalars[1] = eb_rel; tr->scalars[2] = eb; tr->scalars[3] = e2;
    tr->scalars[4] = r; tr->scalars[5] = (double)e2_f; tr->scalars[6] = (double)r_f;
    tr->scalars[7] = maxabs; tr->minmax[0] = mn; tr->minmax[1] = mx;
  }

  int is_const = (vr == 0.0);
  if (!is_const) {
    double lim = dtype == 0 ? 8388608.0 : 134217728.0; /* 2^23, 2^27 */
    if (!(maxabs * r < lim)) return OR_E_RANGE;
  }

  uint8_t *blob;
  if (is_const) {
    blob = (uint8_t *)calloc(1, OR_HDR_BYTES);
    wr_u32(blob + H_MAGIC, OR_MAGIC);
    wr_u16(blob + H_VERSION, OR_VERSION);
    wr_u16(blob + H_FLAGS, (uint16_t)(OR_FLAG_CONST | (domain ? OR_FLAG_TILE : 0) |
                                      (closed ? OR_FLAG_CLOSED : 0) |
                                      (inloop ? OR_FLAG_INLOOP : 0) | (xform ? OR_FLAG_XFORM : 0)));
    if (closed) wr_f64(blob + H_SCALE, scale);
    blob[H_DTYPE] = (uint8_t)dtype; blob[H_NDIM] = (uint8_t)ndim;
    blob[H_LOG2D] = 9; blob[H_LOG2R] = 15; blob[H_LMAX] = OR_LMAX;
    for (int i = 0; i < 3; i++) wr_u64(blob + H_DIMS + 8 * i, i < ndim ? dims[i] : 1);
    wr_u32(blob + H_TILE, (uint32_t)S.tz); wr_u32(blob + H_TILE + 4, (uint32_t)S.ty);
    wr_u32(blob + H_TILE + 8, (uint32_t)S.tx); wr_u32(blob + H_CHUNK, OR_CHUNK);
    wr_f64(blob + H_PSNR, psnr); wr_f64(blob + H_EBREL, eb_rel); wr_f64(blob + H_VR, vr);
    wr_f64(blob + H_EB, eb); wr_f64(blob + H_E2, e2); wr_f64(blob + H_R, r);
    wr_f64(blob + H_MIN, mn); wr_f64(blob + H_MAX, mx); wr_u64(blob + H_N, n);
    if (dtype == 0) { float c = (float)mn; uint32_t b; memcpy(&b, &c, 4); wr_u64(blob + H_CONST, b); }
    else { uint64_t b; memcpy(&b, &mn, 8); wr_u64(blob + H_CONST, b); }
    wr_u64(blob + H_BYTES, OR_HDR_BYTES);
    wr_u64(blob + H_CSUM, or_checksum(blob, OR_HDR_BYTES));
    *blob_out = blob;
    *bytes_out = OR_HDR_BYTES;
    if (tr) { memset(tr->counts, 0, sizeof(tr->counts)); }
    return OR_OK;
  }

  /* 3. prequantization: bin index q = rint(x / (2 eb)) (uniform bins,
   *    midpoint reconstruction q * 2 eb).  In-loop mode quantizes the
   *    prediction errors in the stream walk instead (step 5). */
  int32_t *q = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t *dl = (int32_t *)malloc(sizeof(int32_t) * n);
  float *xrf = inloop && dtype == 0 ? (float *)malloc(4 * n) : NULL;
  double *xrd = inloop && dtype == 1 ? (double *)malloc(8 * n) : NULL;
  for (uint64_t i = 0; i < n && !inloop && !xform; i++) {
    if (dtype == 0) {
      float t = ((const float *)x)[i] * r_f;
      q[i] = (int32_t)rintf(t);
    } else {
      double t = ((const double *)x)[i] * r;
      q[i] = (int32_t)rint(t);
    }
  }
  stage_end(1);

  /* 4. Lorenzo residual: delta = sum over the 8 corners of the unit cube
   *    behind the point of (-1)^(a+b+c) q[z-c][y-b][x-a]; q reads as zero
   *    outside the field (GLOBAL) or outside the point's tile (TILE). */
  if (xform) {
    xform_codes(x, dtype, ndim, &S, r, r_f, dl); /* stream order */
    memcpy(q, dl, 4 * n);
  }
  for (uint64_t z = 0; z < S.nz && !inloop && !xform; z++)
    for (uint64_t y = 0; y < S.ny; y++)
      for (uint64_t xx = 0; xx < S.nx; xx++) {
        uint64_t z0 = 0, y0 = 0, x0 = 0;
        if (domain == 1) { z0 = z / S.tz * S.tz; y0 = y / S.ty * S.ty; x0 = xx / S.tx * S.tx; }
        int64_t acc = 0;
        for (int a = 0; a <= 1; a++)
          for (int b = 0; b <= 1; b++)
            for (int c = 0; c <= 1; c++) {
              if ((c && z == z0) || (b && y == y0) || (a && xx == x0)) continue;
              int64_t v = q[((z - c) * S.ny + (y - b)) * S.nx + (xx - a)];
              acc += ((a + b + c) & 1) ? -v : v;
            }
        dl[(z * S.ny + y) * S.nx + xx] = (int32_t)acc;
      }
  stage_end(2);

  /* 5. walk the stream: symbols, histogram, exception records */
  uint64_t *perm = (uint64_t *)malloc(sizeof(uint64_t) * n);
  if (xform)
    for (uint64_t i = 0; i < n; i++) perm[i] = i; /* codes are already in stream order */
  else
    stream_order(&S, perm);
  int32_t *sym = (int32_t *)malloc(sizeof(int32_t) * n);
  uint32_t *xtra = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t hist[OR_NSYM];
  memset(hist, 0, sizeof(hist));
  uint64_t cap_exc = 1024, n_exc = 0, n_out = 0, n_pat = 0;
  uint32_t *exc = (uint32_t *)malloc(8 * cap_exc);
  uint64_t *tile_exc = (uint64_t *)calloc(S.n_tiles + 1, 8);
  {
    uint64_t p = 0;
    for (uint64_t t = 0; t < S.n_tiles; t++) {
      uint64_t a = t / (S.gy * S.gx), b = (t / S.gx) % S.gy, c = t % S.gx;
      uint64_t ez = (a + 1) * S.tz <= S.nz ? S.tz : S.nz - a * S.tz;
      uint64_t ey = (b + 1) * S.ty <= S.ny ? S.ty : S.ny - b * S.ty;
      uint64_t ex = (c + 1) * S.tx <= S.nx ? S.tx : S.nx - c * S.tx;
      uint64_t nt = ez * ey * ex;
      tile_exc[t] = n_exc;
      for (uint64_t k = 0; k < nt; k++, p++) {
        uint64_t i = perm[p];
        int ne;
        uint32_t ev;
        if (inloop) {
          /* prediction from reconstructed neighbours, quantized error; a
           * point whose code leaves the radius or whose reconstruction
           * misses the bound in floating point is stored exactly */
          uint64_t xz = i / (S.ny * S.nx), xy = (i / S.nx) % S.ny, xx = i % S.nx;
          uint64_t z0 = a * S.tz, y0 = b * S.ty, x0 = c * S.tx;
          int keep;
          int32_t qi;
          if (dtype == 0) {
            float xv = ((const float *)x)[i];
            float pr = il_pred_f(xrf, &S, xz, xy, xx, z0, y0, x0);
            float dd = xv - pr;
            qi = (int32_t)rintf(dd * r_f);
            float rec = pr + (float)qi * e2_f;
            keep = qi > -OR_OUTLIER_MIN && qi < OR_OUTLIER_MIN &&
                   !(fabs((double)xv - (double)rec) > eb);
            xrf[i] = keep ? rec : xv;
          } else {
            double xv = ((const double *)x)[i];
            double pr = il_pred_d(xrd, &S, xz, xy, xx, z0, y0, x0);
            double dd = xv - pr;
            qi = (int32_t)rint(dd * r);
            double rec = pr + (double)qi * e2;
            keep = qi > -OR_OUTLIER_MIN && qi < OR_OUTLIER_MIN && !(fabs(xv - rec) > eb);
            xrd[i] = keep ? rec : xv;
          }
          q[i] = qi;
          dl[i] = keep ? qi : -OR_OUTLIER_MIN; /* the outlier symbol marks an exact point */
        }
        int s = or_symbol(dl[i], &ne, &ev);
        sym[p] = s;
        xtra[p] = ev;
        hist[s]++;
        if (tr && tr->code16) tr->code16[p] = (int16_t)(s == 0 ? -32768 : dl[i]);
        int npush = 0;
        uint32_t rec[6];
        if (s == 0 && !inloop) { rec[0] = (uint32_t)p; rec[1] = (uint32_t)dl[i]; npush = 1; n_out++; }
        /* (transform codes: no exact points; q below is unused) */
        /* patch test: the float reconstruction must lie within eb of x (in
         * in-loop mode: the points marked by the outlier symbol) */
        int patch;
        if (dtype == 0) {
          float xr = (float)q[i] * e2_f;
          patch = xform ? 0 : inloop ? s == 0 : fabs((double)((const float *)x)[i] - (double)xr) > eb;
          if (patch) {
            uint32_t bits;
            memcpy(&bits, &((const float *)x)[i], 4);
            rec[2 * npush] = (uint32_t)p | OR_TAG_PATCH; rec[2 * npush + 1] = bits; npush++;
          }
        } else {
          double xr = (double)q[i] * e2;
          patch = xform ? 0 : inloop ? s == 0 : fabs(((const double *)x)[i] - xr) > eb;
          if (patch) {
            uint64_t bits;
            memcpy(&bits, &((const double *)x)[i], 8);
            rec[2 * npush] = (uint32_t)p | OR_TAG_PATCH; rec[2 * npush + 1] = (uint32_t)bits; npush++;
            rec[2 * npush] = (uint32_t)p | OR_TAG_PATCH; rec[2 * npush + 1] = (uint32_t)(bits >> 32); npush++;
          }
        }
        if (patch) n_pat++;
        for (int j = 0; j < npush; j++) {
          if (n_exc == cap_exc) { cap_exc *= 2; exc = (uint32_t *)realloc(exc, 8 * cap_exc); }
          exc[2 * n_exc] = rec[2 * j];
          exc[2 * n_exc + 1] = rec[2 * j + 1];
          n_exc++;
        }
      }
    }
    tile_exc[S.n_tiles] = n_exc;
  }
  stage_end(3);

  /* 6. Huffman code (length-limited, canonical) */
  uint8_t len[OR_NSYM];
  uint32_t code[OR_NSYM];
  or_code_lengths(hist, OR_NSYM, len);
  or_canonical_codes(len, OR_NSYM, code);
  stage_end(4);

  /* 7. encode: per tile, chunks of 128 symbols, bit-contiguous; each tile
   *    padded to a 32-bit word */
  uint16_t *chunk_bits = (uint16_t *)malloc(2 * (S.n_chunks + 1));
  uint64_t *tile_words = (uint64_t *)calloc(S.n_tiles + 1, 8);
  uint64_t total_bits_bound = 0;
  for (uint64_t p = 0; p < n; p++) total_bits_bound += len[sym[p]] + sym_extra_bits(sym[p]);
  uint64_t words_cap = total_bits_bound / 32 + S.n_tiles + 2;
  uint32_t *words = (uint32_t *)calloc(words_cap, 4);
  {
    uint64_t p = 0, ci = 0, wbase = 0;
    for (uint64_t t = 0; t < S.n_tiles; t++) {
      uint64_t a = t / (S.gy * S.gx), b = (t / S.gx) % S.gy, c = t % S.gx;
      uint64_t ez = (a + 1) * S.tz <= S.nz ? S.tz : S.nz - a * S.tz;
      uint64_t ey = (b + 1) * S.ty <= S.ny ? S.ty : S.ny - b * S.ty;
      uint64_t ex = (c + 1) * S.tx <= S.nx ? S.tx : S.nx - c * S.tx;
      uint64_t nt = ez * ey * ex;
      tile_words[t] = wbase;
      bitw_t bw = {words + wbase, 0};
      for (uint64_t k = 0; k < nt; k += OR_CHUNK) {
        uint64_t before = bw.nbits;
        uint64_t kend = k + OR_CHUNK < nt ? k + OR_CHUNK : nt;
        for (uint64_t j = k; j < kend; j++) {
          int s = sym[p + j];
          put_bits(&bw, code[s], len[s]);
          int ne = sym_extra_bits(s);
          if (ne) put_bits(&bw, xtra[p + j], ne);
        }
        chunk_bits[ci++] = (uint16_t)(bw.nbits - before);
      }
      wbase += (bw.nbits + 31) / 32;
      p += nt;
    }
    tile_words[S.n_tiles] = wbase;
  }
  uint64_t n_words = tile_words[S.n_tiles];
  stage_end(5);

  /* 8. assemble the blob */
  or_layout Lo;
  layout(S.n_tiles, S.n_chunks, n_exc, n_words, &Lo);
  blob = (uint8_t *)calloc(1, Lo.total);
  wr_u32(blob + H_MAGIC, OR_MAGIC);
  wr_u16(blob + H_VERSION, OR_VERSION);
  wr_u16(blob + H_FLAGS, (uint16_t)((domain ? OR_FLAG_TILE : 0) | (closed ? OR_FLAG_CLOSED : 0) |
                                     (inloop ? OR_FLAG_INLOOP : 0) | (xform ? OR_FLAG_XFORM : 0)));
  if (closed) wr_f64(blob + H_SCALE, scale);
  blob[H_DTYPE] = (uint8_t)dtype; blob[H_NDIM] = (uint8_t)ndim;
  blob[H_LOG2D] = 9; blob[H_LOG2R] = 15; blob[H_LMAX] = OR_LMAX;
  for (int i = 0; i < 3; i++) wr_u64(blob + H_DIMS + 8 * i, i < ndim ? dims[i] : 1);
  wr_u32(blob + H_TILE, (uint32_t)S.tz); wr_u32(blob + H_TILE + 4, (uint32_t)S.ty);
  wr_u32(blob + H_TILE + 8, (uint32_t)S.tx); wr_u32(blob + H_CHUNK, OR_CHUNK);
  wr_f64(blob + H_PSNR, psnr); wr_f64(blob + H_EBREL, eb_rel); wr_f64(blob + H_VR, vr);
  wr_f64(blob + H_EB, eb); wr_f64(blob + H_E2, e2); wr_f64(blob + H_R, r);
  if (dtype == 0) {
    uint32_t b1, b2;
    memcpy(&b1, &e2_f, 4); memcpy(&b2, &r_f, 4);
    wr_u64(blob + H_E2T, b1); wr_u64(blob + H_RT, b2);
  } else {
    uint64_t b1, b2;
    memcpy(&b1, &e2, 8); memcpy(&b2, &r, 8);
    wr_u64(blob + H_E2T, b1); wr_u64(blob + H_RT, b2);
  }
  wr_f64(blob + H_MIN, mn); wr_f64(blob + H_MAX, mx); wr_u64(blob + H_N, n);
  wr_u64(blob + H_NTILES, S.n_tiles); wr_u64(blob + H_NCHUNKS, S.n_chunks);
  wr_u64(blob + H_NWORDS, n_words); wr_u64(blob + H_NEXC, n_exc);
  wr_u64(blob + H_NOUT, n_out); wr_u64(blob + H_NPATCH, n_pat);
  wr_u64(blob + H_BYTES, Lo.total);
  memcpy(blob + Lo.off_len, len, OR_NSYM);
  for (uint64_t t = 0; t <= S.n_tiles; t++) wr_u64(blob + Lo.off_two + 8 * t, tile_words[t]);
  for (uint64_t t = 0; t <= S.n_tiles; t++) wr_u64(blob + Lo.off_teo + 8 * t, tile_exc[t]);
  for (uint64_t c = 0; c < S.n_chunks; c++) wr_u16(blob + Lo.off_cb + 2 * c, chunk_bits[c]);
  for (uint64_t e = 0; e < n_exc; e++) {
    wr_u32(blob + Lo.off_exc + 8 * e, exc[2 * e]);
    wr_u32(blob + Lo.off_exc + 8 * e + 4, exc[2 * e + 1]);
  }
  for (uint64_t w = 0; w < n_words; w++) wr_u32(blob + Lo.off_words + 4 * w, words[w]);
  wr_u64(blob + H_CSUM, or_checksum(blob, Lo.total));

  if (tr) {
    if (tr->q) memcpy(tr->q, q, 4 * n);
    if (tr->delta) memcpy(tr->delta, dl, 4 * n);
    if (tr->hist) memcpy(tr->hist, hist, sizeof(hist));
    if (tr->code_len) memcpy(tr->code_len, len, OR_NSYM);
    if (tr->code) memcpy(tr->code, code, sizeof(code));
    tr->counts[0] = S.n_tiles; tr->counts[1] = S.n_chunks; tr->counts[2] = n_words;
    tr->counts[3] = n_exc; tr->counts[4] = n_out; tr->counts[5] = n_pat;
  }
  free(q); free(dl); free(perm); free(sym); free(xtra); free(exc); free(tile_exc);
  free(xrf); free(xrd);
  free(chunk_bits); free(tile_words); free(words);
  stage_end(6);
  *blob_out = blob;
  *bytes_out = Lo.total;
  return OR_OK;
}

int or_compress(const void *x, int dtype, int ndim, const uint64_t *dims, double psnr,
                int domain, uint8_t **blob_out, uint64_t *bytes_out, or_trace *tr) {
  return compress_impl(x, dtype, ndim, dims, psnr, domain, 1.0, 0, 0, blob_out, bytes_out, tr);
}

/* SZ 1.4-style in-loop compression (tile domain): see il_pred_f. */
int or_compress_inloop(const void *x, int dtype, int ndim, const uint64_t *dims, double psnr,
                       uint8_t **blob_out, uint64_t *bytes_out, or_trace *tr) {
  return compress_impl(x, dtype, ndim, dims, psnr, 1, 1.0, 0, 1, blob_out, bytes_out, tr);
}

/* Orthogonal-transform compression (see wht4_f); every dimension of the
 * field must be a multiple of 4. */
int or_compress_xform(const void *x, int dtype, int ndim, const uint64_t *dims, double psnr,
                      uint8_t **blob_out, uint64_t *bytes_out, or_trace *tr) {
  *blob_out = NULL;
  *bytes_out = 0;
  if (ndim < 1 || ndim > 3 || !dims) return OR_E_INVALID_ARG;
  for (int i = 0; i < ndim; i++)
    if (dims[i] % 4) return OR_E_INVALID_ARG;
  return compress_impl(x, dtype, ndim, dims, psnr, 1, 1.0, 0, 2, blob_out, bytes_out, tr);
}

/* Compression with the bound of Eq. 7 multiplied by a given factor, the
 * factor recorded in the blob (the second pass of the closed loop). */
int or_compress_scaled(const void *x, int dtype, int ndim, const uint64_t *dims, double psnr,
                       int domain, double scale, uint8_t **blob_out, uint64_t *bytes_out,
                       or_trace *tr) {
  if (!(scale > 0.0) || !isfinite(scale)) return OR_E_INVALID_ARG;
  return compress_impl(x, dtype, ndim, dims, psnr, domain, scale, 1, 0, blob_out, bytes_out, tr);
}

/* ------------------------------------------------------------------------ */
/* Closed-loop correction for low PSNR targets.                             */
/* Eq. 5 replaces the bin probabilities by a density, which holds only with  */
/* many bins across the value range; at low PSNR the achieved MSE departs    */
/* from eb^2 / 3 (Eq. 6).  The measured MSE of the first pass then gives one */
/* secant step on MSE proportional to eb^2: eb' = eb sqrt(MSE_t / MSE_1),    */
/* with MSE_t the MSE that Eq. 4 turns into the target,                      */
/* MSE_t = vr^2 10^(-PSNR/10).  The first pass needs no decompression: the   */
/* reconstruction is the quantizer's output (Theorem 1), x' = q 2eb, or x at */
/* a patch.                                                                  */
/* ------------------------------------------------------------------------ */
int or_quant_sse(const void *x, int dtype, uint64_t n, double psnr, double *sse_out,
                 double *vr_out) {
  if (n == 0 || (dtype != 0 && dtype != 1)) return OR_E_INVALID_ARG;
  double mn = 0, mx = 0;
  for (uint64_t i = 0; i < n; i++) {
    double v = elem(x, dtype, i);
    if (!isfinite(v)) return OR_E_NONFINITE;
    if (i == 0 || v < mn) mn = v;
    if (i == 0 || v > mx) mx = v;
  }
  double vr = (mx + 0.0) - (mn + 0.0);
  *vr_out = vr;
  *sse_out = 0.0;
  if (vr == 0.0) return OR_OK;
  double eb = vr * or_eb_rel(psnr);
  double e2 = 2.0 * eb, r = 1.0 / e2;
  float e2_f = (float)e2, r_f = (float)r;
  double maxabs = fabs(mn + 0.0) > fabs(mx + 0.0) ? fabs(mn + 0.0) : fabs(mx + 0.0);
  if (!(maxabs * r < (dtype == 0 ? 8388608.0 : 134217728.0))) return OR_E_RANGE;
  double s = 0.0, comp = 0.0;
  for (uint64_t i = 0; i < n; i++) {
    double e;
    if (dtype == 0) {
      float xv = ((const float *)x)[i];
      float xr = (float)(int32_t)rintf(xv * r_f) * e2_f;
      e = (double)xv - (double)xr;
    } else {
      double xv = ((const double *)x)[i];
      double xr = (double)(int32_t)rint(xv * r) * e2;
      e = xv - xr;
    }
    if (fabs(e) > eb) e = 0.0; /* a patch: stored exactly */
    double e2v = e * e, t = s + e2v;
    if (fabs(s) >= fabs(e2v)) comp += (s - t) + e2v;
    else comp += (e2v - t) + s;
    s = t;
  }
  *sse_out = s + comp;
  return OR_OK;
}

/* the secant factor from the first pass (1 when the first pass is exact) */
double or_closed_loop_scale(double sse, uint64_t n, double vr, double psnr) {
  if (!(sse > 0.0)) return 1.0;
  double mse_t = vr * vr * pow(10.0, -psnr / 10.0);
  return sqrt(mse_t / (sse / (double)n));
}

int or_compress_closed_loop(const void *x, int dtype, int ndim, const uint64_t *dims,
                            double psnr, int domain, uint8_t **blob_out, uint64_t *bytes_out,
                            or_trace *tr, double *scale_out) {
  *blob_out = NULL;
  *bytes_out = 0;
  if (!isfinite(psnr)) return OR_E_INVALID_ARG;
  or_shape S;
  int st = make_shape(ndim, dims, &S);
  if (st != OR_OK) return st;
  double sse, vr;
  st = or_quant_sse(x, dtype, S.n, psnr, &sse, &vr);
  if (st != OR_OK) return st;
  double scale = or_closed_loop_scale(sse, S.n, vr, psnr);
  if (scale_out) *scale_out = scale;
  return compress_impl(x, dtype, ndim, dims, psnr, domain, scale, 1, 0, blob_out, bytes_out, tr);
}

/* ------------------------------------------------------------------------ */
/* blob header query                                                        */
/* ------------------------------------------------------------------------ */
int or_blob_info(const uint8_t *blob, uint64_t bytes, int *dtype, int *ndim, uint64_t *dims,
                 double *scal /* psnr, eb_rel, vr, eb */, uint64_t *cnt /* n_exc, n_out, n_patch, n_words */) {
  if (bytes < OR_HDR_BYTES || rd_u32(blob + H_MAGIC) != OR_MAGIC) return OR_E_CORRUPT;
  *dtype = blob[H_DTYPE];
  *ndim = blob[H_NDIM];
  for (int i = 0; i < 3; i++) dims[i] = rd_u64(blob + H_DIMS + 8 * i);
  scal[0] = rd_f64(blob + H_PSNR); scal[1] = rd_f64(blob + H_EBREL);
  scal[2] = rd_f64(blob + H_VR); scal[3] = rd_f64(blob + H_EB);
  cnt[0] = rd_u64(blob + H_NEXC); cnt[1] = rd_u64(blob + H_NOUT);
  cnt[2] = rd_u64(blob + H_NPATCH); cnt[3] = rd_u64(blob + H_NWORDS);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* decompression                                                            */
/* ------------------------------------------------------------------------ */
int or_decompress(const uint8_t *blob, uint64_t bytes, void *out, uint64_t out_bytes) {
  memset(g_stage + 8, 0, 4 * sizeof(double));
  stage_begin();
  if (bytes < OR_HDR_BYTES) return OR_E_CORRUPT;
  if (rd_u32(blob + H_MAGIC) != OR_MAGIC || rd_u16(blob + H_VERSION) != OR_VERSION)
    return OR_E_CORRUPT;
  if (rd_u64(blob + H_BYTES) != bytes) return OR_E_CORRUPT;
  if (rd_u64(blob + H_CSUM) != or_checksum(blob, bytes)) return OR_E_CORRUPT;
  int dtype = blob[H_DTYPE], ndim = blob[H_NDIM];
  uint16_t flags = rd_u16(blob + H_FLAGS);
  if (dtype > 1 || ndim < 1 || ndim > 3) return OR_E_CORRUPT;
  uint64_t dims[3];
  for (int i = 0; i < ndim; i++) dims[i] = rd_u64(blob + H_DIMS + 8 * i);
  or_shape S;
  if (make_shape(ndim, dims, &S) != OR_OK) return OR_E_CORRUPT;
  uint64_t n = S.n;
  uint64_t es = dtype == 0 ? 4 : 8;
  if (out_bytes < n * es) return OR_E_CAPACITY;
  if (flags & OR_FLAG_CONST) {
    uint64_t cb = rd_u64(blob + H_CONST);
    for (uint64_t i = 0; i < n; i++) {
      if (dtype == 0) { uint32_t b = (uint32_t)cb; memcpy((float *)out + i, &b, 4); }
      else memcpy((double *)out + i, &cb, 8);
    }
    return OR_OK;
  }
  int domain = (flags & OR_FLAG_TILE) ? 1 : 0;
  int inloop = (flags & OR_FLAG_INLOOP) ? 1 : 0;
  int xform = (flags & OR_FLAG_XFORM) ? 1 : 0;
  if ((inloop || xform) && !domain) return OR_E_CORRUPT;
  if (inloop && xform) return OR_E_CORRUPT;
  if (xform)
    for (int i = 0; i < ndim; i++)
      if (dims[i] % 4) return OR_E_CORRUPT;
  uint64_t n_tiles = rd_u64(blob + H_NTILES), n_chunks = rd_u64(blob + H_NCHUNKS);
  uint64_t n_words = rd_u64(blob + H_NWORDS), n_exc = rd_u64(blob + H_NEXC);
  if (n_tiles != S.n_tiles || n_chunks != S.n_chunks) return OR_E_CORRUPT;
  or_layout Lo;
  layout(n_tiles, n_chunks, n_exc, n_words, &Lo);
  if (Lo.total != bytes) return OR_E_CORRUPT;
  uint64_t e2b = rd_u64(blob + H_E2T);
  float e2_f;
  double e2;
  { uint32_t b = (uint32_t)e2b; memcpy(&e2_f, &b, 4); memcpy(&e2, &e2b, 8); }

  /* rebuild the canonical decoding tables from the code lengths */
  uint8_t len[OR_NSYM];
  memcpy(len, blob + Lo.off_len, OR_NSYM);
  for (int s = 0; s < OR_NSYM; s++)
    if (len[s] > OR_LMAX) return OR_E_CORRUPT;
  uint32_t code[OR_NSYM];
  or_canonical_codes(len, OR_NSYM, code);
  /* per length: number of codes, first (smallest) code, and the symbols of
   * that length in symbol order */
  uint32_t cnt_l[OR_LMAX + 1], first_l[OR_LMAX + 1], base_l[OR_LMAX + 1];
  int sorted_sym[OR_NSYM];
  {
    int k = 0;
    for (int l = 0; l <= OR_LMAX; l++) {
      cnt_l[l] = 0;
      first_l[l] = 0;
      base_l[l] = (uint32_t)k;
      for (int u = 0; u < OR_NSYM; u++)
        if (len[u] == l && l > 0) {
          if (cnt_l[l] == 0) first_l[l] = code[u];
          cnt_l[l]++;
          sorted_sym[k++] = u;
        }
    }
  }

  const uint32_t *words = (const uint32_t *)(blob + Lo.off_words); /* 8-aligned in blob */
  uint32_t *wcopy = (uint32_t *)malloc(4 * (n_words + 1));
  for (uint64_t w = 0; w < n_words; w++) wcopy[w] = rd_u32(blob + Lo.off_words + 4 * w);
  (void)words;

  uint64_t *perm = (uint64_t *)malloc(sizeof(uint64_t) * n);
  if (xform)
    for (uint64_t i = 0; i < n; i++) perm[i] = i; /* coefficient codes stay in stream order */
  else
    stream_order(&S, perm);
  int32_t *dl = (int32_t *)malloc(sizeof(int32_t) * n); /* field order (stream order: xform) */
  uint8_t *is_out = (uint8_t *)calloc(n, 1);
  stage_end(8);
  int rc = OR_OK;
  uint64_t p = 0, ci = 0;
  for (uint64_t t = 0; t < n_tiles && rc == OR_OK; t++) {
    uint64_t a = t / (S.gy * S.gx), b = (t / S.gx) % S.gy, c = t % S.gx;
    uint64_t ez = (a + 1) * S.tz <= S.nz ? S.tz : S.nz - a * S.tz;
    uint64_t ey = (b + 1) * S.ty <= S.ny ? S.ty : S.ny - b * S.ty;
    uint64_t ex = (c + 1) * S.tx <= S.nx ? S.tx : S.nx - c * S.tx;
    uint64_t nt = ez * ey * ex;
    uint64_t w0 = rd_u64(blob + Lo.off_two + 8 * t), w1 = rd_u64(blob + Lo.off_two + 8 * (t + 1));
    if (w1 < w0 || w1 > n_words) { rc = OR_E_CORRUPT; break; }
    uint64_t bitpos = w0 * 32, bitend = w1 * 32;
    for (uint64_t k = 0; k < nt && rc == OR_OK; k += OR_CHUNK) {
      uint64_t cbits = rd_u16(blob + Lo.off_cb + 2 * ci);
      ci++;
      uint64_t start = bitpos;
      uint64_t kend = k + OR_CHUNK < nt ? k + OR_CHUNK : nt;
      for (uint64_t j = k; j < kend; j++) {
        /* decode one codeword: read bits one at a time; a value v of length l
         * is a codeword iff first[l] <= v < first[l] + count[l] (canonical) */
        uint32_t v = 0;
        int s = -1;
        for (int l = 1; l <= OR_LMAX; l++) {
          if (bitpos >= bitend) { rc = OR_E_CORRUPT; break; }
          v = (v << 1) | get_bit(wcopy, bitpos++);
          if (cnt_l[l] > 0 && v >= first_l[l] && v - first_l[l] < cnt_l[l]) {
            s = sorted_sym[base_l[l] + (v - first_l[l])];
            break;
          }
        }
        if (rc != OR_OK) break;
        if (s < 0) { rc = OR_E_CORRUPT; break; }
        int32_t d = 0;
        uint64_t i = perm[p + j];
        if (s == 0) {
          is_out[i] = 1;
        } else {
          int ne = sym_extra_bits(s);
          uint32_t ev = 0;
          for (int u = 0; u < ne; u++) {
            if (bitpos >= bitend) { rc = OR_E_CORRUPT; break; }
            ev = (ev << 1) | get_bit(wcopy, bitpos++);
          }
          d = or_unsymbol(s, ev);
        }
        dl[i] = d;
      }
      if (rc == OR_OK && bitpos - start != cbits) rc = OR_E_CORRUPT;
    }
    p += nt;
  }
  /* outlier residuals and patches from the exception list */
  uint8_t *patched = (uint8_t *)calloc(n, 1);
  uint64_t *pbits = (uint64_t *)calloc(n, 8);
  if (rc == OR_OK) {
    for (uint64_t e = 0; e < n_exc; e++) {
      uint32_t key = rd_u32(blob + Lo.off_exc + 8 * e), val = rd_u32(blob + Lo.off_exc + 8 * e + 4);
      uint64_t pos = key & ~OR_TAG_PATCH;
      if (pos >= n) { rc = OR_E_CORRUPT; break; }
      uint64_t i = perm[pos];
      if (key & OR_TAG_PATCH) {
        if (dtype == 0) { pbits[i] = val; }
        else {
          if (e + 1 >= n_exc || rd_u32(blob + Lo.off_exc + 8 * (e + 1)) != key) { rc = OR_E_CORRUPT; break; }
          uint32_t hi = rd_u32(blob + Lo.off_exc + 8 * (e + 1) + 4);
          pbits[i] = (uint64_t)val | ((uint64_t)hi << 32);
          e++;
        }
        patched[i] = 1;
      } else {
        if (!is_out[i] || inloop) { rc = OR_E_CORRUPT; break; }
        dl[i] = (int32_t)val;
        is_out[i] = 2;
      }
    }
    for (uint64_t i = 0; i < n && rc == OR_OK; i++) {
      if (inloop) {
        /* in-loop blobs: the outlier symbol marks exactly the stored points */
        if ((is_out[i] == 1) != (patched[i] != 0)) rc = OR_E_CORRUPT;
      } else if (is_out[i] == 1) {
        rc = OR_E_CORRUPT; /* outlier symbol without a value */
      }
    }
  }
  if (rc == OR_OK && inloop) {
    /* repeat the compressor's in-loop prediction point by point, tile by
     * tile, in stream order (each point's neighbours come before it) */
    stage_end(9);
    uint64_t p2 = 0;
    for (uint64_t t = 0; t < n_tiles; t++) {
      uint64_t a = t / (S.gy * S.gx), b = (t / S.gx) % S.gy, c = t % S.gx;
      uint64_t ez = (a + 1) * S.tz <= S.nz ? S.tz : S.nz - a * S.tz;
      uint64_t ey = (b + 1) * S.ty <= S.ny ? S.ty : S.ny - b * S.ty;
      uint64_t ex = (c + 1) * S.tx <= S.nx ? S.tx : S.nx - c * S.tx;
      uint64_t nt = ez * ey * ex;
      uint64_t z0 = a * S.tz, y0 = b * S.ty, x0 = c * S.tx;
      for (uint64_t k = 0; k < nt; k++, p2++) {
        uint64_t i = perm[p2];
        uint64_t xz = i / (S.ny * S.nx), xy = (i / S.nx) % S.ny, xx = i % S.nx;
        if (dtype == 0) {
          float v;
          if (patched[i]) { uint32_t bb = (uint32_t)pbits[i]; memcpy(&v, &bb, 4); }
          else v = il_pred_f((const float *)out, &S, xz, xy, xx, z0, y0, x0) + (float)dl[i] * e2_f;
          ((float *)out)[i] = v;
        } else {
          double v;
          if (patched[i]) memcpy(&v, &pbits[i], 8);
          else v = il_pred_d((const double *)out, &S, xz, xy, xx, z0, y0, x0) + (double)dl[i] * e2;
          ((double *)out)[i] = v;
        }
      }
    }
    stage_end(11);
  }
  if (rc == OR_OK && xform) {
    /* undo the DC differences, dequantize, inverse transform (H again) */
    stage_end(9);
    const int bs = ndim == 3 ? 64 : ndim == 2 ? 16 : 4;
    const int bz = ndim == 3 ? 4 : 1, by = ndim >= 2 ? 4 : 1;
    uint64_t p2 = 0;
    for (uint64_t t = 0; t < n_tiles; t++) {
      uint64_t a = t / (S.gy * S.gx), b = (t / S.gx) % S.gy, c = t % S.gx;
      uint64_t z0 = a * S.tz, y0 = b * S.ty, x0 = c * S.tx;
      uint64_t ez = z0 + S.tz <= S.nz ? S.tz : S.nz - z0;
      uint64_t ey = y0 + S.ty <= S.ny ? S.ty : S.ny - y0;
      uint64_t ex = x0 + S.tx <= S.nx ? S.tx : S.nx - x0;
      uint32_t dc = 0;
      for (uint64_t kz = 0; kz < ez; kz += bz)
        for (uint64_t ky = 0; ky < ey; ky += by)
          for (uint64_t kx = 0; kx < ex; kx += 4) {
            float bf[64];
            double bd[64];
            for (int u = 0; u < bs; u++) {
              int32_t qv = dl[p2 + u];
              if (u == 0) { dc += (uint32_t)qv; qv = (int32_t)dc; }
              if (dtype == 0) bf[u] = (float)qv * e2_f;
              else bd[u] = (double)qv * e2;
            }
            if (dtype == 0) wht_block_f(bf, ndim);
            else wht_block_d(bd, ndim);
            for (int u = 0; u < bs; u++) {
              int uz = u / 16, uy = (u / 4) % 4, ux = u % 4;
              if (ndim == 2) { uz = 0; uy = u / 4; }
              if (ndim == 1) { uz = 0; uy = 0; }
              uint64_t i = ((z0 + kz + uz) * S.ny + (y0 + ky + uy)) * S.nx + (x0 + kx + ux);
              if (dtype == 0) ((float *)out)[i] = bf[u];
              else ((double *)out)[i] = bd[u];
            }
            p2 += (uint64_t)bs;
          }
    }
    stage_end(11);
  }
  if (!inloop && !xform) stage_end(9);
  if (rc == OR_OK && !inloop && !xform) {
    /* undo the prediction: inclusive prefix sums along x, y and z, over the
     * whole field (GLOBAL) or restarting at every tile edge (TILE).  Sums are
     * taken modulo 2^32; the true bin indexes fit in 32 bits, so the
     * result is exact. */
    uint32_t *qq = (uint32_t *)malloc(4 * n);
    for (uint64_t i = 0; i < n; i++) qq[i] = (uint32_t)dl[i];
    for (uint64_t z = 0; z < S.nz; z++)
      for (uint64_t y = 0; y < S.ny; y++)
        for (uint64_t xx = 1; xx < S.nx; xx++)
          if (!(domain && xx % S.tx == 0))
            qq[(z * S.ny + y) * S.nx + xx] += qq[(z * S.ny + y) * S.nx + xx - 1];
    for (uint64_t z = 0; z < S.nz; z++)
      for (uint64_t y = 1; y < S.ny; y++)
        if (!(domain && y % S.ty == 0))
          for (uint64_t xx = 0; xx < S.nx; xx++)
            qq[(z * S.ny + y) * S.nx + xx] += qq[(z * S.ny + y - 1) * S.nx + xx];
    for (uint64_t z = 1; z < S.nz; z++)
      if (!(domain && z % S.tz == 0))
        for (uint64_t y = 0; y < S.ny; y++)
          for (uint64_t xx = 0; xx < S.nx; xx++)
            qq[(z * S.ny + y) * S.nx + xx] += qq[((z - 1) * S.ny + y) * S.nx + xx];
    stage_end(10);
    /* bin midpoints q * 2 eb; patched points take their exact value */
    for (uint64_t i = 0; i < n; i++) {
      int32_t qi = (int32_t)qq[i];
      if (dtype == 0) {
        float v = (float)qi * e2_f;
        if (patched[i]) { uint32_t b = (uint32_t)pbits[i]; memcpy(&v, &b, 4); }
        ((float *)out)[i] = v;
      } else {
        double v = (double)qi * e2;
        if (patched[i]) memcpy(&v, &pbits[i], 8);
        ((double *)out)[i] = v;
      }
    }
    free(qq);
    stage_end(11);
  }
  free(wcopy); free(perm); free(dl); free(is_out); free(patched); free(pbits);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Eq. 4 (first two lines): MSE, NRMSE = sqrt(MSE)/vr, PSNR = -20 log10 NRMSE */
/* SSE accumulated with Neumaier-compensated summation in float64.          */
/* ------------------------------------------------------------------------ */
int or_stats(const void *x, const void *y, int dtype, uint64_t n, double vr, double eb,
             double *out /* sse, mse, psnr, max_abs_err */, uint64_t *n_over) {
  if (n == 0) return OR_E_INVALID_ARG;
  g_stage[12] = 0.0;
  stage_begin();
  double s = 0.0, comp = 0.0, mx = 0.0;
  uint64_t over = 0;
  for (uint64_t i = 0; i < n; i++) {
    double e = elem(x, dtype, i) - elem(y, dtype, i);
    double e2 = e * e;
    double t = s + e2;
    if (fabs(s) >= fabs(e2)) comp += (s - t) + e2;
    else comp += (e2 - t) + s;
    s = t;
    double ae = fabs(e);
    if (ae > mx) mx = ae;
    if (ae > eb) over++;
  }
  double sse = s + comp;
  double mse = sse / (double)n;
  out[0] = sse;
  out[1] = mse;
  out[2] = -20.0 * log10(sqrt(mse) / vr);
  out[3] = mx;
  *n_over = over;
  stage_end(12);
  return OR_OK;
}

void or_free(void *p) { free(p); }
