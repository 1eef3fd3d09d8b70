/*
 * fpsz.h -- C ABI of the MI355X (gfx950) fixed-PSNR SZ-style compressor.
 *
 * Method: D. Tao, S. Di, X. Liang, Z. Chen, F. Cappello, "Fixed-PSNR Lossy
 * Compression for Scientific Data", arXiv:1805.07384.  The user fixes the
 * PSNR of a field; the value-range-relative error bound follows from Eq. 7,
 * eb_rel = sqrt(3) * 10^(-PSNR/20), and an SZ-style prediction + uniform
 * quantization + Huffman compressor runs with eb_abs = eb_rel * vr (Sec. IV,
 * the three-step fixed-PSNR workflow after Eq. 7).  The achieved PSNR is the
 * one measured after decompression (Sec. V, Eq. 4).
 *
 * Conventions for every entry point:
 *  - Device pointers are plain HIP device addresses (e.g. torch tensor
 *    data_ptr()); host pointers are ordinary process memory.  The caller owns
 *    every buffer; the library never frees caller memory and allocates
 *    nothing per call (only the small context in fpsz_create).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is stream-ordered.  Entry points that return host values
 *    (sizes, fpsz_info, fpsz_stats) synchronize that stream before returning.
 *  - Fields are C-ordered with dims given slowest-first (NumPy order);
 *    ndim is 1, 2 or 3 and the element count must be below 2^31.
 *  - Errors are status codes; no exception crosses the ABI.  On an error the
 *    contents of output buffers are undefined.  fpsz_last_error() gives a
 *    message for the last failing call on a context.
 *  - Calls on one context must not overlap in time (one host thread per
 *    context at a time).  Separate contexts are independent.
 */
#ifndef FPSZ_H
#define FPSZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FPSZ_F32 = 0, FPSZ_F64 = 1 } fpsz_dtype;

/* Lorenzo prediction domain.  GLOBAL: the predictor reads zero only outside
 * the field (the prefix-sum inverse spans the whole field).  TILE: it reads
 * zero outside each 8192-point tile.  Both reconstruct the same values
 * (Theorem 1 and Theorem 3: the error is that of the quantizer alone); only
 * the bitstream differs. */
typedef enum { FPSZ_DOMAIN_GLOBAL = 0, FPSZ_DOMAIN_TILE = 1 } fpsz_domain;

typedef enum {
  FPSZ_OK = 0,
  FPSZ_E_INVALID_ARG = 1, /* bad dims/ndim/dtype/target/sizes/pointers */
  FPSZ_E_NONFINITE = 2,   /* the field holds NaN or Inf */
  FPSZ_E_RANGE = 3,       /* target needs more than 2^23 (f32) / 2^27 (f64) bins */
  FPSZ_E_CORRUPT = 4,     /* blob fails its checks (magic, sizes, checksum, code) */
  FPSZ_E_CAPACITY = 5,    /* a caller buffer is too small; see the entry point */
  FPSZ_E_NOMEM = 6,       /* context allocation failed */
  FPSZ_E_DEVICE = 7,      /* a HIP runtime call failed */
  FPSZ_E_UNSUPPORTED = 8  /* no gfx950 device / feature not built */
} fpsz_status;

typedef struct fpsz_ctx fpsz_ctx;

/* Per-call report of fpsz_compress. */
typedef struct {
  double target_psnr; /* as requested */
  double eb_rel;      /* Eq. 7 */
  double vr;          /* value range max - min of the input (definition under Eq. 4) */
  double eb;          /* eb_abs = eb_rel * vr (remark after Eq. 6) */
  double min, max;
  uint64_t n;            /* element count */
  uint64_t n_outliers;   /* residuals |d| >= 2^15 kept in the exception list */
  uint64_t n_patches;    /* points stored exactly (float rounding past eb) */
  uint64_t n_exceptions; /* 8-byte exception records in the blob */
  uint64_t blob_bytes;
  double bits_per_value; /* 8 * blob_bytes / n */
  uint32_t is_const;     /* vr == 0: the blob only records the value */
  uint32_t domain;       /* fpsz_domain used */
  double eb_scale;       /* closed loop: factor applied to Eq. 7's eb_rel (eb_rel above
                            includes it); 1 for plain compression */
  uint32_t variant;      /* 0 plain, 1 in-loop prediction (fpsz_compress_inloop),
                            2 block transform (fpsz_compress_xform) */
  uint32_t reserved;
} fpsz_info;

/* Eq. 4: SSE, MSE = SSE / n, PSNR = -20 log10(sqrt(MSE) / vr), max |x - x'|,
 * and the number of points with |x - x'| > eb.  All in float64. */
typedef struct {
  double sse, mse, psnr, max_abs_err;
  uint64_t n_over_eb;
} fpsz_stats;

/* Create a context bound to HIP device `hip_device` (must be gfx950).
 * Allocates a few KiB of device memory for status words.  *out receives the
 * context or NULL on error. */
fpsz_status fpsz_create(int hip_device, fpsz_ctx **out);
void fpsz_destroy(fpsz_ctx *ctx);
const char *fpsz_status_str(fpsz_status s);
const char *fpsz_last_error(const fpsz_ctx *ctx);
/* Library version string (format version + build). */
const char *fpsz_version(void);

/* Eq. 7 on the host: eb_rel = sqrt(3) * 10^(-psnr/20).  INVALID_ARG for a
 * non-finite psnr. */
fpsz_status fpsz_eb_rel(double target_psnr, double *eb_rel);

/* Device workspace needed by fpsz_compress / fpsz_decompress / fpsz_verify
 * for a field of this shape and dtype (bytes, 256-aligned).  The workspace is
 * scratch: its contents need not be initialised and are clobbered. */
fpsz_status fpsz_compress_workspace_bytes(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                          uint64_t *bytes);
fpsz_status fpsz_decompress_workspace_bytes(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                            uint64_t *bytes);
fpsz_status fpsz_verify_workspace_bytes(uint64_t n, uint64_t *bytes);

/* A blob capacity that fits every field of this shape: header, tables, and
 * per point 32 code bits plus its largest possible exception records (an
 * outlier record and a patch of 1 (f32) or 2 (f64) records).  Typical blobs
 * are far smaller; fpsz_compress reports the exact size on FPSZ_E_CAPACITY. */
fpsz_status fpsz_compress_bound(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                uint64_t *bytes);

/* Compress one field at a target PSNR (the three-step fixed-PSNR workflow
 * after Eq. 7: target -> eb_rel -> SZ-style compression with eb_rel * vr).
 *   field_dev      device, ndim/dims/dtype as described; read only
 *   workspace_dev  device scratch of >= fpsz_compress_workspace_bytes
 *   blob_dev       device output of blob_capacity bytes
 *   blob_bytes     host out: size written; on FPSZ_E_CAPACITY the size needed
 *   info           host out, may be NULL
 * Synchronizes `stream`.  Status: INVALID_ARG, NONFINITE, RANGE, CAPACITY,
 * DEVICE.  A constant field (vr == 0) yields a 256-byte blob. */
fpsz_status fpsz_compress(fpsz_ctx *ctx, const void *field_dev, int ndim, const uint64_t *dims,
                          fpsz_dtype dtype, double target_psnr, fpsz_domain domain,
                          void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                          uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                          void *stream);

/* fpsz_compress with a closed-loop correction for low PSNR targets, where
 * Eq. 5's density approximation (many bins across the value range) fails and
 * the achieved PSNR departs from the target.  A first pass over the field
 * measures the MSE of the quantizer's output at the Eq. 7 bound (by Theorem 1
 * the reconstruction error; patched points are exact); one secant step on
 * MSE ~ eb^2 (Eq. 6) then gives eb_rel' = eb_rel * sqrt(MSE_t / MSE_1), with
 * MSE_t = vr^2 10^(-PSNR/10) the MSE that Eq. 4 maps to the target, and the
 * field is compressed with eb_rel'.  The factor is recorded in the blob
 * (header flag 4, float64 at byte 216) and in info->eb_scale; decompression
 * is unchanged.  Costs one extra read of the field.  Arguments, workspace and
 * status as fpsz_compress. */
fpsz_status fpsz_compress_closed_loop(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                      const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                      fpsz_domain domain, void *workspace_dev,
                                      uint64_t workspace_bytes, void *blob_dev,
                                      uint64_t blob_capacity, uint64_t *blob_bytes,
                                      fpsz_info *info, void *stream);

/* The SZ 1.4-style in-loop variant (Sec. II-A step (1), Sec. III Eq. 1): each
 * point's Lorenzo prediction reads the reconstructed values of its preceding
 * neighbours, the prediction error is quantized with bin 2 eb (Eq. 7's bound
 * as in fpsz_compress), and the point is reconstructed at once.  Points whose
 * code leaves the radius 2^15 or whose reconstruction misses eb in floating
 * point are stored exactly.  Prediction runs inside each 8192-point tile
 * (zero outside it; a whole-field in-loop predictor would serialize the
 * field), each tile swept by diagonals on the device.  The blob (header flag
 * 8, tile domain) decompresses with fpsz_decompress; |x - x'| <= eb at every
 * point.  Arguments, workspace and status as fpsz_compress. */
fpsz_status fpsz_compress_inloop(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                 const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                 void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                                 uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                                 void *stream);

/* The orthogonal-transform variant (Sec. III Theorem 2, Sec. IV Theorem 3):
 * blocks of 4 (1D), 4x4 (2D) or 4x4x4 (3D) points are transformed by the
 * orthonormal 4-point Walsh-Hadamard matrix H = 1/2 [[1,1,1,1], [1,1,-1,-1],
 * [1,-1,-1,1], [1,-1,1,-1]] along x, y, z, and the coefficients quantized with
 * bin 2 eb (Eq. 7's bound).  An orthonormal transform keeps the squared error,
 * so the PSNR follows Eq. 7 as for prediction, but there is no pointwise
 * bound.  A block's first (DC) bin is coded as its difference from the
 * previous block's in the tile.  Every dimension must be a multiple of 4
 * (INVALID_ARG otherwise).  The blob (header flag 16, tile domain)
 * decompresses with fpsz_decompress.  Arguments, workspace and status as
 * fpsz_compress. */
fpsz_status fpsz_compress_xform(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                                uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                                void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fpsz_compress
 * with the library's own device workspace instead of workspace_dev.  That
 * workspace is a static array of FPSZ_STATIC_WORKSPACE_BYTES per device (held
 * from the library's load until the process ends); its address is looked up
 * once per device in fpsz_create.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); arguments and results are those of
 * fpsz_compress.  CAPACITY (nothing launched, *blob_bytes = 0) when
 * fpsz_compress_workspace_bytes for the shape exceeds
 * FPSZ_STATIC_WORKSPACE_BYTES; DEVICE when the workspace address could not be
 * had.  Every call on one device shares that device's array and leaves its
 * contents behind (each call clears what it needs): calls that overlap in
 * time on one device, from any contexts or threads, race and corrupt each
 * other's output. */
#define FPSZ_STATIC_WORKSPACE_BYTES (64ull << 20)
fpsz_status fpsz_compress_static(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                 const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                 fpsz_domain domain, void *blob_dev, uint64_t blob_capacity,
                                 uint64_t *blob_bytes, fpsz_info *info, void *stream);

/* Outcome of fpsz_compress_async, written to device memory by the call's last
 * kernel (48 bytes, 8-byte aligned).  status is an fpsz_status as
 * fpsz_compress would return it for the device-side part (NONFINITE, RANGE,
 * CAPACITY when the blob did not fit blob_capacity, DEVICE); blob_bytes is
 * valid when status is OK (and, with CAPACITY, is the size needed). */
typedef struct {
  uint32_t status;
  uint32_t is_const;
  uint64_t blob_bytes;
  uint64_t n_outliers;
  uint64_t n_patches;
  double vr;
  double eb;
} fpsz_async_result;

/* fpsz_compress (Sec. IV workflow after Eq. 7: range, bound, prediction,
 * quantization, Huffman coding) without any synchronization or host read:
 * every step is enqueued on `stream` and the outcome is written to
 * result_dev (device memory, one fpsz_async_result).  The call allocates
 * nothing and makes no memset or copy, so a stream capture of it replays as
 * a graph.  Arguments as fpsz_compress.  The return value covers only what
 * the host checks before enqueueing (INVALID_ARG, CAPACITY for a small
 * workspace); blob and result are defined once the stream reaches the end of
 * the call.  No stage times are recorded. */
fpsz_status fpsz_compress_async(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                fpsz_domain domain, void *workspace_dev, uint64_t workspace_bytes,
                                void *blob_dev, uint64_t blob_capacity,
                                fpsz_async_result *result_dev, void *stream);

/* Parse a blob header held in HOST memory (the first 256 bytes suffice).
 * dims receives 3 entries (unused ones = 1).  CORRUPT on a bad magic or
 * version, INVALID_ARG on NULL pointers or bytes < 256. */
fpsz_status fpsz_blob_header(const void *blob_host, uint64_t bytes, int *ndim, uint64_t *dims,
                             fpsz_dtype *dtype, fpsz_info *info);

/* Outcome of fpsz_decompress_async, written to device memory by the call's
 * last kernel (48 bytes, 8-byte aligned).  status: OK or CORRUPT.  checked:
 * 1 when an original was given, and then stats holds Eq. 4 against it (the
 * PSNR with the blob's value range). */
typedef struct {
  uint32_t status;
  uint32_t checked;
  fpsz_stats stats;
} fpsz_decompress_result;

/* fpsz_decompress / fpsz_decompress_verify (Sec. III reconstruction, Eq. 4
 * check) without any synchronization or host read: the blob's header comes
 * from the caller in HOST memory (header_host, its first 256 bytes, e.g.
 * kept when the blob was stored), so the call needs no device-to-host copy
 * of it; the device checks that the blob in device memory carries the same
 * header (else CORRUPT) besides its checksum.  orig_dev may be NULL (no
 * check).  The outcome goes to result_dev (device memory).  The call
 * allocates nothing and makes no memset or copy, so a stream capture of it
 * replays as a graph (for the same blob header).  Other arguments as
 * fpsz_decompress_verify.  The return value covers only what the host
 * checks before enqueueing (INVALID_ARG, CORRUPT for a malformed host
 * header, CAPACITY for a small workspace or output). */
fpsz_status fpsz_decompress_async(fpsz_ctx *ctx, const void *blob_dev, uint64_t blob_bytes,
                                  const void *header_host, void *workspace_dev,
                                  uint64_t workspace_bytes, void *field_out_dev,
                                  uint64_t out_bytes, const void *orig_dev,
                                  fpsz_decompress_result *result_dev, void *stream);

/* Decompress a blob produced by fpsz_compress (Sec. III: decode, repeat the
 * prediction by inclusive prefix sums, reconstruct bin midpoints q * 2 eb).
 *   blob_dev       device, blob_bytes long; read only
 *   workspace_dev  device scratch of >= fpsz_decompress_workspace_bytes for
 *                  the blob's shape
 *   field_out_dev  device output, out_bytes >= n * element size
 * Synchronizes `stream`.  Status: INVALID_ARG, CORRUPT (header, sizes,
 * checksum, Huffman code or exception list inconsistent), CAPACITY
 * (out_bytes or workspace too small), DEVICE. */
fpsz_status fpsz_decompress(fpsz_ctx *ctx, const void *blob_dev, uint64_t blob_bytes,
                            void *workspace_dev, uint64_t workspace_bytes, void *field_out_dev,
                            uint64_t out_bytes, void *stream);

/* fpsz_decompress, and the Eq. 4 check of the reconstruction against the
 * original in the same pass (Sec. V evaluates every compression by the PSNR
 * it reaches): the statistics of each tile are taken while the tile is
 * written, so field_out_dev is not read back.  vr and eb are the blob's.
 *   orig_dev   device, the original field (n elements of the blob's dtype,
 *              element-aligned); read only
 *   out        host, receives the statistics (fpsz_verify's meaning; the
 *              float64 sum runs over tiles in a fixed order, so repeated
 *              calls return identical bits, which may differ from
 *              fpsz_verify's in the last places)
 * The workspace must hold fpsz_decompress_workspace_bytes for the blob's
 * shape, also for a constant field.  Synchronizes `stream`.  Status: as
 * fpsz_decompress; CAPACITY when the workspace is too small. */
fpsz_status fpsz_decompress_verify(fpsz_ctx *ctx, const void *blob_dev, uint64_t blob_bytes,
                                   void *workspace_dev, uint64_t workspace_bytes,
                                   void *field_out_dev, uint64_t out_bytes, const void *orig_dev,
                                   fpsz_stats *out, void *stream);

/* Eq. 4 check of a reconstruction against the original (both device, n
 * elements of dtype).  vr and eb as reported by fpsz_compress.  The float64
 * reduction order is fixed, so repeated calls return identical bits.
 * Synchronizes `stream`. */
fpsz_status fpsz_verify(fpsz_ctx *ctx, const void *orig_dev, const void *recon_dev, uint64_t n,
                        fpsz_dtype dtype, double vr, double eb, void *workspace_dev,
                        uint64_t workspace_bytes, fpsz_stats *out, void *stream);

/* Per-stage timing.  When enabled, each call records HIP events on its
 * stream between its kernels (a small cost); after the call returns,
 * fpsz_last_stage_times copies up to `max` (stage name, milliseconds) pairs of
 * that call and sets *count to the number recorded.  Enabling creates the
 * events once (DEVICE on failure). */
typedef struct {
  char name[24];
  double ms;
} fpsz_stage_time;
fpsz_status fpsz_set_profiling(fpsz_ctx *ctx, int enable);
fpsz_status fpsz_last_stage_times(const fpsz_ctx *ctx, fpsz_stage_time *out, int max, int *count);

/* Offsets (bytes) of intermediates inside a compress workspace, for tests
 * and diagnostics: which = 0 parameter block, 1 histogram (u32[1036]),
 * 2 code lengths (u8[1036]), 3 codewords (u32[1036]), 4 residual codes in
 * stream order (i16[n]: the residual, or -32768 for an outlier). */
fpsz_status fpsz_compress_workspace_offset(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                           int which, uint64_t *offset);

/* ---- batched compression ------------------------------------------------
 * Many fields, each with its own shape, dtype, target PSNR and Lorenzo
 * domain, compressed together: applications write 100+ fields per snapshot
 * and the user fixes the PSNR of each (Sec. I; the fixed-PSNR workflow after
 * Eq. 7 applied per field).  Fields are grouped by (dtype, ndim, domain);
 * every pipeline step is one launch per group over all its fields.  The
 * blobs are byte-identical to those of one fpsz_compress call per field. */
typedef struct {
  const void *field_dev;  /* device, C order, element-aligned */
  int32_t ndim;           /* 1..3 */
  int32_t dtype;          /* fpsz_dtype */
  uint64_t dims[3];       /* slowest-first; entries past ndim ignored */
  double target_psnr;
  int32_t domain;         /* fpsz_domain */
  int32_t reserved;       /* 0 */
  void *blob_dev;         /* device output, 8-byte aligned */
  uint64_t blob_capacity;
} fpsz_field_desc;

typedef struct fpsz_batch fpsz_batch;

/* Workspace (device, 256-aligned) for a batch of these fields: a job table,
 * a parameter table and one compress workspace per field. */
fpsz_status fpsz_batch_workspace_bytes(int n, const fpsz_field_desc *fields, uint64_t *bytes);

/* Plan a batch of n (1..65535) fields: checks every field (INVALID_ARG /
 * CAPACITY name the field in fpsz_last_error), lays out the workspace,
 * uploads the job table (synchronously) and, with use_graph != 0, captures
 * the whole launch sequence into a hipGraph on a private stream.  The
 * workspace, fields and blobs must stay allocated, and the workspace unused
 * by anything else, until fpsz_batch_destroy.  Host memory of the batch
 * object: O(n). */
fpsz_status fpsz_batch_create(fpsz_ctx *ctx, int n, const fpsz_field_desc *fields,
                              void *workspace_dev, uint64_t workspace_bytes, int use_graph,
                              fpsz_batch **out);

/* Run the batch on `stream` (graph replay when captured), synchronize, and
 * report per field (caller's order): blob_bytes[i] (the size needed on
 * CAPACITY), info[i] (may be NULL) and status[i].  Returns OK when every
 * field succeeded, else the first failing field's status. */
fpsz_status fpsz_batch_run(fpsz_batch *b, void *stream, uint64_t *blob_bytes, fpsz_info *info,
                           fpsz_status *status);

/* Time the batch for candidate launch shapes (grid sizes of the range,
 * quantization, encoding and checksum kernels per field group, one at a time,
 * `reps` runs each, median) and keep the fastest; re-captures the graph.  The
 * shapes do not change any output bit.  *best_ms (may be NULL) receives the
 * best batch time.  The blobs hold valid output of the last timed run. */
fpsz_status fpsz_batch_autotune(fpsz_batch *b, void *stream, int reps, double *best_ms);

/* Current launch shape of field group `cls` (groups in (dtype, ndim, domain)
 * order): shape4 = {range blocks, quantization grid, encode grid, checksum
 * blocks} per field. */
fpsz_status fpsz_batch_launch_shape(const fpsz_batch *b, int cls, uint32_t *shape4);

/* Number of field groups of the batch (the cls range of the shape calls). */
fpsz_status fpsz_batch_class_count(const fpsz_batch *b, int *count);

/* Set the launch shape of field group `cls` (shape4 as above), e.g. one that
 * fpsz_batch_autotune found for the same fields earlier and a cache kept:
 * every entry must lie in 1..the bound that fpsz_batch_autotune uses (the
 * group's tile count for the two grids, 1024 for the range and checksum
 * blocks), else INVALID_ARG and nothing changes.  Re-captures the graph.
 * Shapes do not change any output bit. */
fpsz_status fpsz_batch_set_launch_shape(fpsz_batch *b, int cls, const uint32_t *shape4);

void fpsz_batch_destroy(fpsz_batch *b);

/* One-shot convenience: create (no graph), run, destroy. */
fpsz_status fpsz_compress_batch(fpsz_ctx *ctx, int n, const fpsz_field_desc *fields,
                                void *workspace_dev, uint64_t workspace_bytes,
                                uint64_t *blob_bytes, fpsz_info *info, fpsz_status *status,
                                void *stream);

/* ---- serving ---------------------------------------------------------------
 * A request loop for compress / decompress requests arriving over time, each
 * compress with its own target PSNR (the fixed-PSNR workflow after Eq. 7 per
 * request).  A worker thread admits requests in arrival order while their
 * HBM footprint (input + output + workspace bytes) fits `hbm_budget_bytes`
 * and one of `max_inflight` result slots is free; requests arriving while
 * others run join the next admission round (continuous batching).  Compress
 * requests of one round that share (dtype, ndim, domain) run as one batched
 * launch; rounds go to `n_streams` streams (default priority) and overlap on
 * the device, at most one unfinished round per stream: while every stream is
 * busy, arrivals wait and then form one round together.  Workspaces come from a device arena of `arena_bytes`
 * allocated at creation; no device memory is allocated per request.  Every
 * result is bit-identical to the plain call on the same inputs.
 *
 * Buffers named in a request are the caller's.  Inputs must be complete
 * when the request starts on the device: either their producing work is
 * synchronized before submission, or `ready_event` is a hipEvent_t the caller
 * recorded on the producing stream after that work (the server's stream waits
 * on it before the request's first copy or launch; the event must stay valid,
 * and not be recorded again, until the request is done).  Inputs stay
 * untouched, and outputs must not be read, until the request is done. */
enum { FPSZ_REQ_COMPRESS = 0, FPSZ_REQ_DECOMPRESS = 1 };

typedef struct {
  int32_t kind;         /* FPSZ_REQ_COMPRESS or FPSZ_REQ_DECOMPRESS */
  int32_t ndim;         /* shape of the field (compress input / decompress output) */
  int32_t dtype;        /* fpsz_dtype */
  int32_t domain;       /* fpsz_domain (compress) */
  uint64_t dims[3];     /* slowest-first */
  double target_psnr;   /* compress */
  const void *src_dev;  /* compress: field; decompress: blob */
  uint64_t src_bytes;   /* decompress: blob bytes */
  void *dst_dev;        /* compress: blob buffer; decompress: field buffer */
  uint64_t dst_capacity;
  void *ready_event;    /* hipEvent_t marking the inputs complete, or NULL */
} fpsz_request;

typedef struct {
  fpsz_status status;
  uint32_t reserved;
  uint64_t out_bytes;   /* blob bytes (the size needed on CAPACITY) or field bytes */
  fpsz_info info;       /* compress report, or the decompressed blob's header */
  double t_submit, t_start, t_done; /* seconds on the server's clock */
} fpsz_result;

typedef struct {
  uint64_t submitted, completed, failed;
  uint64_t rounds;            /* admission rounds launched */
  uint64_t batched_launches;  /* compress groups launched as one batch */
  uint64_t peak_inflight;
  uint64_t peak_held_bytes;
  uint64_t held_bytes;        /* now */
  double now;                 /* server clock, seconds */
} fpsz_server_stats;

typedef struct fpsz_server fpsz_server;

/* Create a server on ctx's device (the server uses a private context).
 * INVALID_ARG for zero budgets, max_inflight outside 1..4096 or n_streams
 * outside 1..16; DEVICE / NOMEM when its memory cannot be had. */
fpsz_status fpsz_server_create(fpsz_ctx *ctx, uint64_t hbm_budget_bytes, uint64_t arena_bytes,
                               int max_inflight, int n_streams, fpsz_server **out);
/* Queue a request; *id identifies it.  Malformed requests complete at once
 * with INVALID_ARG; requests larger than the budget complete with CAPACITY. */
fpsz_status fpsz_server_submit(fpsz_server *srv, const fpsz_request *req, uint64_t *id);
/* Non-blocking: *done = 1 and *res filled when the request has finished (its
 * record is then released; an id is reported once). */
fpsz_status fpsz_server_poll(fpsz_server *srv, uint64_t id, int *done, fpsz_result *res);
/* Blocking variant of fpsz_server_poll. */
fpsz_status fpsz_server_wait(fpsz_server *srv, uint64_t id, fpsz_result *res);
fpsz_status fpsz_server_get_stats(fpsz_server *srv, fpsz_server_stats *out);
/* Finishes every submitted request, then frees the server. */
void fpsz_server_destroy(fpsz_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* FPSZ_H */
