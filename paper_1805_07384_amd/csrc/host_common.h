// host_common.h -- host-side helpers shared by the C ABI sources: the
// context, error reporting, the per-field plan (shape, tile grid, fixed blob
// sections), workspace layouts and the stage timer.
#ifndef FPSZ_HOST_COMMON_H
#define FPSZ_HOST_COMMON_H

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "fpsz_internal.h"

struct fpsz_ctx {
  int device;
  char err[512];
  fpsz::DevParams *host;  // pinned read-back buffer
  bool profiling;
  bool events_made;
  fpsz::Timer timer;
  int n_stages;
  fpsz_stage_time stages[fpsz::Timer::kMax];
};

namespace fpsz {


inline fpsz_status fail(fpsz_ctx *c, fpsz_status s, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Normalized shape, tile grid and fixed blob sections.
inline fpsz_status make_plan(int ndim, const uint64_t *dims, fpsz_dtype dtype, Plan *P) {
  if (ndim < 1 || ndim > 3 || !dims) return FPSZ_E_INVALID_ARG;
  if (dtype != FPSZ_F32 && dtype != FPSZ_F64) return FPSZ_E_INVALID_ARG;
  memset(P, 0, sizeof(*P));
  P->ndim = ndim;
  P->dtype = dtype;
  uint64_t d[3] = {1, 1, 1};
  for (int i = 0; i < 3; i++) P->dims[i] = 1;
  for (int i = 0; i < ndim; i++) {
    if (dims[i] == 0 || dims[i] >= (1ull << 31)) return FPSZ_E_INVALID_ARG;
    d[3 - ndim + i] = dims[i];
    P->dims[i] = dims[i];
  }
  P->nz = d[0];
  P->ny = d[1];
  P->nx = d[2];
  const unsigned __int128 n = (unsigned __int128)d[0] * d[1] * d[2];
  if (n >= ((unsigned __int128)1 << 31)) return FPSZ_E_INVALID_ARG;
  P->n = (uint64_t)n;
  if (ndim == 1) { P->tz = 1; P->ty = 1; P->tx = 8192; }
  else if (ndim == 2) { P->tz = 1; P->ty = 64; P->tx = 128; }
  else { P->tz = 16; P->ty = 16; P->tx = 32; }
  P->gz = (uint32_t)ceil_div(P->nz, P->tz);
  P->gy = (uint32_t)ceil_div(P->ny, P->ty);
  P->gx = (uint32_t)ceil_div(P->nx, P->tx);
  P->n_tiles = (uint64_t)P->gz * P->gy * P->gx;
  // pad_: 1 when some tile is clipped by the field's edge
  P->pad_ = (P->nz % P->tz) || (P->ny % P->ty) || (P->nx % P->tx) ? 1 : 0;
  // total chunks = chunk_base of a one-past-the-end tile: sum over all tiles
  {
    const uint64_t ex_last = P->nx - (uint64_t)(P->gx - 1) * P->tx;
    const uint64_t ey_last = P->ny - (uint64_t)(P->gy - 1) * P->ty;
    const uint64_t ez_last = P->nz - (uint64_t)(P->gz - 1) * P->tz;
    auto row = [&](uint64_t ez, uint64_t ey) {
      return (uint64_t)(P->gx - 1) * chunks_of(ez, ey, P->tx) + chunks_of(ez, ey, ex_last);
    };
    auto slab = [&](uint64_t ez) { return (uint64_t)(P->gy - 1) * row(ez, P->ty) + row(ez, ey_last); };
    P->n_chunks = (uint64_t)(P->gz - 1) * slab(P->tz) + slab(ez_last);
  }
  uint64_t o = kHdr;
  P->off_len = o;
  o = align8(o + kNSym);
  P->off_two = o;
  o = align8(o + 8 * (P->n_tiles + 1));
  P->off_teo = o;
  o = align8(o + 8 * (P->n_tiles + 1));
  P->off_cb = o;
  o = align8(o + 2 * P->n_chunks);
  P->off_exc = o;
  return FPSZ_OK;
}

struct CompressLayout {
  uint64_t off_part, off_hist, off_len, off_code, off_word_state, off_w8, off_exc_cnt, off_exc_off,
      off_stage, off_codes, zero, total;
};

inline CompressLayout compress_layout(const Plan &P) {
  CompressLayout L;
  uint64_t o = align256(sizeof(DevParams));
  L.off_part = o;
  o = align256(o + 3 * 8 * (uint64_t)kRangeBlocks);
  L.off_hist = o;
  o = align256(o + 4 * (uint64_t)kNSym * kHistCopies);
  L.off_len = o;
  o = align256(o + (uint64_t)kNSym);
  L.off_code = o;
  o = align256(o + 4 * (uint64_t)kNSym);
  L.off_word_state = o;
  o = align256(o + 8 * P.n_tiles);
  L.off_w8 = o;  // one byte per wave of a tile (4 per tile)
  o = align256(o + 4 * P.n_tiles);
  L.zero = o;  // everything before this is cleared at the start of a call
  L.off_exc_cnt = o;
  o = align256(o + 4 * P.n_tiles);
  L.off_exc_off = o;
  o = align256(o + 8 * P.n_tiles);
  L.off_stage = o;
  o = align256(o + 8 * 64 * P.n_tiles);  // kStage records of 8 bytes per tile
  L.off_codes = o;
  o = align256(o + 2 * P.n);
  L.total = o;
  return L;
}

struct DecompressLayout {
  uint64_t off_lut, off_ltab, off_sorted, off_fz, off_fy, off_fx, off_gx, off_gy, off_gz, off_tt,
      off_tmp, off_vpart, off_codes, off_res8, off_res8m, total;
};

inline DecompressLayout decompress_layout(const Plan &P) {
  DecompressLayout L;
  const uint64_t T = P.n_tiles;
  const uint64_t fz = P.ndim == 3 ? (uint64_t)P.ty * P.tx : 0, fy = P.ndim >= 2 ? (uint64_t)P.tz * P.tx : 0;
  const uint64_t fx = (uint64_t)P.tz * P.ty;
  uint64_t o = align256(sizeof(DevParams));
  L.off_lut = o;
  o = align256(o + 2 * 8192);
  L.off_ltab = o;
  o = align256(o + 4 * 96);
  L.off_sorted = o;
  o = align256(o + 2 * (uint64_t)kNSym);
  L.off_fz = o;
  o = align256(o + 4 * T * fz);
  L.off_fy = o;
  o = align256(o + 4 * T * fy);
  L.off_fx = o;
  o = align256(o + 4 * T * fx);
  L.off_gx = o;
  o = align256(o + 4 * T * (P.ndim == 3 ? P.tx : 0));
  L.off_gy = o;
  o = align256(o + 4 * T * (P.ndim == 3 ? P.ty : 0));
  L.off_gz = o;
  o = align256(o + 4 * T * (P.ndim >= 2 ? P.tz : 0));
  L.off_tt = o;
  o = align256(o + 4 * T);
  // segment sums of a scan with len > 32 along its axis: ceil(len / 32) <=
  // len / 16 per column, so at most one per 16 elements of the largest array
  uint64_t big = T * fz;
  if (T * fy > big) big = T * fy;
  if (T * fx > big) big = T * fx;
  if (T * P.tx > big) big = T * P.tx;
  L.off_tmp = o;
  o = align256(o + 4 * (big / 16 + 64));
  // per-tile partials of the check against the original (also the verify
  // partials of a constant field)
  L.off_vpart = o;
  o = align256(o + 3 * 8 * (T > (uint64_t)kVerifyBlocks ? T : (uint64_t)kVerifyBlocks));
  L.off_codes = o;
  o = align256(o + 2 * P.n);
  L.off_res8 = o;  // int8 residual parts (one byte per point)
  o = align256(o + P.n);
  L.off_res8m = o;  // four 64-bit part masks per tile
  o = align256(o + 32 * T);
  L.total = o;
  return L;
}

inline uint64_t verify_ws_bytes() { return align256(sizeof(DevParams)) + align256(3 * 8 * (uint64_t)kVerifyBlocks); }

template <typename V> V rd(const uint8_t *p) {
  V v;
  memcpy(&v, p, sizeof(V));
  return v;
}

inline fpsz_status hip_fail(fpsz_ctx *c, hipError_t e, const char *what) {
  return fail(c, FPSZ_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

inline Timer *timer_begin(fpsz_ctx *c) {
  c->timer.n = 0;
  c->timer.on = c->profiling && c->events_made;
  c->n_stages = 0;
  return &c->timer;
}

// after the stream has been synchronized: stage i spans marks i-1 .. i
inline void timer_collect(fpsz_ctx *c) {
  Timer &t = c->timer;
  c->n_stages = 0;
  for (int i = 1; i < t.n; i++) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[i - 1], t.ev[i]) != hipSuccess) ms = -1.f;
    fpsz_stage_time &st = c->stages[c->n_stages++];
    memset(st.name, 0, sizeof(st.name));
    strncpy(st.name, t.names[i], sizeof(st.name) - 1);
    st.ms = ms;
  }
  t.on = false;
}


// Checks one compress request and fills its job: plan, input, workspace
// carved from ws (compress_layout), output.  Sets *blob_bytes = 256 when the
// capacity cannot even hold the header.
inline fpsz_status prepare_compress(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                    const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                    fpsz_domain domain, void *workspace_dev,
                                    uint64_t workspace_bytes, void *blob_dev,
                                    uint64_t blob_capacity, uint64_t *blob_bytes, CJob *job) {
  if (!field_dev || !workspace_dev || !blob_dev || !blob_bytes)
    return fail(ctx, FPSZ_E_INVALID_ARG, "null pointer argument");
  if (!isfinite(target_psnr)) return fail(ctx, FPSZ_E_INVALID_ARG, "target PSNR is not finite");
  if (domain != FPSZ_DOMAIN_GLOBAL && domain != FPSZ_DOMAIN_TILE)
    return fail(ctx, FPSZ_E_INVALID_ARG, "bad domain %d", (int)domain);
  Plan P;
  fpsz_status st = make_plan(ndim, dims, dtype, &P);
  if (st != FPSZ_OK) return fail(ctx, st, "bad shape or dtype");
  const size_t esz = dtype == FPSZ_F32 ? 4 : 8;
  if ((uintptr_t)field_dev % esz) return fail(ctx, FPSZ_E_INVALID_ARG, "field not element-aligned");
  if ((uintptr_t)workspace_dev % 256 || (uintptr_t)blob_dev % 8)
    return fail(ctx, FPSZ_E_INVALID_ARG, "workspace must be 256-aligned, blob 8-aligned");
  const CompressLayout L = compress_layout(P);
  if (workspace_bytes < L.total)
    return fail(ctx, FPSZ_E_CAPACITY, "workspace needs %llu bytes", (unsigned long long)L.total);
  *blob_bytes = 0;
  if (blob_capacity < kHdr) {
    *blob_bytes = kHdr;
    return fail(ctx, FPSZ_E_CAPACITY, "blob capacity below the 256-byte header");
  }
  P.domain = domain;
  P.capacity = blob_capacity;
  P.target_psnr = target_psnr;
  P.eb_rel = sqrt(3.0) * pow(10.0, -target_psnr / 20.0);  // Eq. 7, as fpsz_eb_rel
  // the MSE that Eq. 4 maps to the target is vr^2 * 10^(-PSNR/10) (closed loop)
  P.mse_factor = pow(10.0, -target_psnr / 10.0);
  P.closed = 0;
  P.variant = kVarPlain;
  uint8_t *ws = (uint8_t *)workspace_dev;
  CompressWs &W = job->W;
  W.P = (DevParams *)ws;
  W.range_part = ws + L.off_part;
  W.hist = (uint32_t *)(ws + L.off_hist);
  W.code_len = ws + L.off_len;
  W.code = (uint32_t *)(ws + L.off_code);
  W.exc_cnt = (uint32_t *)(ws + L.off_exc_cnt);
  W.exc_off = (uint64_t *)(ws + L.off_exc_off);
  W.stage = (uint32_t *)(ws + L.off_stage);
  W.word_state = (uint64_t *)(ws + L.off_word_state);
  W.code_w8 = ws + L.off_w8;
  W.codes = (int16_t *)(ws + L.off_codes);
  W.zero_bytes = L.zero;
  job->P = P;
  job->x = field_dev;
  job->blob = (uint8_t *)blob_dev;
  return FPSZ_OK;
}

inline void fill_compress_info(fpsz_info *info, const Plan &P, const DevParams &D) {
  memset(info, 0, sizeof(*info));
  info->target_psnr = P.target_psnr;
  info->eb_rel = P.closed ? D.eb_rel : P.eb_rel;  // the closed loop's includes its factor
  info->vr = D.vr;
  info->eb = D.eb;
  info->min = D.mn;
  info->max = D.mx;
  info->n = P.n;
  info->n_outliers = D.n_out;
  info->n_patches = D.n_pat;
  info->n_exceptions = D.n_exc;
  info->blob_bytes = D.blob_bytes;
  info->bits_per_value = 8.0 * (double)D.blob_bytes / (double)P.n;
  info->is_const = D.is_const;
  info->domain = (uint32_t)P.domain;
  info->eb_scale = P.closed ? D.scale : 1.0;
  info->variant = (uint32_t)P.variant;
}

// Status of a finished compress from its parameter block.
inline fpsz_status compress_result(fpsz_ctx *ctx, const Plan &P, const DevParams &D,
                                   uint64_t *blob_bytes) {
  if (D.status == FPSZ_E_NONFINITE)
    return fail(ctx, FPSZ_E_NONFINITE, "%llu non-finite values", (unsigned long long)D.nonfinite);
  if (D.status == FPSZ_E_RANGE)
    return fail(ctx, FPSZ_E_RANGE, "max|x| / (2 eb) exceeds the integer range of %s",
                P.dtype == FPSZ_F32 ? "float32 (2^23)" : "float64 (2^27)");
  if (D.status != 0) return fail(ctx, (fpsz_status)D.status, "device status %u", D.status);
  if (D.spin_fail)
    return fail(ctx, FPSZ_E_DEVICE, "device-side wait or invariant failed (code %u)", D.spin_fail);
  *blob_bytes = D.blob_bytes;
  if (D.overflow || D.blob_bytes > P.capacity)
    return fail(ctx, FPSZ_E_CAPACITY, "blob needs %llu bytes, capacity %llu",
                (unsigned long long)D.blob_bytes, (unsigned long long)P.capacity);
  return FPSZ_OK;
}

// One decompression after its header (a host copy) has been checked.
struct DJob {
  Plan P;
  const uint8_t *blob;
  void *out;
  const void *ref;  // original field to check the reconstruction against, or null
  DecompressWs W;
  uint64_t off_words, n_words, n_exc;
  double e2, eb, vr;
  float e2_f;
  bool is_const;
  uint64_t const_bits, csum;
};

// Checks a blob header held in host memory against the blob size, the output
// buffer and the workspace, and fills the job.
inline fpsz_status prepare_decompress(fpsz_ctx *ctx, const uint8_t *h, const void *blob_dev,
                                      uint64_t blob_bytes, void *workspace_dev,
                                      uint64_t workspace_bytes, void *field_out_dev,
                                      uint64_t out_bytes, DJob *J) {
  if (!blob_dev || !workspace_dev || !field_out_dev)
    return fail(ctx, FPSZ_E_INVALID_ARG, "null pointer argument");
  if (blob_bytes < kHdr || blob_bytes % 8)
    return fail(ctx, FPSZ_E_CORRUPT, "blob size %llu", (unsigned long long)blob_bytes);
  if ((uintptr_t)blob_dev % 8 || (uintptr_t)workspace_dev % 256)
    return fail(ctx, FPSZ_E_INVALID_ARG, "blob must be 8-aligned, workspace 256-aligned");
  if (rd<uint32_t>(h + H_MAGIC) != kMagic || rd<uint16_t>(h + H_VERSION) != kVersion)
    return fail(ctx, FPSZ_E_CORRUPT, "bad magic or version");
  const int nd = h[H_NDIM], dtc = h[H_DTYPE];
  if (nd < 1 || nd > 3 || dtc > 1) return fail(ctx, FPSZ_E_CORRUPT, "bad ndim or dtype");
  uint64_t dims[3];
  for (int i = 0; i < 3; i++) dims[i] = rd<uint64_t>(h + H_DIMS + 8 * i);
  const fpsz_dtype dt = (fpsz_dtype)dtc;
  Plan &P = J->P;
  if (make_plan(nd, dims, dt, &P) != FPSZ_OK) return fail(ctx, FPSZ_E_CORRUPT, "bad dims in header");
  if (rd<uint64_t>(h + H_BYTES) != blob_bytes || rd<uint64_t>(h + H_N) != P.n)
    return fail(ctx, FPSZ_E_CORRUPT, "size fields disagree with the blob");
  const size_t esz = dt == FPSZ_F32 ? 4 : 8;
  if (out_bytes < P.n * esz)
    return fail(ctx, FPSZ_E_CAPACITY, "output needs %llu bytes", (unsigned long long)(P.n * esz));
  if ((uintptr_t)field_out_dev % esz) return fail(ctx, FPSZ_E_INVALID_ARG, "output not element-aligned");
  const uint16_t flags = rd<uint16_t>(h + H_FLAGS);
  P.domain = (flags & kFlagTile) ? FPSZ_DOMAIN_TILE : FPSZ_DOMAIN_GLOBAL;
  P.variant = (flags & kFlagInloop) ? kVarInloop : (flags & kFlagXform) ? kVarXform : kVarPlain;
  if (P.variant != kVarPlain && P.domain != FPSZ_DOMAIN_TILE)
    return fail(ctx, FPSZ_E_CORRUPT, "variant blob outside the tile domain");
  if ((flags & kFlagInloop) && (flags & kFlagXform))
    return fail(ctx, FPSZ_E_CORRUPT, "two variants in one blob");
  if (P.variant == kVarXform)
    for (int i = 0; i < nd; i++)
      if (dims[i] % 4) return fail(ctx, FPSZ_E_CORRUPT, "transform blob dims not multiples of 4");
  P.capacity = blob_bytes;
  J->blob = (const uint8_t *)blob_dev;
  J->out = field_out_dev;
  J->ref = nullptr;
  J->csum = rd<uint64_t>(h + H_CSUM);
  J->is_const = (flags & kFlagConst) != 0;
  J->eb = rd<double>(h + H_EB);
  J->vr = rd<double>(h + H_VR);
  uint8_t *ws = (uint8_t *)workspace_dev;
  if (J->is_const) {
    if (blob_bytes != kHdr) return fail(ctx, FPSZ_E_CORRUPT, "constant blob size");
    if (workspace_bytes < align256(sizeof(DevParams)))
      return fail(ctx, FPSZ_E_CAPACITY, "workspace too small");
    memset(&J->W, 0, sizeof(J->W));
    J->W.P = (DevParams *)ws;
    const DecompressLayout L = decompress_layout(P);
    if (workspace_bytes >= L.off_vpart + 3 * 8 * (uint64_t)kVerifyBlocks)
      J->W.vpart = (double *)(ws + L.off_vpart);
    J->const_bits = rd<uint64_t>(h + H_CONST);
    return FPSZ_OK;
  }
  if (rd<uint64_t>(h + H_NTILES) != P.n_tiles || rd<uint64_t>(h + H_NCHUNKS) != P.n_chunks)
    return fail(ctx, FPSZ_E_CORRUPT, "tile / chunk counts disagree with the shape");
  if (rd<uint32_t>(h + H_TILE) != P.tz || rd<uint32_t>(h + H_TILE + 4) != P.ty ||
      rd<uint32_t>(h + H_TILE + 8) != P.tx || rd<uint32_t>(h + H_CHUNK) != (uint32_t)kChunk ||
      h[H_LMAX] != kLMax)
    return fail(ctx, FPSZ_E_CORRUPT, "format constants differ");
  J->n_words = rd<uint64_t>(h + H_NWORDS);
  J->n_exc = rd<uint64_t>(h + H_NEXC);
  if (J->n_exc > 3 * P.n || J->n_words > blob_bytes / 4)
    return fail(ctx, FPSZ_E_CORRUPT, "section counts out of range");
  J->off_words = align8(P.off_exc + 8 * J->n_exc);
  if (align8(J->off_words + 4 * J->n_words) != blob_bytes)
    return fail(ctx, FPSZ_E_CORRUPT, "section sizes disagree with the blob size");
  const DecompressLayout L = decompress_layout(P);
  if (workspace_bytes < L.total)
    return fail(ctx, FPSZ_E_CAPACITY, "workspace needs %llu bytes", (unsigned long long)L.total);
  const uint64_t e2b = rd<uint64_t>(h + H_E2T);
  memcpy(&J->e2, &e2b, 8);
  const uint32_t e2fb = (uint32_t)e2b;
  memcpy(&J->e2_f, &e2fb, 4);
  DecompressWs &W = J->W;
  W.P = (DevParams *)ws;
  W.lut = (uint16_t *)(ws + L.off_lut);
  W.ltab = (uint32_t *)(ws + L.off_ltab);
  W.sorted = (uint16_t *)(ws + L.off_sorted);
  W.fz = (uint32_t *)(ws + L.off_fz);
  W.fy = (uint32_t *)(ws + L.off_fy);
  W.fx = (uint32_t *)(ws + L.off_fx);
  W.gx = (uint32_t *)(ws + L.off_gx);
  W.gy = (uint32_t *)(ws + L.off_gy);
  W.gz = (uint32_t *)(ws + L.off_gz);
  W.tt = (uint32_t *)(ws + L.off_tt);
  W.tmp = (uint32_t *)(ws + L.off_tmp);
  W.codes = (int16_t *)(ws + L.off_codes);
  W.res8 = ws + L.off_res8;
  W.res8_mask = (uint64_t *)(ws + L.off_res8m);
  W.vpart = (double *)(ws + L.off_vpart);
  W.zero_bytes = align256(sizeof(DevParams));
  return FPSZ_OK;
}

// Enqueues the decompression (no synchronization).
inline hipError_t launch_decompress_job(const DJob &J, hipStream_t s, Timer *tm,
                                        const HdrBytes *hdr = nullptr) {
  if (J.is_const) {
    hipError_t e = launch_fill_zero(J.W.P, sizeof(DevParams), s);
    if (e == hipSuccess && hdr) e = launch_hdr_check(J.blob, *hdr, J.W.P, s);
    if (e == hipSuccess) e = launch_checksum(J.blob, kHdr, J.W.P, s);
    if (e == hipSuccess) e = launch_const_fill_bits(J.P, J.const_bits, J.out, s);
    // a constant field is checked by the plain verify kernels
    if (e == hipSuccess && J.ref)
      e = launch_verify(J.ref, J.out, J.P.n, J.P.dtype, J.eb, J.W.P, J.W.vpart, s, tm);
    return e;
  }
  return launch_decompress_args(J.P, J.blob, J.W, J.off_words, J.n_words, J.n_exc, J.e2, J.e2_f,
                                J.out, J.ref, J.eb, s, tm, hdr);
}

// Status of a finished decompression from its parameter block.
inline fpsz_status decompress_result(fpsz_ctx *ctx, const DJob &J, const DevParams &D) {
  if (J.is_const) {
    if (D.checksum != J.csum) return fail(ctx, FPSZ_E_CORRUPT, "checksum mismatch");
    return FPSZ_OK;
  }
  if (D.corrupt) return fail(ctx, FPSZ_E_CORRUPT, "blob failed a consistency check");
  return FPSZ_OK;
}
}  // namespace fpsz

#endif
