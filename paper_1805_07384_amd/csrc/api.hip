// api.hip -- host side of the C ABI declared in include/fpsz.h: argument
// checks, the per-call plan and workspace layout, kernel launches and the one
// synchronizing read-back per call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "fpsz_internal.h"

using namespace fpsz;

struct fpsz_ctx {
  int device;
  char err[512];
  DevParams *host;  // pinned read-back buffer
  bool profiling;
  bool events_made;
  Timer timer;
  int n_stages;
  fpsz_stage_time stages[Timer::kMax];
};

namespace {

fpsz_status fail(fpsz_ctx *c, fpsz_status s, const char *fmt, ...) {
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
fpsz_status make_plan(int ndim, const uint64_t *dims, fpsz_dtype dtype, Plan *P) {
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
  uint64_t off_part, off_hist, off_len, off_code, off_word_state, off_exc_cnt, off_exc_off,
      off_stage, off_codes, zero, total;
};

CompressLayout compress_layout(const Plan &P) {
  CompressLayout L;
  uint64_t o = align256(sizeof(DevParams));
  L.off_part = o;
  o = align256(o + 3 * 8 * (uint64_t)kRangeBlocks);
  L.off_hist = o;
  o = align256(o + 4 * (uint64_t)kNSym);
  L.off_len = o;
  o = align256(o + (uint64_t)kNSym);
  L.off_code = o;
  o = align256(o + 4 * (uint64_t)kNSym);
  L.off_word_state = o;
  o = align256(o + 8 * P.n_tiles);
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
      off_tmp, off_codes, total;
};

DecompressLayout decompress_layout(const Plan &P) {
  DecompressLayout L;
  const uint64_t T = P.n_tiles;
  const uint64_t fz = P.ndim == 3 ? (uint64_t)P.ty * P.tx : 0, fy = P.ndim >= 2 ? (uint64_t)P.tz * P.tx : 0;
  const uint64_t fx = (uint64_t)P.tz * P.ty;
  uint64_t o = align256(sizeof(DevParams));
  L.off_lut = o;
  o = align256(o + 4 * 4096);
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
  L.off_codes = o;
  o = align256(o + 2 * P.n);
  L.total = o;
  return L;
}

uint64_t verify_ws_bytes() { return align256(sizeof(DevParams)) + align256(3 * 8 * (uint64_t)kVerifyBlocks); }

template <typename V> V rd(const uint8_t *p) {
  V v;
  memcpy(&v, p, sizeof(V));
  return v;
}

fpsz_status hip_fail(fpsz_ctx *c, hipError_t e, const char *what) {
  return fail(c, FPSZ_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

Timer *timer_begin(fpsz_ctx *c) {
  c->timer.n = 0;
  c->timer.on = c->profiling && c->events_made;
  c->n_stages = 0;
  return &c->timer;
}

// after the stream has been synchronized: stage i spans marks i-1 .. i
void timer_collect(fpsz_ctx *c) {
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

}  // namespace

extern "C" {

const char *fpsz_version(void) { return "fpsz format 1, gfx950"; }

const char *fpsz_status_str(fpsz_status s) {
  switch (s) {
    case FPSZ_OK: return "ok";
    case FPSZ_E_INVALID_ARG: return "invalid argument";
    case FPSZ_E_NONFINITE: return "field holds NaN or Inf";
    case FPSZ_E_RANGE: return "target PSNR needs more bins than the precision allows";
    case FPSZ_E_CORRUPT: return "corrupt blob";
    case FPSZ_E_CAPACITY: return "buffer too small";
    case FPSZ_E_NOMEM: return "out of memory";
    case FPSZ_E_DEVICE: return "HIP device error";
    case FPSZ_E_UNSUPPORTED: return "unsupported device";
  }
  return "unknown status";
}

const char *fpsz_last_error(const fpsz_ctx *ctx) { return ctx ? ctx->err : "no context"; }

fpsz_status fpsz_create(int hip_device, fpsz_ctx **out) {
  if (!out) return FPSZ_E_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
    return FPSZ_E_UNSUPPORTED;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return FPSZ_E_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FPSZ_E_UNSUPPORTED;
  fpsz_ctx *c = new (std::nothrow) fpsz_ctx;
  if (!c) return FPSZ_E_NOMEM;
  memset(c, 0, sizeof(*c));
  c->device = hip_device;
  DeviceGuard g(hip_device);
  if (!g.ok || hipHostMalloc((void **)&c->host, sizeof(DevParams), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return FPSZ_E_NOMEM;
  }
  *out = c;
  return FPSZ_OK;
}

void fpsz_destroy(fpsz_ctx *ctx) {
  if (!ctx) return;
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->events_made)
    for (int i = 0; i < Timer::kMax; i++) (void)hipEventDestroy(ctx->timer.ev[i]);
  delete ctx;
}

fpsz_status fpsz_set_profiling(fpsz_ctx *ctx, int enable) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  if (enable && !ctx->events_made) {
    DeviceGuard g(ctx->device);
    for (int i = 0; i < Timer::kMax; i++)
      if (hipEventCreate(&ctx->timer.ev[i]) != hipSuccess) {
        for (int j = 0; j < i; j++) (void)hipEventDestroy(ctx->timer.ev[j]);
        return fail(ctx, FPSZ_E_DEVICE, "hipEventCreate failed");
      }
    ctx->events_made = true;
  }
  ctx->profiling = enable != 0;
  return FPSZ_OK;
}

fpsz_status fpsz_last_stage_times(const fpsz_ctx *ctx, fpsz_stage_time *out, int max, int *count) {
  if (!ctx || !count || (max > 0 && !out)) return FPSZ_E_INVALID_ARG;
  const int n = ctx->n_stages < max ? ctx->n_stages : max;
  for (int i = 0; i < n; i++) out[i] = ctx->stages[i];
  *count = ctx->n_stages;
  return FPSZ_OK;
}

fpsz_status fpsz_eb_rel(double target_psnr, double *eb_rel) {
  if (!eb_rel || !isfinite(target_psnr)) return FPSZ_E_INVALID_ARG;
  // Eq. 7
  *eb_rel = sqrt(3.0) * pow(10.0, -target_psnr / 20.0);
  return FPSZ_OK;
}

fpsz_status fpsz_compress_workspace_bytes(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                          uint64_t *bytes) {
  Plan P;
  if (!bytes) return FPSZ_E_INVALID_ARG;
  fpsz_status s = make_plan(ndim, dims, dtype, &P);
  if (s != FPSZ_OK) return s;
  *bytes = compress_layout(P).total;
  return FPSZ_OK;
}

fpsz_status fpsz_decompress_workspace_bytes(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                            uint64_t *bytes) {
  Plan P;
  if (!bytes) return FPSZ_E_INVALID_ARG;
  fpsz_status s = make_plan(ndim, dims, dtype, &P);
  if (s != FPSZ_OK) return s;
  *bytes = decompress_layout(P).total;
  return FPSZ_OK;
}

fpsz_status fpsz_verify_workspace_bytes(uint64_t n, uint64_t *bytes) {
  if (!bytes || n == 0) return FPSZ_E_INVALID_ARG;
  *bytes = verify_ws_bytes();
  return FPSZ_OK;
}

fpsz_status fpsz_compress_bound(int ndim, const uint64_t *dims, fpsz_dtype dtype, uint64_t *bytes) {
  Plan P;
  if (!bytes) return FPSZ_E_INVALID_ARG;
  fpsz_status s = make_plan(ndim, dims, dtype, &P);
  if (s != FPSZ_OK) return s;
  const uint64_t per = 4 + 8 + (dtype == FPSZ_F32 ? 8 : 16);
  *bytes = align8(P.off_exc + per * P.n + 8);
  return FPSZ_OK;
}

fpsz_status fpsz_compress_workspace_offset(int ndim, const uint64_t *dims, fpsz_dtype dtype,
                                           int which, uint64_t *offset) {
  Plan P;
  if (!offset) return FPSZ_E_INVALID_ARG;
  fpsz_status s = make_plan(ndim, dims, dtype, &P);
  if (s != FPSZ_OK) return s;
  const CompressLayout L = compress_layout(P);
  switch (which) {
    case 0: *offset = 0; break;
    case 1: *offset = L.off_hist; break;
    case 2: *offset = L.off_len; break;
    case 3: *offset = L.off_code; break;
    case 4: *offset = L.off_codes; break;
    default: return FPSZ_E_INVALID_ARG;
  }
  return FPSZ_OK;
}

fpsz_status fpsz_compress(fpsz_ctx *ctx, const void *field_dev, int ndim, const uint64_t *dims,
                          fpsz_dtype dtype, double target_psnr, fpsz_domain domain,
                          void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                          uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                          void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
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
  fpsz_eb_rel(target_psnr, &P.eb_rel);

  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  uint8_t *ws = (uint8_t *)workspace_dev;
  CompressWs W;
  W.P = (DevParams *)ws;
  W.range_part = ws + L.off_part;
  W.hist = (uint32_t *)(ws + L.off_hist);
  W.code_len = ws + L.off_len;
  W.code = (uint32_t *)(ws + L.off_code);
  W.exc_cnt = (uint32_t *)(ws + L.off_exc_cnt);
  W.exc_off = (uint64_t *)(ws + L.off_exc_off);
  W.stage = (uint32_t *)(ws + L.off_stage);
  W.word_state = (uint64_t *)(ws + L.off_word_state);
  W.codes = (int16_t *)(ws + L.off_codes);
  W.zero_bytes = L.zero;
  hipStream_t s = (hipStream_t)stream;
  Timer *tm = timer_begin(ctx);
  hipError_t e = launch_compress(P, field_dev, W, (uint8_t *)blob_dev, s, tm);
  if (e != hipSuccess) return hip_fail(ctx, e, "compress launch");
  e = hipMemcpyAsync(ctx->host, W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "read-back");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "compress");
  timer_collect(ctx);
  const DevParams &D = *ctx->host;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->target_psnr = target_psnr;
    info->eb_rel = P.eb_rel;
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
    info->domain = (uint32_t)domain;
  }
  if (D.status == FPSZ_E_NONFINITE)
    return fail(ctx, FPSZ_E_NONFINITE, "%llu non-finite values", (unsigned long long)D.nonfinite);
  if (D.status == FPSZ_E_RANGE)
    return fail(ctx, FPSZ_E_RANGE, "max|x| / (2 eb) exceeds the integer range of %s",
                dtype == FPSZ_F32 ? "float32 (2^23)" : "float64 (2^27)");
  if (D.status != 0) return fail(ctx, (fpsz_status)D.status, "device status %u", D.status);
  if (D.spin_fail) return fail(ctx, FPSZ_E_DEVICE, "device-side wait or invariant failed (code %u)", D.spin_fail);
  *blob_bytes = D.blob_bytes;
  if (D.overflow || D.blob_bytes > blob_capacity)
    return fail(ctx, FPSZ_E_CAPACITY, "blob needs %llu bytes, capacity %llu",
                (unsigned long long)D.blob_bytes, (unsigned long long)blob_capacity);
  return FPSZ_OK;
}

fpsz_status fpsz_blob_header(const void *blob_host, uint64_t bytes, int *ndim, uint64_t *dims,
                             fpsz_dtype *dtype, fpsz_info *info) {
  if (!blob_host || bytes < kHdr || !ndim || !dims || !dtype) return FPSZ_E_INVALID_ARG;
  const uint8_t *h = (const uint8_t *)blob_host;
  if (rd<uint32_t>(h + H_MAGIC) != kMagic || rd<uint16_t>(h + H_VERSION) != kVersion)
    return FPSZ_E_CORRUPT;
  const int nd = h[H_NDIM], dt = h[H_DTYPE];
  if (nd < 1 || nd > 3 || dt > 1) return FPSZ_E_CORRUPT;
  *ndim = nd;
  *dtype = (fpsz_dtype)dt;
  for (int i = 0; i < 3; i++) dims[i] = rd<uint64_t>(h + H_DIMS + 8 * i);
  if (info) {
    memset(info, 0, sizeof(*info));
    info->target_psnr = rd<double>(h + H_PSNR);
    info->eb_rel = rd<double>(h + H_EBREL);
    info->vr = rd<double>(h + H_VR);
    info->eb = rd<double>(h + H_EB);
    info->min = rd<double>(h + H_MIN);
    info->max = rd<double>(h + H_MAX);
    info->n = rd<uint64_t>(h + H_N);
    info->n_outliers = rd<uint64_t>(h + H_NOUT);
    info->n_patches = rd<uint64_t>(h + H_NPATCH);
    info->n_exceptions = rd<uint64_t>(h + H_NEXC);
    info->blob_bytes = rd<uint64_t>(h + H_BYTES);
    info->bits_per_value = info->n ? 8.0 * (double)info->blob_bytes / (double)info->n : 0.0;
    const uint16_t fl = rd<uint16_t>(h + H_FLAGS);
    info->is_const = (fl & kFlagConst) ? 1 : 0;
    info->domain = (fl & kFlagTile) ? 1 : 0;
  }
  return FPSZ_OK;
}

fpsz_status fpsz_decompress(fpsz_ctx *ctx, const void *blob_dev, uint64_t blob_bytes,
                            void *workspace_dev, uint64_t workspace_bytes, void *field_out_dev,
                            uint64_t out_bytes, void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!blob_dev || !workspace_dev || !field_out_dev)
    return fail(ctx, FPSZ_E_INVALID_ARG, "null pointer argument");
  if (blob_bytes < kHdr || blob_bytes % 8) return fail(ctx, FPSZ_E_CORRUPT, "blob size %llu", (unsigned long long)blob_bytes);
  if ((uintptr_t)blob_dev % 8 || (uintptr_t)workspace_dev % 256)
    return fail(ctx, FPSZ_E_INVALID_ARG, "blob must be 8-aligned, workspace 256-aligned");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  uint8_t *hh = (uint8_t *)ctx->host;  // sizeof(DevParams) >= 256
  static_assert(sizeof(DevParams) >= kHdr, "read-back buffer holds a header");
  hipError_t e = hipMemcpyAsync(hh, blob_dev, kHdr, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "header read");
  uint8_t h[kHdr];
  memcpy(h, hh, kHdr);
  int nd;
  uint64_t dims[3];
  fpsz_dtype dt;
  if (fpsz_blob_header(h, kHdr, &nd, dims, &dt, nullptr) != FPSZ_OK)
    return fail(ctx, FPSZ_E_CORRUPT, "bad magic, version, ndim or dtype");
  Plan P;
  if (make_plan(nd, dims, dt, &P) != FPSZ_OK) return fail(ctx, FPSZ_E_CORRUPT, "bad dims in header");
  if (rd<uint64_t>(h + H_BYTES) != blob_bytes || rd<uint64_t>(h + H_N) != P.n)
    return fail(ctx, FPSZ_E_CORRUPT, "size fields disagree with the blob");
  const size_t esz = dt == FPSZ_F32 ? 4 : 8;
  if (out_bytes < P.n * esz)
    return fail(ctx, FPSZ_E_CAPACITY, "output needs %llu bytes", (unsigned long long)(P.n * esz));
  if ((uintptr_t)field_out_dev % esz) return fail(ctx, FPSZ_E_INVALID_ARG, "output not element-aligned");
  const uint16_t flags = rd<uint16_t>(h + H_FLAGS);
  P.domain = (flags & kFlagTile) ? FPSZ_DOMAIN_TILE : FPSZ_DOMAIN_GLOBAL;
  P.capacity = blob_bytes;
  if (flags & kFlagConst) {
    if (blob_bytes != kHdr) return fail(ctx, FPSZ_E_CORRUPT, "constant blob size");
    // the header checksum still has to hold
    if (workspace_bytes < align256(sizeof(DevParams)))
      return fail(ctx, FPSZ_E_CAPACITY, "workspace too small");
    DevParams *dp = (DevParams *)workspace_dev;
    e = launch_fill_zero(dp, sizeof(DevParams), s);
    if (e == hipSuccess) e = launch_checksum((const uint8_t *)blob_dev, kHdr, dp, s);
    if (e == hipSuccess) e = launch_const_fill_bits(P, rd<uint64_t>(h + H_CONST), field_out_dev, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->host, dp, sizeof(DevParams), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "constant fill");
    if (ctx->host->checksum != rd<uint64_t>(h + H_CSUM)) return fail(ctx, FPSZ_E_CORRUPT, "checksum mismatch");
    return FPSZ_OK;
  }
  if (rd<uint64_t>(h + H_NTILES) != P.n_tiles || rd<uint64_t>(h + H_NCHUNKS) != P.n_chunks)
    return fail(ctx, FPSZ_E_CORRUPT, "tile / chunk counts disagree with the shape");
  if (rd<uint32_t>(h + H_TILE) != P.tz || rd<uint32_t>(h + H_TILE + 4) != P.ty ||
      rd<uint32_t>(h + H_TILE + 8) != P.tx || rd<uint32_t>(h + H_CHUNK) != (uint32_t)kChunk ||
      h[H_LMAX] != kLMax)
    return fail(ctx, FPSZ_E_CORRUPT, "format constants differ");
  const uint64_t n_words = rd<uint64_t>(h + H_NWORDS), n_exc = rd<uint64_t>(h + H_NEXC);
  if (n_exc > 3 * P.n || n_words > blob_bytes / 4)
    return fail(ctx, FPSZ_E_CORRUPT, "section counts out of range");
  const uint64_t off_words = align8(P.off_exc + 8 * n_exc);
  if (align8(off_words + 4 * n_words) != blob_bytes)
    return fail(ctx, FPSZ_E_CORRUPT, "section sizes disagree with the blob size");
  const DecompressLayout L = decompress_layout(P);
  if (workspace_bytes < L.total)
    return fail(ctx, FPSZ_E_CAPACITY, "workspace needs %llu bytes", (unsigned long long)L.total);
  const uint64_t e2b = rd<uint64_t>(h + H_E2T);
  double e2;
  float e2_f;
  memcpy(&e2, &e2b, 8);
  const uint32_t e2fb = (uint32_t)e2b;
  memcpy(&e2_f, &e2fb, 4);
  uint8_t *ws = (uint8_t *)workspace_dev;
  DecompressWs W;
  W.P = (DevParams *)ws;
  W.lut = (uint32_t *)(ws + L.off_lut);
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
  W.zero_bytes = align256(sizeof(DevParams));
  Timer *tm = timer_begin(ctx);
  e = launch_decompress_args(P, (const uint8_t *)blob_dev, W, off_words, n_words, n_exc, e2, e2_f,
                             field_out_dev, s, tm);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress launch");
  e = hipMemcpyAsync(ctx->host, W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress");
  timer_collect(ctx);
  if (ctx->host->corrupt) return fail(ctx, FPSZ_E_CORRUPT, "blob failed a consistency check");
  return FPSZ_OK;
}

fpsz_status fpsz_verify(fpsz_ctx *ctx, const void *orig_dev, const void *recon_dev, uint64_t n,
                        fpsz_dtype dtype, double vr, double eb, void *workspace_dev,
                        uint64_t workspace_bytes, fpsz_stats *out, void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!orig_dev || !recon_dev || !workspace_dev || !out || n == 0)
    return fail(ctx, FPSZ_E_INVALID_ARG, "null pointer or empty field");
  if (dtype != FPSZ_F32 && dtype != FPSZ_F64) return fail(ctx, FPSZ_E_INVALID_ARG, "bad dtype");
  if (workspace_bytes < verify_ws_bytes() || (uintptr_t)workspace_dev % 256)
    return fail(ctx, FPSZ_E_CAPACITY, "verify workspace needs %llu bytes, 256-aligned",
                (unsigned long long)verify_ws_bytes());
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  DevParams *dp = (DevParams *)workspace_dev;
  void *part = (uint8_t *)workspace_dev + align256(sizeof(DevParams));
  Timer *tm = timer_begin(ctx);
  hipError_t e = launch_verify(orig_dev, recon_dev, n, dtype, eb, dp, part, s, tm);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->host, dp, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "verify");
  timer_collect(ctx);
  const DevParams &D = *ctx->host;
  out->sse = D.v_sse;
  out->mse = D.v_sse / (double)n;
  // Eq. 4: PSNR = -20 log10(NRMSE), NRMSE = sqrt(MSE) / vr
  out->psnr = -20.0 * log10(sqrt(out->mse) / vr);
  out->max_abs_err = D.v_max;
  out->n_over_eb = D.v_over;
  return FPSZ_OK;
}

}  // extern "C"
