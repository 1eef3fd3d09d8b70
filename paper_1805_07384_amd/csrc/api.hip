// api.hip -- host side of the C ABI declared in include/fpsz.h: argument
// checks, the per-call plan and workspace layout, kernel launches and the one
// synchronizing read-back per call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "host_common.h"

using namespace fpsz;

// Device workspace of fpsz_compress_static.  In host code `scratch` names a
// host-side stand-in, not the device address: kernels and copies get the
// per-device address looked up in fpsz_create (scratch_ptr).
static __device__ __align__(256) uint8_t scratch[FPSZ_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Once per device, with that device current.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  if (e == hipSuccess) g_scratch_ptr[dev] = p;
}

void *scratch_ptr(int dev, hipError_t *err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
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
  // the static workspace's address on this device (fpsz_compress_static
  // reports a failure here when it is called)
  scratch_setup(hip_device);
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

static fpsz_status compress_one(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                fpsz_domain domain, void *workspace_dev, uint64_t workspace_bytes,
                                void *blob_dev, uint64_t blob_capacity, uint64_t *blob_bytes,
                                fpsz_info *info, void *stream, int closed,
                                int variant = kVarPlain) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  CJob job;
  fpsz_status st = prepare_compress(ctx, field_dev, ndim, dims, dtype, target_psnr, domain,
                                    workspace_dev, workspace_bytes, blob_dev, blob_capacity,
                                    blob_bytes, &job);
  if (st != FPSZ_OK) return st;
  job.P.closed = closed;
  job.P.variant = variant;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  Timer *tm = timer_begin(ctx);
  hipError_t e = launch_compress_jobs(job, nullptr, 1, job.P, default_launch_cfg(job.P), s, tm);
  if (e != hipSuccess) return hip_fail(ctx, e, "compress launch");
  e = hipMemcpyAsync(ctx->host, job.W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "read-back");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "compress");
  timer_collect(ctx);
  const DevParams &D = *ctx->host;
  if (info) fill_compress_info(info, job.P, D);
  return compress_result(ctx, job.P, D, blob_bytes);
}

fpsz_status fpsz_compress_async(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                fpsz_domain domain, void *workspace_dev, uint64_t workspace_bytes,
                                void *blob_dev, uint64_t blob_capacity,
                                fpsz_async_result *result_dev, void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!result_dev || (uintptr_t)result_dev % 8)
    return fail(ctx, FPSZ_E_INVALID_ARG, "result must be a non-null 8-aligned device pointer");
  CJob job;
  uint64_t nb = 0;
  fpsz_status st = prepare_compress(ctx, field_dev, ndim, dims, dtype, target_psnr, domain,
                                    workspace_dev, workspace_bytes, blob_dev, blob_capacity, &nb,
                                    &job);
  if (st != FPSZ_OK) return st;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  Timer off;  // no events: nothing to collect without a synchronization
  hipError_t e = launch_compress_jobs(job, nullptr, 1, job.P, default_launch_cfg(job.P), s, &off);
  if (e == hipSuccess) e = launch_async_result(job, result_dev, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "compress launch");
  return FPSZ_OK;
}

fpsz_status fpsz_compress(fpsz_ctx *ctx, const void *field_dev, int ndim, const uint64_t *dims,
                          fpsz_dtype dtype, double target_psnr, fpsz_domain domain,
                          void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                          uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                          void *stream) {
  return compress_one(ctx, field_dev, ndim, dims, dtype, target_psnr, domain, workspace_dev,
                      workspace_bytes, blob_dev, blob_capacity, blob_bytes, info, stream, 0);
}

fpsz_status fpsz_compress_inloop(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                 const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                 void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                                 uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                                 void *stream) {
  return compress_one(ctx, field_dev, ndim, dims, dtype, target_psnr, FPSZ_DOMAIN_TILE,
                      workspace_dev, workspace_bytes, blob_dev, blob_capacity, blob_bytes, info,
                      stream, 0, kVarInloop);
}

fpsz_status fpsz_compress_xform(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                void *workspace_dev, uint64_t workspace_bytes, void *blob_dev,
                                uint64_t blob_capacity, uint64_t *blob_bytes, fpsz_info *info,
                                void *stream) {
  if (ctx) ctx->err[0] = 0;
  if (!ctx || !dims || ndim < 1 || ndim > 3) return FPSZ_E_INVALID_ARG;
  for (int i = 0; i < ndim; i++)
    if (dims[i] % 4) return fail(ctx, FPSZ_E_INVALID_ARG, "dims must be multiples of 4");
  return compress_one(ctx, field_dev, ndim, dims, dtype, target_psnr, FPSZ_DOMAIN_TILE,
                      workspace_dev, workspace_bytes, blob_dev, blob_capacity, blob_bytes, info,
                      stream, 0, kVarXform);
}

fpsz_status fpsz_compress_closed_loop(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                      const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                      fpsz_domain domain, void *workspace_dev,
                                      uint64_t workspace_bytes, void *blob_dev,
                                      uint64_t blob_capacity, uint64_t *blob_bytes,
                                      fpsz_info *info, void *stream) {
  return compress_one(ctx, field_dev, ndim, dims, dtype, target_psnr, domain, workspace_dev,
                      workspace_bytes, blob_dev, blob_capacity, blob_bytes, info, stream, 1);
}

fpsz_status fpsz_compress_static(fpsz_ctx *ctx, const void *field_dev, int ndim,
                                 const uint64_t *dims, fpsz_dtype dtype, double target_psnr,
                                 fpsz_domain domain, void *blob_dev, uint64_t blob_capacity,
                                 uint64_t *blob_bytes, fpsz_info *info, void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (blob_bytes) *blob_bytes = 0;
  Plan P;
  if (make_plan(ndim, dims, dtype, &P) != FPSZ_OK)
    return fail(ctx, FPSZ_E_INVALID_ARG, "bad shape or dtype");
  const uint64_t need = compress_layout(P).total;
  if (need > FPSZ_STATIC_WORKSPACE_BYTES)
    return fail(ctx, FPSZ_E_CAPACITY, "field needs %llu workspace bytes; the static workspace holds %llu",
                (unsigned long long)need, (unsigned long long)FPSZ_STATIC_WORKSPACE_BYTES);
  hipError_t e = hipSuccess;
  void *ws = scratch_ptr(ctx->device, &e);
  if (!ws) return fail(ctx, FPSZ_E_DEVICE, "static workspace address: %s", hipGetErrorString(e));
  return fpsz_compress(ctx, field_dev, ndim, dims, dtype, target_psnr, domain, ws,
                       FPSZ_STATIC_WORKSPACE_BYTES, blob_dev, blob_capacity, blob_bytes, info,
                       stream);
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
    info->eb_scale = (fl & kFlagClosed) ? rd<double>(h + H_SCALE) : 1.0;
    info->variant = (fl & kFlagInloop) ? kVarInloop : (fl & kFlagXform) ? kVarXform : kVarPlain;
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
  if (blob_bytes < kHdr || blob_bytes % 8)
    return fail(ctx, FPSZ_E_CORRUPT, "blob size %llu", (unsigned long long)blob_bytes);
  if ((uintptr_t)blob_dev % 8) return fail(ctx, FPSZ_E_INVALID_ARG, "blob must be 8-aligned");
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
  DJob J;
  fpsz_status st = prepare_decompress(ctx, h, blob_dev, blob_bytes, workspace_dev, workspace_bytes,
                                      field_out_dev, out_bytes, &J);
  if (st != FPSZ_OK) return st;
  Timer *tm = timer_begin(ctx);
  e = launch_decompress_job(J, s, tm);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress launch");
  e = hipMemcpyAsync(ctx->host, J.W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress");
  timer_collect(ctx);
  return decompress_result(ctx, J, *ctx->host);
}

fpsz_status fpsz_decompress_async(fpsz_ctx *ctx, const void *blob_dev, uint64_t blob_bytes,
                                  const void *header_host, void *workspace_dev,
                                  uint64_t workspace_bytes, void *field_out_dev,
                                  uint64_t out_bytes, const void *orig_dev,
                                  fpsz_decompress_result *result_dev, void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!blob_dev || !header_host || !workspace_dev || !field_out_dev || !result_dev)
    return fail(ctx, FPSZ_E_INVALID_ARG, "null pointer argument");
  if ((uintptr_t)result_dev % 8) return fail(ctx, FPSZ_E_INVALID_ARG, "result must be 8-aligned");
  if (blob_bytes < kHdr || blob_bytes % 8)
    return fail(ctx, FPSZ_E_CORRUPT, "blob size %llu", (unsigned long long)blob_bytes);
  if ((uintptr_t)blob_dev % 8) return fail(ctx, FPSZ_E_INVALID_ARG, "blob must be 8-aligned");
  HdrBytes hb;
  memcpy(hb.w, header_host, kHdr);
  DJob J;
  fpsz_status st = prepare_decompress(ctx, reinterpret_cast<const uint8_t *>(hb.w), blob_dev,
                                      blob_bytes, workspace_dev, workspace_bytes, field_out_dev,
                                      out_bytes, &J);
  if (st != FPSZ_OK) return st;
  if (orig_dev) {
    if (!J.W.vpart)
      return fail(ctx, FPSZ_E_CAPACITY, "workspace needs %llu bytes",
                  (unsigned long long)decompress_layout(J.P).total);
    const size_t esz = J.P.dtype == FPSZ_F32 ? 4 : 8;
    if ((uintptr_t)orig_dev % esz)
      return fail(ctx, FPSZ_E_INVALID_ARG, "original not element-aligned");
    J.ref = orig_dev;
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  Timer off;  // no events: nothing to collect without a synchronization
  hipError_t e = launch_decompress_job(J, s, &off, &hb);
  if (e == hipSuccess)
    e = launch_dasync_result(J.W.P, result_dev, J.is_const ? 1 : 0, J.csum, orig_dev ? 1 : 0,
                             J.P.n, J.vr, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress launch");
  return FPSZ_OK;
}

fpsz_status fpsz_decompress_verify(fpsz_ctx *ctx, const void *blob_dev, uint64_t blob_bytes,
                                   void *workspace_dev, uint64_t workspace_bytes,
                                   void *field_out_dev, uint64_t out_bytes, const void *orig_dev,
                                   fpsz_stats *out, void *stream) {
  if (!ctx) return FPSZ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!blob_dev || !workspace_dev || !field_out_dev || !orig_dev || !out)
    return fail(ctx, FPSZ_E_INVALID_ARG, "null pointer argument");
  if (blob_bytes < kHdr || blob_bytes % 8)
    return fail(ctx, FPSZ_E_CORRUPT, "blob size %llu", (unsigned long long)blob_bytes);
  if ((uintptr_t)blob_dev % 8) return fail(ctx, FPSZ_E_INVALID_ARG, "blob must be 8-aligned");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, FPSZ_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  uint8_t *hh = (uint8_t *)ctx->host;
  hipError_t e = hipMemcpyAsync(hh, blob_dev, kHdr, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "header read");
  uint8_t h[kHdr];
  memcpy(h, hh, kHdr);
  DJob J;
  fpsz_status st = prepare_decompress(ctx, h, blob_dev, blob_bytes, workspace_dev, workspace_bytes,
                                      field_out_dev, out_bytes, &J);
  if (st != FPSZ_OK) return st;
  if (!J.W.vpart)
    return fail(ctx, FPSZ_E_CAPACITY, "workspace needs %llu bytes",
                (unsigned long long)decompress_layout(J.P).total);
  const size_t esz = J.P.dtype == FPSZ_F32 ? 4 : 8;
  if ((uintptr_t)orig_dev % esz) return fail(ctx, FPSZ_E_INVALID_ARG, "original not element-aligned");
  J.ref = orig_dev;
  Timer *tm = timer_begin(ctx);
  e = launch_decompress_job(J, s, tm);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress launch");
  e = hipMemcpyAsync(ctx->host, J.W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "decompress");
  timer_collect(ctx);
  const DevParams D = *ctx->host;
  st = decompress_result(ctx, J, D);
  if (st != FPSZ_OK) return st;
  out->sse = D.v_sse;
  out->mse = D.v_sse / (double)J.P.n;
  // Eq. 4: PSNR = -20 log10(NRMSE), NRMSE = sqrt(MSE) / vr
  out->psnr = -20.0 * log10(sqrt(out->mse) / J.vr);
  out->max_abs_err = D.v_max;
  out->n_over_eb = D.v_over;
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
