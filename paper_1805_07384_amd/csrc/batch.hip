// batch.hip -- many fields, each with its own shape and target PSNR,
// compressed together.  Applications write 100+ fields per snapshot and the
// user fixes a PSNR per field (Sec. I); this is that workload on one GPU.
//
// Fields are grouped by class (dtype, ndim, Lorenzo domain).  Every step of
// the compress pipeline is one launch per class whose grid has one y-row per
// field (blockIdx.y selects the field's job from a device table), so small
// fields share the machine instead of queueing behind each other: 120
// codebooks run as 120 concurrent workgroups, not 120 serial launches.  The
// whole sequence -- every class, then one gather of the parameter blocks and
// one read-back -- can be captured once into a hipGraph and replayed.  A
// launch-shape autotuner times the bit-neutral grid sizes on the batch
// itself: the tile format is fixed by the blob header, so the output does
// not depend on them.
#include <algorithm>
#include <new>
#include <vector>

#include "host_common.h"

using namespace fpsz;

namespace fpsz {

// Copies each field's parameter block into one table for a single read-back.
__global__ void k_gather_params(const CJob *__restrict__ jobs, DevParams *__restrict__ out) {
  const CJob J = jobs[blockIdx.x];
  const uint32_t *src = reinterpret_cast<const uint32_t *>(J.W.P);
  uint32_t *dst = reinterpret_cast<uint32_t *>(out + blockIdx.x);
  for (uint32_t i = threadIdx.x; i < sizeof(DevParams) / 4; i += blockDim.x) dst[i] = src[i];
}

}  // namespace fpsz

namespace {

struct BatchClass {
  int dtype, ndim, domain;
  int first, count;  // jobs [first, first + count) of the class-ordered table
  Plan maxP;         // class, largest n / n_tiles / capacity
  LaunchCfg cfg;
};

struct BatchLayout {
  uint64_t off_jobs, off_params, off_fields, total;
};

BatchLayout batch_layout(int n, const std::vector<Plan> &plans) {
  BatchLayout L;
  uint64_t o = 0;
  L.off_jobs = o;
  o = align256(o + (uint64_t)n * sizeof(CJob));
  L.off_params = o;
  o = align256(o + (uint64_t)n * sizeof(DevParams));
  L.off_fields = o;
  for (const Plan &P : plans) o += compress_layout(P).total;
  L.total = o;
  return L;
}

}  // namespace

struct fpsz_batch {
  fpsz_ctx *ctx = nullptr;
  int n = 0;
  std::vector<CJob> jobs;   // class-ordered
  std::vector<int> user;    // user[k] = caller's index of job k
  std::vector<BatchClass> classes;
  CJob *jobs_dev = nullptr;
  DevParams *params_dev = nullptr;
  DevParams *params_host = nullptr;  // pinned
  bool use_graph = false;
  bool captured = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
};

namespace {

hipError_t enqueue_batch(fpsz_batch *b, hipStream_t s) {
  Timer off;  // no per-stage events inside a batch
  off.on = false;
  off.n = 0;
  CJob none;
  memset(&none, 0, sizeof(none));
  for (const BatchClass &c : b->classes) {
    hipError_t e = launch_compress_jobs(none, b->jobs_dev + c.first, c.count, c.maxP, c.cfg, s, &off);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gather_params, dim3(b->n), dim3(64), 0, s, b->jobs_dev, b->params_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(b->params_host, b->params_dev, (size_t)b->n * sizeof(DevParams),
                        hipMemcpyDeviceToHost, s);
}

void drop_graph(fpsz_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->captured = false;
}

fpsz_status capture(fpsz_batch *b) {
  drop_graph(b);
  fpsz_ctx *ctx = b->ctx;
  hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(ctx, e, "begin capture");
  hipError_t le = enqueue_batch(b, b->cap_stream);
  e = hipStreamEndCapture(b->cap_stream, &b->graph);
  if (le != hipSuccess) return hip_fail(ctx, le, "batch launch under capture");
  if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return hip_fail(ctx, e, "graph instantiate");
  }
  b->captured = true;
  return FPSZ_OK;
}

// prepare every field's job; plans in caller order
fpsz_status prepare_all(fpsz_ctx *ctx, int n, const fpsz_field_desc *f, uint8_t *ws,
                        uint64_t ws_bytes, std::vector<Plan> *plans, std::vector<CJob> *jobs) {
  plans->resize(n);
  for (int i = 0; i < n; i++) {
    if (make_plan(f[i].ndim, f[i].dims, (fpsz_dtype)f[i].dtype, &(*plans)[i]) != FPSZ_OK)
      return fail(ctx, FPSZ_E_INVALID_ARG, "field %d: bad shape or dtype", i);
  }
  const BatchLayout L = batch_layout(n, *plans);
  if (ws && ws_bytes < L.total)
    return fail(ctx, FPSZ_E_CAPACITY, "batch workspace needs %llu bytes",
                (unsigned long long)L.total);
  if (!jobs) return FPSZ_OK;
  jobs->resize(n);
  uint64_t o = L.off_fields;
  for (int i = 0; i < n; i++) {
    const uint64_t need = compress_layout((*plans)[i]).total;
    uint64_t bb = 0;
    fpsz_status st = prepare_compress(ctx, f[i].field_dev, f[i].ndim, f[i].dims,
                                      (fpsz_dtype)f[i].dtype, f[i].target_psnr,
                                      (fpsz_domain)f[i].domain, ws + o, need, f[i].blob_dev,
                                      f[i].blob_capacity, &bb, &(*jobs)[i]);
    if (st != FPSZ_OK) {
      char msg[sizeof(ctx->err)];
      snprintf(msg, sizeof(msg), "field %d: %s", i, ctx->err);
      memcpy(ctx->err, msg, sizeof(msg));
      return st;
    }
    o += need;
  }
  return FPSZ_OK;
}

}  // namespace

extern "C" {

fpsz_status fpsz_batch_workspace_bytes(int n, const fpsz_field_desc *fields, uint64_t *bytes) {
  if (n < 1 || !fields || !bytes) return FPSZ_E_INVALID_ARG;
  std::vector<Plan> plans(n);
  for (int i = 0; i < n; i++)
    if (make_plan(fields[i].ndim, fields[i].dims, (fpsz_dtype)fields[i].dtype, &plans[i]) != FPSZ_OK)
      return FPSZ_E_INVALID_ARG;
  *bytes = batch_layout(n, plans).total;
  return FPSZ_OK;
}

fpsz_status fpsz_batch_create(fpsz_ctx *ctx, int n, const fpsz_field_desc *fields,
                              void *workspace_dev, uint64_t workspace_bytes, int use_graph,
                              fpsz_batch **out) {
  if (!ctx || !out) return FPSZ_E_INVALID_ARG;
  *out = nullptr;
  ctx->err[0] = 0;
  if (n < 1 || n > 65535 || !fields || !workspace_dev)
    return fail(ctx, FPSZ_E_INVALID_ARG, "need 1..65535 fields and a workspace");
  if ((uintptr_t)workspace_dev % 256) return fail(ctx, FPSZ_E_INVALID_ARG, "workspace must be 256-aligned");
  std::vector<Plan> plans;
  std::vector<CJob> jobs;
  fpsz_status st = prepare_all(ctx, n, fields, (uint8_t *)workspace_dev, workspace_bytes, &plans, &jobs);
  if (st != FPSZ_OK) return st;
  const BatchLayout L = batch_layout(n, plans);

  fpsz_batch *b = new (std::nothrow) fpsz_batch;
  if (!b) return fail(ctx, FPSZ_E_NOMEM, "batch object");
  b->ctx = ctx;
  b->n = n;
  // class order: stable by (dtype, ndim, domain)
  std::vector<int> idx(n);
  for (int i = 0; i < n; i++) idx[i] = i;
  auto key = [&](int i) { return (jobs[i].P.dtype * 4 + jobs[i].P.ndim) * 2 + jobs[i].P.domain; };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return key(a) < key(c); });
  for (int k = 0; k < n; k++) {
    b->jobs.push_back(jobs[idx[k]]);
    b->user.push_back(idx[k]);
    const Plan &P = jobs[idx[k]].P;
    if (b->classes.empty() || key(idx[k]) != key(idx[k - 1])) {
      BatchClass c;
      c.dtype = P.dtype;
      c.ndim = P.ndim;
      c.domain = P.domain;
      c.first = k;
      c.count = 0;
      c.maxP = P;
      b->classes.push_back(c);
    }
    BatchClass &c = b->classes.back();
    c.count++;
    c.maxP.n = std::max(c.maxP.n, P.n);
    c.maxP.n_tiles = std::max(c.maxP.n_tiles, P.n_tiles);
    c.maxP.capacity = std::max(c.maxP.capacity, P.capacity);
    c.maxP.pad_ |= P.pad_;
  }
  for (BatchClass &c : b->classes) c.cfg = default_launch_cfg(c.maxP);

  DeviceGuard g(ctx->device);
  uint8_t *ws = (uint8_t *)workspace_dev;
  b->jobs_dev = (CJob *)(ws + L.off_jobs);
  b->params_dev = (DevParams *)(ws + L.off_params);
  hipError_t e = hipHostMalloc((void **)&b->params_host, (size_t)n * sizeof(DevParams),
                               hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipMemcpy(b->jobs_dev, b->jobs.data(), (size_t)n * sizeof(CJob), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    fpsz_batch_destroy(b);
    return hip_fail(ctx, e, "batch set-up");
  }
  b->use_graph = use_graph != 0;
  if (b->use_graph) {
    st = capture(b);
    if (st != FPSZ_OK) {
      fpsz_batch_destroy(b);
      return st;
    }
  }
  *out = b;
  return FPSZ_OK;
}

void fpsz_batch_destroy(fpsz_batch *b) {
  if (!b) return;
  DeviceGuard g(b->ctx->device);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->params_host) (void)hipHostFree(b->params_host);
  delete b;
}

fpsz_status fpsz_batch_run(fpsz_batch *b, void *stream, uint64_t *blob_bytes, fpsz_info *info,
                           fpsz_status *status) {
  if (!b) return FPSZ_E_INVALID_ARG;
  fpsz_ctx *ctx = b->ctx;
  ctx->err[0] = 0;
  if (!blob_bytes || !status) return fail(ctx, FPSZ_E_INVALID_ARG, "null result arrays");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = b->captured ? hipGraphLaunch(b->exec, s) : enqueue_batch(b, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch");
  fpsz_status first = FPSZ_OK;
  char first_msg[sizeof(ctx->err)] = {0};
  for (int k = 0; k < b->n; k++) {
    const int i = b->user[k];
    const CJob &J = b->jobs[k];
    const DevParams &D = b->params_host[k];
    if (info) fill_compress_info(&info[i], J.P, D);
    blob_bytes[i] = 0;
    status[i] = compress_result(ctx, J.P, D, &blob_bytes[i]);
    if (status[i] != FPSZ_OK && first == FPSZ_OK) {
      first = status[i];
      snprintf(first_msg, sizeof(first_msg), "field %d: %s", i, ctx->err);
    }
  }
  memcpy(ctx->err, first_msg, sizeof(first_msg));
  return first;
}

fpsz_status fpsz_batch_autotune(fpsz_batch *b, void *stream, int reps, double *best_ms) {
  if (!b || reps < 1) return FPSZ_E_INVALID_ARG;
  fpsz_ctx *ctx = b->ctx;
  ctx->err[0] = 0;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ctx, FPSZ_E_DEVICE, "event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, FPSZ_E_DEVICE, "event");
  }
  fpsz_status st = FPSZ_OK;
  // median of `reps` eager runs of the whole batch with the current shapes
  auto time_batch = [&](double *ms) -> bool {
    std::vector<float> t;
    for (int r = 0; r < reps; r++) {
      if (hipEventRecord(e0, s) != hipSuccess || enqueue_batch(b, s) != hipSuccess ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return false;
      float v = 0.f;
      if (hipEventElapsedTime(&v, e0, e1) != hipSuccess) return false;
      t.push_back(v);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return true;
  };
  double best = 0.0;
  if (!time_batch(&best)) st = fail(ctx, FPSZ_E_DEVICE, "autotune timing");
  static const uint32_t kGrid[] = {32, 64, 128, 256, 512, 1024, 2048, 4096};
  static const uint32_t kRange[] = {16, 32, 64, 128, 256, 512, 1024};
  static const uint32_t kCsum[] = {8, 32, 128, 512, 1024};
  for (size_t ci = 0; ci < b->classes.size() && st == FPSZ_OK; ci++) {
    BatchClass &c = b->classes[ci];
    // one parameter at a time, the others held at their best so far
    for (int which = 0; which < 4 && st == FPSZ_OK; which++) {
      const uint32_t *cand = which == 2 ? kRange : which == 3 ? kCsum : kGrid;
      const int nc = which == 2 ? 7 : which == 3 ? 5 : 8;
      uint32_t *field = which == 0 ? &c.cfg.quant_grid : which == 1 ? &c.cfg.encode_grid
                        : which == 2 ? &c.cfg.range_blocks : &c.cfg.csum_blocks;
      const uint32_t limit = which <= 1 ? (uint32_t)c.maxP.n_tiles
                             : which == 2 ? (uint32_t)kRangeBlocks : 1024u;
      uint32_t keep = *field;
      for (int k = 0; k < nc; k++) {
        const uint32_t v = cand[k] < limit ? cand[k] : limit;
        if (v == keep || v == 0) continue;
        *field = v;
        double ms = 0.0;
        if (!time_batch(&ms)) {
          st = fail(ctx, FPSZ_E_DEVICE, "autotune timing");
          break;
        }
        if (ms < best) {
          best = ms;
          keep = v;
        }
      }
      *field = keep;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FPSZ_OK) return st;
  if (best_ms) *best_ms = best;
  if (b->use_graph) return capture(b);
  return FPSZ_OK;
}

fpsz_status fpsz_batch_launch_shape(const fpsz_batch *b, int cls, uint32_t *shape4) {
  if (!b || !shape4 || cls < 0 || cls >= (int)b->classes.size()) return FPSZ_E_INVALID_ARG;
  const LaunchCfg &c = b->classes[cls].cfg;
  shape4[0] = c.range_blocks;
  shape4[1] = c.quant_grid;
  shape4[2] = c.encode_grid;
  shape4[3] = c.csum_blocks;
  return FPSZ_OK;
}

fpsz_status fpsz_batch_class_count(const fpsz_batch *b, int *count) {
  if (!b || !count) return FPSZ_E_INVALID_ARG;
  *count = (int)b->classes.size();
  return FPSZ_OK;
}

fpsz_status fpsz_batch_set_launch_shape(fpsz_batch *b, int cls, const uint32_t *shape4) {
  if (!b || !shape4 || cls < 0 || cls >= (int)b->classes.size()) return FPSZ_E_INVALID_ARG;
  fpsz_ctx *ctx = b->ctx;
  ctx->err[0] = 0;
  BatchClass &c = b->classes[cls];
  const uint64_t lim[4] = {(uint64_t)kRangeBlocks, c.maxP.n_tiles, c.maxP.n_tiles, 1024};
  for (int k = 0; k < 4; k++)
    if (shape4[k] < 1 || shape4[k] > lim[k])
      return fail(ctx, FPSZ_E_INVALID_ARG, "shape entry %d = %u outside 1..%llu", k,
                  (unsigned)shape4[k], (unsigned long long)lim[k]);
  c.cfg.range_blocks = shape4[0];
  c.cfg.quant_grid = shape4[1];
  c.cfg.encode_grid = shape4[2];
  c.cfg.csum_blocks = shape4[3];
  if (b->use_graph) {
    DeviceGuard g(ctx->device);
    return capture(b);
  }
  return FPSZ_OK;
}

fpsz_status fpsz_compress_batch(fpsz_ctx *ctx, int n, const fpsz_field_desc *fields,
                                void *workspace_dev, uint64_t workspace_bytes,
                                uint64_t *blob_bytes, fpsz_info *info, fpsz_status *status,
                                void *stream) {
  fpsz_batch *b = nullptr;
  fpsz_status st = fpsz_batch_create(ctx, n, fields, workspace_dev, workspace_bytes, 0, &b);
  if (st != FPSZ_OK) return st;
  st = fpsz_batch_run(b, stream, blob_bytes, info, status);
  fpsz_batch_destroy(b);
  return st;
}

}  // extern "C"
