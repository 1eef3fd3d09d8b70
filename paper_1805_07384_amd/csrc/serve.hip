// serve.hip -- a request loop for compress / decompress requests that
// arrive over time (the fixed-PSNR workflow after Eq. 7, applied per
// request, with decompression and the PSNR known afterwards, Sec. V).
//
// One worker thread per server owns a private library context, a device
// arena for request workspaces and a few streams (default priority).
// Requests are admitted in arrival order while their HBM footprint (input +
// output + workspace) fits the budget and a result slot is free; requests
// that arrive while others run join the next admission round (continuous
// batching).  The compress requests of one round that share a field class
// go out as one batched launch (one launch per pipeline step over all of
// them); decompress requests first read their 256-byte header
// asynchronously, then launch.  Rounds run on different streams, so their
// work overlaps on the device; a stream takes a new round only when its
// previous one has finished, so under load arrivals accumulate into larger
// rounds.  Nothing is synchronized on the host: the
// worker polls events.  Every request computes exactly what a plain call
// computes, so results are bit-identical alone and in the mix.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "host_common.h"

using namespace fpsz;

namespace {

// First-fit allocator over [0, size) in 256-byte units.
struct Arena {
  std::map<uint64_t, uint64_t> free_;  // offset -> size
  void init(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(uint64_t n, uint64_t *off) {
    n = align256(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const uint64_t o = it->first, rem = it->second - n;
      free_.erase(it);
      if (rem) free_[o + n] = rem;
      *off = o;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = align256(n ? n : 1);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum RState { R_PENDING, R_HEADER, R_RUNNING, R_DONE };

struct SReq {
  uint64_t id = 0;
  fpsz_request r;
  RState st = R_PENDING;
  Plan plan;                 // from the request's shape (both kinds)
  uint64_t ws_bytes = 0, hold = 0, ws_off = 0;
  int slot = -1, stream = 0;
  int64_t group = -1;        // batched compress launch it belongs to
  CJob cj;
  DJob dj;
  fpsz_result res;
};

struct Group {
  uint64_t tab_off = 0, tab_bytes = 0;
  int remaining = 0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct fpsz_server {
  fpsz_ctx *ctx = nullptr;  // private context of the worker
  int device = 0;
  uint64_t budget = 0, held = 0;
  int max_slots = 0;
  uint8_t *arena_dev = nullptr;
  Arena arena;
  uint64_t arena_bytes = 0;
  CJob *tab_dev = nullptr;   // batched job tables
  CJob *tab_host = nullptr;  // pinned staging of the tables (same offsets)
  Arena tab_arena;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
  uint8_t *pinned = nullptr;  // per slot: DevParams, then a 256-byte header
  std::vector<hipEvent_t> slot_ev;
  std::vector<int> free_slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::map<uint64_t, SReq> reqs;
  std::vector<uint64_t> active;
  std::map<int64_t, Group> groups;
  int64_t next_group = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0;
  fpsz_server_stats stats;
};

namespace {

constexpr size_t kSlotBytes = ((sizeof(DevParams) + kHdr + 255) / 256) * 256;

DevParams *slot_params(fpsz_server *S, int slot) {
  return reinterpret_cast<DevParams *>(S->pinned + (size_t)slot * kSlotBytes);
}
uint8_t *slot_header(fpsz_server *S, int slot) {
  return S->pinned + (size_t)slot * kSlotBytes + sizeof(DevParams);
}

void finish(fpsz_server *S, SReq &q, fpsz_status st) {
  q.res.status = st;
  q.res.t_done = now_s(S->t0);
  q.st = R_DONE;
  if (q.slot >= 0) S->free_slots.push_back(q.slot);
  q.slot = -1;
  if (q.ws_bytes && q.hold) S->arena.release(q.ws_off, q.ws_bytes);
  S->held -= q.hold;
  q.hold = 0;
  q.ws_bytes = 0;
  if (q.group >= 0) {
    auto it = S->groups.find(q.group);
    if (it != S->groups.end() && --it->second.remaining == 0) {
      if (it->second.tab_bytes) S->tab_arena.release(it->second.tab_off, it->second.tab_bytes);
      S->groups.erase(it);
    }
  }
  S->stats.completed++;
  if (st != FPSZ_OK) S->stats.failed++;
  S->cv_done.notify_all();
}

// decompress phase 2: header in the slot, launch the decode
void launch_decompress_req(fpsz_server *S, SReq &q) {
  hipStream_t s = S->streams[q.stream];
  const uint8_t *h = slot_header(S, q.slot);
  fpsz_status st = prepare_decompress(S->ctx, h, q.r.src_dev, q.r.src_bytes,
                                      S->arena_dev + q.ws_off, q.ws_bytes, q.r.dst_dev,
                                      q.r.dst_capacity, &q.dj);
  if (st == FPSZ_OK &&
      (q.dj.P.ndim != q.plan.ndim || q.dj.P.dtype != q.plan.dtype || q.dj.P.n != q.plan.n ||
       q.dj.P.nz != q.plan.nz || q.dj.P.ny != q.plan.ny || q.dj.P.nx != q.plan.nx))
    st = fail(S->ctx, FPSZ_E_INVALID_ARG, "blob shape differs from the request");
  if (st != FPSZ_OK) {
    finish(S, q, st);
    return;
  }
  int nd;
  uint64_t dims[3];
  fpsz_dtype dt;
  (void)fpsz_blob_header(h, kHdr, &nd, dims, &dt, &q.res.info);
  Timer off;
  off.on = false;
  hipError_t e = launch_decompress_job(q.dj, s, &off);
  if (e == hipSuccess)
    e = hipMemcpyAsync(slot_params(S, q.slot), q.dj.W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(S->slot_ev[q.slot], s);
  if (e != hipSuccess) {
    finish(S, q, hip_fail(S->ctx, e, "decompress launch"));
    return;
  }
  q.st = R_RUNNING;
}

// launch the compress requests `ids` (same class) on stream si
void launch_compress_group(fpsz_server *S, const std::vector<uint64_t> &ids, int si) {
  hipStream_t s = S->streams[si];
  Timer off;
  off.on = false;
  hipError_t e = hipSuccess;
  // the callers' inputs are complete before anything of the group runs
  for (uint64_t id : ids) {
    const SReq &q = S->reqs[id];
    if (q.r.ready_event && e == hipSuccess)
      e = hipStreamWaitEvent(s, (hipEvent_t)q.r.ready_event, 0);
  }
  Plan maxP = S->reqs[ids[0]].cj.P;
  for (uint64_t id : ids) {
    const Plan &P = S->reqs[id].cj.P;
    maxP.n = std::max(maxP.n, P.n);
    maxP.n_tiles = std::max(maxP.n_tiles, P.n_tiles);
    maxP.capacity = std::max(maxP.capacity, P.capacity);
    maxP.pad_ |= P.pad_;
  }
  const LaunchCfg cfg = default_launch_cfg(maxP);
  uint64_t toff = 0;
  const uint64_t tbytes = ids.size() * sizeof(CJob);
  if (e == hipSuccess && ids.size() > 1 && S->tab_arena.alloc(tbytes, &toff)) {
    // one batched launch per step over the group
    const int64_t g = S->next_group++;
    Group &G = S->groups[g];
    G.tab_off = toff;
    G.tab_bytes = tbytes;
    G.remaining = (int)ids.size();
    CJob *th = reinterpret_cast<CJob *>(reinterpret_cast<uint8_t *>(S->tab_host) + toff);
    CJob *td = reinterpret_cast<CJob *>(reinterpret_cast<uint8_t *>(S->tab_dev) + toff);
    for (size_t k = 0; k < ids.size(); k++) {
      th[k] = S->reqs[ids[k]].cj;
      S->reqs[ids[k]].group = g;
    }
    e = hipMemcpyAsync(td, th, tbytes, hipMemcpyHostToDevice, s);
    CJob none;
    memset(&none, 0, sizeof(none));
    if (e == hipSuccess) e = launch_compress_jobs(none, td, (int)ids.size(), maxP, cfg, s, &off);
    S->stats.batched_launches++;
  } else {
    for (uint64_t id : ids) {
      const CJob &J = S->reqs[id].cj;
      if (e == hipSuccess) e = launch_compress_jobs(J, nullptr, 1, J.P, default_launch_cfg(J.P), s, &off);
    }
  }
  for (uint64_t id : ids) {
    SReq &q = S->reqs[id];
    if (e == hipSuccess)
      e = hipMemcpyAsync(slot_params(S, q.slot), q.cj.W.P, sizeof(DevParams), hipMemcpyDeviceToHost, s);
  }
  for (uint64_t id : ids) {
    SReq &q = S->reqs[id];
    if (e == hipSuccess) e = hipEventRecord(S->slot_ev[q.slot], s);
  }
  for (uint64_t id : ids) {
    SReq &q = S->reqs[id];
    if (e != hipSuccess) finish(S, q, hip_fail(S->ctx, e, "compress launch"));
    else q.st = R_RUNNING;
  }
}

// A stream with no unfinished request of an earlier round, or -1.  At most
// one round is in flight per stream: while every stream is busy, arrivals
// wait and the next round takes all of them (one batched launch per class)
// instead of queueing one launch sequence per request behind the others.
int free_stream(fpsz_server *S) {
  const int ns = (int)S->streams.size();
  std::vector<char> busy(ns, 0);
  for (uint64_t id : S->active) {
    const SReq &q = S->reqs[id];
    if (q.st != R_DONE) busy[q.stream] = 1;
  }
  for (int k = 0; k < ns; k++) {
    const int si = (S->next_stream + k) % ns;
    if (!busy[si]) return si;
  }
  return -1;
}

// admission of pending requests in arrival order; returns true if any
bool admit(fpsz_server *S) {
  if (S->pending.empty()) return false;
  const int si = free_stream(S);
  if (si < 0) return false;
  std::vector<uint64_t> round;
  const double t = now_s(S->t0);
  while (!S->pending.empty() && !S->free_slots.empty()) {
    SReq &q = S->reqs[S->pending.front()];
    if (q.hold > S->budget || q.ws_bytes > S->arena_bytes) {
      S->pending.pop_front();
      q.hold = 0;
      q.ws_bytes = 0;
      finish(S, q, fail(S->ctx, FPSZ_E_CAPACITY, "request exceeds the server's HBM budget"));
      continue;
    }
    if (S->held + q.hold > S->budget) break;
    uint64_t off = 0;
    if (!S->arena.alloc(q.ws_bytes, &off)) break;
    S->pending.pop_front();
    q.ws_off = off;
    S->held += q.hold;
    q.slot = S->free_slots.back();
    S->free_slots.pop_back();
    q.res.t_start = t;
    round.push_back(q.id);
  }
  if (round.empty()) return false;
  S->next_stream = (si + 1) % (int)S->streams.size();
  S->stats.rounds++;
  hipStream_t s = S->streams[si];
  // compress requests grouped by class; decompress requests read headers
  std::map<int, std::vector<uint64_t>> cls;
  for (uint64_t id : round) {
    SReq &q = S->reqs[id];
    q.stream = si;
    S->active.push_back(id);
    if (q.r.kind == FPSZ_REQ_COMPRESS) {
      uint64_t bb = 0;
      fpsz_status st = prepare_compress(S->ctx, q.r.src_dev, q.r.ndim, q.r.dims,
                                        (fpsz_dtype)q.r.dtype, q.r.target_psnr,
                                        (fpsz_domain)q.r.domain, S->arena_dev + q.ws_off,
                                        q.ws_bytes, q.r.dst_dev, q.r.dst_capacity, &bb, &q.cj);
      if (st != FPSZ_OK) {
        q.res.out_bytes = bb;
        finish(S, q, st);
        continue;
      }
      cls[(q.cj.P.dtype * 4 + q.cj.P.ndim) * 2 + q.cj.P.domain].push_back(id);
    } else {
      hipError_t e = hipSuccess;
      if (q.r.ready_event) e = hipStreamWaitEvent(s, (hipEvent_t)q.r.ready_event, 0);
      if (e == hipSuccess)
        e = hipMemcpyAsync(slot_header(S, q.slot), q.r.src_dev, kHdr, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(S->slot_ev[q.slot], s);
      if (e != hipSuccess) {
        finish(S, q, hip_fail(S->ctx, e, "header read"));
        continue;
      }
      q.st = R_HEADER;
    }
  }
  for (auto &kv : cls) launch_compress_group(S, kv.second, si);
  size_t inflight = 0;
  for (uint64_t id : S->active)
    if (S->reqs[id].st != R_DONE) inflight++;
  if (inflight > S->stats.peak_inflight) S->stats.peak_inflight = inflight;
  if (S->held > S->stats.peak_held_bytes) S->stats.peak_held_bytes = S->held;
  return true;
}

// completions; returns true if any request changed state
bool progress(fpsz_server *S) {
  bool any = false;
  std::vector<uint64_t> keep;
  for (uint64_t id : S->active) {
    SReq &q = S->reqs[id];
    if (q.st == R_DONE) continue;
    hipError_t e = hipEventQuery(S->slot_ev[q.slot]);
    if (e == hipErrorNotReady) {
      keep.push_back(id);
      continue;
    }
    any = true;
    if (e != hipSuccess) {
      finish(S, q, hip_fail(S->ctx, e, "request"));
      continue;
    }
    if (q.st == R_HEADER) {
      launch_decompress_req(S, q);
      if (q.st != R_DONE) keep.push_back(id);
      continue;
    }
    const DevParams &D = *slot_params(S, q.slot);
    if (q.r.kind == FPSZ_REQ_COMPRESS) {
      fill_compress_info(&q.res.info, q.cj.P, D);
      uint64_t bb = 0;
      const fpsz_status st = compress_result(S->ctx, q.cj.P, D, &bb);
      q.res.out_bytes = bb;
      finish(S, q, st);
    } else {
      const fpsz_status st = decompress_result(S->ctx, q.dj, D);
      q.res.out_bytes = q.dj.P.n * (q.dj.P.dtype == FPSZ_F32 ? 4 : 8);
      finish(S, q, st);
    }
  }
  S->active.swap(keep);
  return any;
}

void worker_main(fpsz_server *S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool moved = progress(S);
    moved = admit(S) || moved;
    if (S->stop && S->pending.empty() && S->active.empty()) break;
    if (moved) continue;
    if (S->active.empty())
      S->cv_work.wait(lk);  // idle: until a submission or stop
    else
      S->cv_work.wait_for(lk, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

fpsz_status fpsz_server_create(fpsz_ctx *ctx, uint64_t hbm_budget_bytes, uint64_t arena_bytes,
                               int max_inflight, int n_streams, fpsz_server **out) {
  if (!ctx || !out) return FPSZ_E_INVALID_ARG;
  *out = nullptr;
  if (hbm_budget_bytes == 0 || arena_bytes == 0 || max_inflight < 1 || max_inflight > 4096 ||
      n_streams < 1 || n_streams > 16)
    return fail(ctx, FPSZ_E_INVALID_ARG, "bad server limits");
  fpsz_server *S = new (std::nothrow) fpsz_server;
  if (!S) return fail(ctx, FPSZ_E_NOMEM, "server object");
  memset(&S->stats, 0, sizeof(S->stats));
  S->device = ctx->device;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_inflight;
  S->arena_bytes = align256(arena_bytes);
  S->t0 = std::chrono::steady_clock::now();
  fpsz_status st = fpsz_create(ctx->device, &S->ctx);
  if (st != FPSZ_OK) {
    delete S;
    return fail(ctx, st, "server context");
  }
  DeviceGuard g(ctx->device);
  const uint64_t tab_bytes = align256((uint64_t)max_inflight * sizeof(CJob)) * 2;
  hipError_t e = hipMalloc((void **)&S->arena_dev, S->arena_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&S->tab_dev, tab_bytes);
  if (e == hipSuccess) e = hipHostMalloc((void **)&S->tab_host, tab_bytes, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&S->pinned, (size_t)max_inflight * kSlotBytes, hipHostMallocDefault);
  for (int i = 0; i < n_streams && e == hipSuccess; i++) {
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) S->streams.push_back(s);
  }
  for (int i = 0; i < max_inflight && e == hipSuccess; i++) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) {
      S->slot_ev.push_back(ev);
      S->free_slots.push_back(max_inflight - 1 - i);
    }
  }
  if (e != hipSuccess) {
    fpsz_server_destroy(S);
    return hip_fail(ctx, e, "server set-up");
  }
  S->arena.init(S->arena_bytes);
  S->tab_arena.init(tab_bytes);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return FPSZ_OK;
}

fpsz_status fpsz_server_submit(fpsz_server *S, const fpsz_request *req, uint64_t *id) {
  if (!S || !req || !id) return FPSZ_E_INVALID_ARG;
  SReq q;
  memset(&q.res, 0, sizeof(q.res));
  q.r = *req;
  fpsz_status st = FPSZ_OK;
  if (req->kind != FPSZ_REQ_COMPRESS && req->kind != FPSZ_REQ_DECOMPRESS) st = FPSZ_E_INVALID_ARG;
  else if (!req->src_dev || !req->dst_dev) st = FPSZ_E_INVALID_ARG;
  else st = make_plan(req->ndim, req->dims, (fpsz_dtype)req->dtype, &q.plan);
  std::lock_guard<std::mutex> lk(S->mu);
  q.id = S->next_id++;
  q.res.t_submit = now_s(S->t0);
  S->stats.submitted++;
  *id = q.id;
  if (st == FPSZ_OK) {
    const uint64_t esz = req->dtype == FPSZ_F32 ? 4 : 8;
    if (req->kind == FPSZ_REQ_COMPRESS) {
      q.ws_bytes = compress_layout(q.plan).total;
      q.hold = q.plan.n * esz + req->dst_capacity + q.ws_bytes;
    } else {
      q.ws_bytes = decompress_layout(q.plan).total;
      q.hold = req->src_bytes + q.plan.n * esz + q.ws_bytes;
    }
    S->reqs[q.id] = q;
    S->pending.push_back(q.id);
  } else {
    q.st = R_DONE;
    q.res.status = st;
    q.res.t_done = q.res.t_submit;
    S->stats.completed++;
    S->stats.failed++;
    S->reqs[q.id] = q;
  }
  S->cv_work.notify_one();
  return FPSZ_OK;
}

fpsz_status fpsz_server_poll(fpsz_server *S, uint64_t id, int *done, fpsz_result *res) {
  if (!S || !done) return FPSZ_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return FPSZ_E_INVALID_ARG;
  *done = it->second.st == R_DONE;
  if (*done) {
    if (res) *res = it->second.res;
    S->reqs.erase(it);
  }
  return FPSZ_OK;
}

fpsz_status fpsz_server_wait(fpsz_server *S, uint64_t id, fpsz_result *res) {
  if (!S) return FPSZ_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return FPSZ_E_INVALID_ARG;
  S->cv_done.wait(lk, [&] { return S->reqs[id].st == R_DONE; });
  it = S->reqs.find(id);
  if (res) *res = it->second.res;
  S->reqs.erase(it);
  return FPSZ_OK;
}

fpsz_status fpsz_server_get_stats(fpsz_server *S, fpsz_server_stats *out) {
  if (!S || !out) return FPSZ_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->now = now_s(S->t0);
  out->held_bytes = S->held;
  return FPSZ_OK;
}

void fpsz_server_destroy(fpsz_server *S) {
  if (!S) return;
  if (S->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    S->worker.join();  // finishes every submitted request first
  }
  DeviceGuard g(S->device);
  for (hipEvent_t ev : S->slot_ev) (void)hipEventDestroy(ev);
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  if (S->pinned) (void)hipHostFree(S->pinned);
  if (S->tab_host) (void)hipHostFree(S->tab_host);
  if (S->tab_dev) (void)hipFree(S->tab_dev);
  if (S->arena_dev) (void)hipFree(S->arena_dev);
  if (S->ctx) fpsz_destroy(S->ctx);
  delete S;
}

}  // extern "C"
