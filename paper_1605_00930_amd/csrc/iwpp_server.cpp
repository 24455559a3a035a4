// iwpp_server.cpp -- continuous-batching request server (C ABI in iwpp.h).
//
// Requests are reconstructions whose buffers already live on the device.  A
// dispatcher thread admits pending requests in arrival order while the
// device bytes they hold fit in the budget and fewer than `max_inflight`
// requests are unfinished.  The requests admitted together become one
// batched persistent launch (one tile queue for all their tiles) on a free
// stream slot; several slots run at once, so requests that arrive while
// others are on the GPU start as soon as a slot and memory free up, and
// their work overlaps with the launches already running.  Completion is
// reported by a host callback queued behind each launch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "iwpp.h"
#include "iwpp_internal.h"
#include "iwpp_runtime.h"

using namespace iwpp;

namespace {

double now_us() {
  using namespace std::chrono;
  return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() *
         1e-3;
}

struct Request {
  iwpp_image img{};
  const void* init = nullptr;  // optional pristine marker copied in first
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  uint64_t ticket = 0;
  size_t bytes = 0;
  int64_t tiles = 0;
  double t_submit = 0, t_done = 0;
  int status = IWPP_OK;
  bool done = false;
};

struct Slot;

}  // namespace

struct iwpp_server {
  int dtype = 0, conn = 8, device = 0;
  size_t budget = 0, in_use = 0;
  int max_inflight = 0, inflight = 0, busy_slots = 0;
  Resolved rp{};
  Variant v{};
  std::vector<Slot*> slots;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> all;
  std::mutex mu;
  std::condition_variable cv_dispatch, cv_done;
  std::thread dispatcher;
  bool stop = false;
  uint64_t next_ticket = 1;
  int launch_error = IWPP_OK;
  std::vector<hipEvent_t> events;  // free events for the requests' ready marks
  int64_t slot_tiles = 0;          // tiles each slot's workspace holds (allocated at create)
};

namespace {

struct Slot {
  iwpp_server* srv = nullptr;
  hipStream_t st = nullptr;
  Buffers buf;
  DevImage* staging = nullptr;  // pinned descriptor staging
  int staging_cap = 0;
  std::vector<Request*> reqs;
  bool busy = false;
};

size_t elem_size(int dtype) { return dtype == IWPP_U8 ? 1 : 4; }

int64_t request_tiles(const iwpp_image& im, int tile_h) {
  return ((im.H + tile_h - 1) / tile_h) * ((im.W + kTileW - 1) / kTileW);
}

// Library workspace per tile of a launch: state word, first-visit flag, image
// index, ring slot, packed side columns of I and J.
size_t tile_bytes(int dtype, int tile_h) {
  return 4 + 1 + 4 + 4 + (size_t)2 * 2 * tile_h * elem_size(dtype);
}

// Device bytes a request holds: its marker and mask (the caller's) and its
// tiles' share of the slot workspace (allocated once, at create).
size_t request_bytes(const iwpp_image& im, int dtype, int tile_h) {
  const int64_t ld = im.ld ? im.ld : im.W;
  return (size_t)(2 * ((im.H - 1) * ld + im.W)) * elem_size(dtype) +
         (size_t)request_tiles(im, tile_h) * tile_bytes(dtype, tile_h);
}

// Host callback behind a launch: record completion (no HIP calls here).
void on_done(void* arg) {
  Slot* s = (Slot*)arg;
  iwpp_server* srv = s->srv;
  const double t = now_us();
  std::lock_guard<std::mutex> g(srv->mu);
  const int status = status_of(*s->buf.host_ctl, 0, false);
  for (Request* r : s->reqs) {
    r->status = status;
    r->t_done = t;
    r->done = true;
    srv->in_use -= r->bytes;
    srv->inflight--;
  }
  s->reqs.clear();
  s->busy = false;
  srv->busy_slots--;
  srv->cv_done.notify_all();
  srv->cv_dispatch.notify_all();
}

// Queue one batched launch of `batch` on slot s (the server lock is not held).
int launch_batch(iwpp_server* srv, Slot* s, std::vector<Request*>& batch) {
  const int n = (int)batch.size();
  if (n > s->staging_cap) {
    if (s->staging) (void)hipHostFree(s->staging);
    s->staging = nullptr;
    const int cap = n < 64 ? 64 : n;
    if (hipHostMalloc(&s->staging, cap * sizeof(DevImage), hipHostMallocDefault) != hipSuccess)
      return IWPP_E_NOMEM;
    s->staging_cap = cap;
  }
  int64_t base = 0;
  for (int k = 0; k < n; ++k) {
    s->staging[k] = make_dev_image(batch[k]->img, srv->rp.tile_h, base);
    base += (int64_t)s->staging[k].tiles_y * s->staging[k].tiles_x;
  }
  int grid = 0;
  KParams kp{};
  int rc = plan_queues(srv->v, srv->rp, base, n, s->staging[0], &grid, &kp);
  if (rc) return rc;
  // The workspace was sized at create for the most tiles the budget admits
  // at once (admission keeps a batch within it), so nothing is allocated or
  // freed here.  Only the queue rings of a request wider than about 65,000
  // pixels could outgrow it; ensure() then grows them (and waits for the
  // slot's stream).
  rc = s->buf.ensure(base, kp.qcap * (uint32_t)kp.nq, n, false);
  if (!rc) rc = s->buf.ensure_cols_for(srv->v.dtype, srv->v.tile_h, base);
  if (rc) return rc;
  // the requests' buffers are ready once the work queued before submit on
  // the callers' streams has run
  for (Request* r : batch)
    if (r->ready && hipStreamWaitEvent(s->st, r->ready, 0) != hipSuccess) return IWPP_E_HIP;
  if (hipMemcpyAsync(s->buf.descs, s->staging, n * sizeof(DevImage), hipMemcpyHostToDevice,
                     s->st) != hipSuccess)
    return IWPP_E_HIP;
  for (Request* r : batch) {
    if (!r->init) continue;
    const int64_t ld = r->img.ld ? r->img.ld : r->img.W;
    const size_t es = elem_size(srv->dtype);
    if (hipMemcpy2DAsync(r->img.marker, ld * es, r->init, ld * es, r->img.W * es, r->img.H,
                         hipMemcpyDeviceToDevice, s->st) != hipSuccess)
      return IWPP_E_HIP;
  }
  int64_t launches = 0;
  rc = enqueue(s->buf, srv->v, srv->rp, s->staging[0], s->buf.descs, n, base, s->st, &launches);
  if (rc) return rc;
  if (hipLaunchHostFunc(s->st, on_done, s) != hipSuccess) return IWPP_E_HIP;
  return IWPP_OK;
}

void dispatcher_main(iwpp_server* srv) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    if (srv->stop && srv->pending.empty()) break;
    Slot* free_slot = nullptr;
    for (Slot* s : srv->slots)
      if (!s->busy) {
        free_slot = s;
        break;
      }
    std::vector<Request*> batch;
    if (free_slot) {
      // continuous batching: everything that has arrived and fits goes now
      int64_t tiles = 0;
      while (!srv->pending.empty() && srv->inflight < srv->max_inflight) {
        Request* r = srv->pending.front();
        if (srv->in_use + r->bytes > srv->budget) break;  // wait for memory (FIFO order)
        if (tiles + r->tiles > srv->slot_tiles) break;    // the rest goes to the next launch
        srv->pending.pop_front();
        srv->in_use += r->bytes;
        srv->inflight++;
        tiles += r->tiles;
        batch.push_back(r);
      }
    }
    if (batch.empty()) {
      srv->cv_dispatch.wait(lk);
      continue;
    }
    free_slot->busy = true;
    free_slot->reqs = batch;
    srv->busy_slots++;
    lk.unlock();
    const int rc = launch_batch(srv, free_slot, batch);
    lk.lock();
    if (rc != IWPP_OK) {
      // the launch never started: fail its requests
      srv->launch_error = rc;
      const double t = now_us();
      for (Request* r : free_slot->reqs) {
        r->status = rc;
        r->t_done = t;
        r->done = true;
        srv->in_use -= r->bytes;
        srv->inflight--;
      }
      free_slot->reqs.clear();
      free_slot->busy = false;
      srv->busy_slots--;
      srv->cv_done.notify_all();
    }
  }
}

}  // namespace

extern "C" {

int iwpp_server_create(size_t budget_bytes, int dtype, int conn, int streams, int max_inflight,
                       iwpp_server** out) {
  if (!out) return IWPP_E_ARG;
  *out = nullptr;
  int rc = check_common(dtype, conn, 0);
  if (rc) return rc;
  if (budget_bytes == 0 || streams < 1 || streams > 16 || max_inflight < 1) return IWPP_E_ARG;
  iwpp_server* srv = new iwpp_server();
  srv->dtype = dtype;
  srv->conn = conn;
  srv->budget = budget_bytes;
  srv->max_inflight = max_inflight;
  srv->rp = resolve_params(nullptr, dtype, conn, 4096, 4096);
  srv->rp.mode = 0;
  srv->v = Variant{dtype, conn, srv->rp.tile_h};
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return IWPP_E_HIP;
  }
  // launches share the device: each gets its slice of the resident workgroups
  int full = 0;
  rc = device_grid(srv->v, int64_t(1) << 40, 0, &full);
  if (rc) {
    delete srv;
    return rc;
  }
  srv->rp.grid = full / streams > 8 ? full / streams : 8;
  for (int k = 0; k < streams; ++k) {
    Slot* s = new Slot();
    s->srv = srv;
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      for (Slot* o : srv->slots) {
        (void)hipStreamDestroy(o->st);
        delete o;
      }
      delete srv;
      return IWPP_E_HIP;
    }
    s->buf.stream_owner = s->st;
    srv->slots.push_back(s);
  }
  // Each slot's workspace holds the most tiles the budget admits at once
  // (requests of whole tiles: marker and mask bytes plus workspace per
  // tile), allocated now so that no allocation or free (which would wait for
  // the device) falls on the dispatch path.
  const size_t full_tile = (size_t)2 * srv->rp.tile_h * kTileW * elem_size(dtype) +
                           tile_bytes(dtype, srv->rp.tile_h);
  srv->slot_tiles = (int64_t)(budget_bytes / full_tile);
  if (srv->slot_tiles < 1024) srv->slot_tiles = 1024;
  const int64_t ring = srv->slot_tiles + (int64_t)kMaxQueues * (srv->rp.grid + 64 + 4096);
  for (Slot* s : srv->slots) {
    if (ring >= (int64_t(1) << 31)) rc = IWPP_E_ARG;
    if (!rc) rc = s->buf.ensure(srv->slot_tiles, (uint32_t)ring, max_inflight, false);
    if (!rc) rc = s->buf.ensure_cols_for(dtype, srv->rp.tile_h, srv->slot_tiles);
    if (!rc && hipHostMalloc(&s->staging, max_inflight * sizeof(DevImage), hipHostMallocDefault) !=
                   hipSuccess)
      rc = IWPP_E_NOMEM;
    if (!rc) s->staging_cap = max_inflight;
  }
  if (rc) {
    for (Slot* o : srv->slots) {
      o->buf.release();
      if (o->staging) (void)hipHostFree(o->staging);
      (void)hipStreamDestroy(o->st);
      delete o;
    }
    delete srv;
    return rc;
  }
  srv->dispatcher = std::thread(dispatcher_main, srv);
  *out = srv;
  return IWPP_OK;
}

int iwpp_server_submit(iwpp_server* srv, const iwpp_image* img, const void* marker_init,
                       iwpp_stream_t stream, uint64_t* ticket) {
  if (!srv || !ticket) return IWPP_E_ARG;
  int rc = check_image(img, srv->dtype);
  if (rc) return rc;
  Request* r = new Request();
  r->img = *img;
  r->init = marker_init;
  r->bytes = request_bytes(*img, srv->dtype, srv->rp.tile_h);
  r->tiles = request_tiles(*img, srv->rp.tile_h);
  if (r->bytes > srv->budget || r->tiles > srv->slot_tiles) {
    delete r;
    return IWPP_E_BUDGET;
  }
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (!srv->events.empty()) {
      r->ready = srv->events.back();
      srv->events.pop_back();
    }
  }
  if (!r->ready && hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) {
    delete r;
    return IWPP_E_HIP;
  }
  // the request's work waits for what the caller queued on `stream` so far
  if (hipEventRecord(r->ready, (hipStream_t)stream) != hipSuccess) {
    (void)hipEventDestroy(r->ready);
    delete r;
    return IWPP_E_HIP;
  }
  r->t_submit = now_us();
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->stop) {
    srv->events.push_back(r->ready);
    delete r;
    return IWPP_E_ARG;
  }
  r->ticket = srv->next_ticket++;
  srv->all[r->ticket] = r;
  srv->pending.push_back(r);
  *ticket = r->ticket;
  srv->cv_dispatch.notify_all();
  return IWPP_OK;
}

int iwpp_server_wait(iwpp_server* srv, uint64_t ticket, int64_t timeout_us, double* latency_us) {
  if (!srv) return IWPP_E_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return IWPP_E_ARG;
  Request* r = it->second;
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, [&] { return r->done; });
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                    [&] { return r->done; })) {
    return IWPP_E_TIMEOUT;
  }
  const int status = r->status;
  if (latency_us) *latency_us = r->t_done - r->t_submit;
  srv->all.erase(it);
  if (r->ready) srv->events.push_back(r->ready);  // the launch that waited on it is over
  delete r;
  return status;
}

int iwpp_server_destroy(iwpp_server* srv) {
  if (!srv) return IWPP_E_ARG;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv_dispatch.notify_all();
  }
  srv->dispatcher.join();  // the dispatcher leaves once nothing is pending
  for (Slot* s : srv->slots) (void)hipStreamSynchronize(s->st);
  {
    // all callbacks have run once every stream is idle
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->busy_slots == 0; });
  }
  for (Slot* s : srv->slots) {
    s->buf.release();
    if (s->staging) (void)hipHostFree(s->staging);
    (void)hipStreamDestroy(s->st);
    delete s;
  }
  for (auto& kv : srv->all) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  for (hipEvent_t e : srv->events) (void)hipEventDestroy(e);
  delete srv;
  return IWPP_OK;
}

}  // extern "C"
