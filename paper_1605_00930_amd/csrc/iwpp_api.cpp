// iwpp_api.cpp -- host runtime behind the C ABI in include/iwpp.h:
// argument checks, per-(device, stream) workspaces, the persistent and
// host-driven-round launch sequences, batch plans with HIP-graph replay and
// the autotuner.  All GPU work is done by the kernels in iwpp_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "iwpp.h"
#include "iwpp_internal.h"
#include "iwpp_runtime.h"

using namespace iwpp;

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return IWPP_E_HIP;
}

#define HIP_TRY(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

std::mutex g_mu;  // guards the workspace map, tuned table and device caches

// ------------------------------------------------------------------ params

std::map<std::tuple<int, int, int>, iwpp_params> g_tuned;  // (dtype, conn, log2 px)
bool g_tuned_loaded = false;

int size_class(int64_t H, int64_t W) {
  double px = (double)H * (double)W;
  return px <= 1.0 ? 0 : (int)std::floor(std::log2(px));
}

void load_tune_cache_locked() {
  if (g_tuned_loaded) return;
  g_tuned_loaded = true;
  const char* path = std::getenv("IWPP_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  // one JSON object per line: {"dtype":0,"conn":8,"cls":24,"tile_h":64,"sweeps":2,"mode":0,
  // "seed_queue":32,"queue_waves":16} (the last two may be absent)
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    int dt, cn, cls, th, sw, md, sq = 0, qw = 0;
    const int got = std::sscanf(line,
                                " {\"dtype\":%d,\"conn\":%d,\"cls\":%d,\"tile_h\":%d,\"sweeps\":%d,"
                                "\"mode\":%d,\"seed_queue\":%d,\"queue_waves\":%d",
                                &dt, &cn, &cls, &th, &sw, &md, &sq, &qw);
    if (got == 6 || got == 8) {
      iwpp_params p{};
      p.tile_h = th;
      p.sweeps = sw;
      p.mode = md;
      p.seed_queue = sq;
      p.queue_waves = qw;
      g_tuned[{dt, cn, cls}] = p;
    }
  }
  std::fclose(f);
}

void save_tune_cache_locked() {
  const char* path = std::getenv("IWPP_TUNE_CACHE");
  if (!path || !*path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto& kv : g_tuned) {
    std::fprintf(f,
                 "{\"dtype\":%d,\"conn\":%d,\"cls\":%d,\"tile_h\":%d,\"sweeps\":%d,\"mode\":%d,"
                 "\"seed_queue\":%d,\"queue_waves\":%d}\n",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                 kv.second.tile_h, kv.second.sweeps, kv.second.mode, kv.second.seed_queue,
                 kv.second.queue_waves);
  }
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

}  // namespace

namespace iwpp {

int default_tile_h(int dtype) { return dtype == IWPP_U8 ? 64 : 32; }

// Resolve user params (NULL / zero fields) against tuned and default values
// (with `tuned` false the autotuner's table is not consulted: the defaults
// and the user's values only).
Resolved resolve_params(const iwpp_params* user, int dtype, int conn, int64_t H, int64_t W,
                        bool tuned) {
  Resolved r{};
  iwpp_params base{};
  base.tile_h = default_tile_h(dtype);
  // uint8 (fill-holes): a round of passes is cheap next to a scan and queue
  // waves over a winding front, so a tile gets up to 16 rounds first
  base.sweeps = dtype == IWPP_U8 ? 16 : 1;
  base.mode = 0;
  // uint8: fill-holes fronts wind through whole tiles, so re-visits go
  // straight to rounds of passes; int32 (h-dome): short fronts, few seeds
  base.seed_queue = dtype == IWPP_U8 ? -1 : 8;
  base.queue_waves = 4;
  // uint8 (fill-holes): fronts travel in from the frame, so the second group
  // of first visits should start beside finished tiles; int32 (h-domes):
  // fronts stay local, and the diagonal groups first leave half the tiles
  // with every edge neighbour finished
  base.first_pass = dtype == IWPP_U8 ? 1 : 2;
  if (tuned) {
    std::lock_guard<std::mutex> g(g_mu);
    load_tune_cache_locked();
    auto it = g_tuned.find({dtype, conn, size_class(H, W)});
    if (it != g_tuned.end()) {
      if (it->second.tile_h) base.tile_h = it->second.tile_h;
      if (it->second.sweeps) base.sweeps = it->second.sweeps < 0 ? 0 : it->second.sweeps;
      base.mode = it->second.mode;
      if (it->second.seed_queue) base.seed_queue = it->second.seed_queue;
      if (it->second.queue_waves) base.queue_waves = it->second.queue_waves;
    }
  }
  r.tile_h = base.tile_h;
  r.sweeps = base.sweeps;
  r.mode = base.mode;
  r.grid = 0;
  r.max_visits = 0;
  r.order_seed = 0;
  r.spin_limit = 1u << 24;
  r.timing = 0;
  r.seed_queue_max = base.seed_queue < 0 ? 0 : base.seed_queue;
  r.bands = 16;
  r.first_pass = base.first_pass;
  r.queue_waves = base.queue_waves < 0 ? UINT32_MAX : (uint32_t)base.queue_waves;
  if (user) {
    r.timing = user->timing;
    if (user->seed_queue) r.seed_queue_max = user->seed_queue < 0 ? 0 : user->seed_queue;
    if (user->queue_waves)
      r.queue_waves = user->queue_waves < 0 ? UINT32_MAX : (uint32_t)user->queue_waves;
    if (user->bands) r.bands = user->bands;
    if (user->first_pass) r.first_pass = user->first_pass;
    if (user->tile_h) r.tile_h = user->tile_h;
    if (user->sweeps) r.sweeps = user->sweeps < 0 ? 0 : user->sweeps;
    if (user->mode) r.mode = user->mode;
    r.grid = user->grid;
    r.max_visits = user->max_tile_visits;
    r.order_seed = user->order_seed;
    if (user->spin_limit) r.spin_limit = user->spin_limit;
  }
  return r;
}

int check_params(const iwpp_params* p) {
  if (!p) return IWPP_OK;
  if (p->tile_h != 0 && p->tile_h != 32 && p->tile_h != 64 && p->tile_h != 128)
    return IWPP_E_ARG;
  if (p->sweeps < -1 || p->sweeps > 64) return IWPP_E_ARG;
  if (p->mode < 0 || p->mode > 2) return IWPP_E_ARG;
  if (p->bands < 0 || p->bands > 4096) return IWPP_E_ARG;
  if (p->first_pass < 0 || p->first_pass > 2) return IWPP_E_ARG;
  if (p->grid < 0 || p->max_tile_visits < 0) return IWPP_E_ARG;
  return IWPP_OK;
}

int check_image(const iwpp_image* im, int dtype) {
  if (!im || !im->marker || !im->mask) return IWPP_E_ARG;
  if (im->H < 1 || im->W < 1) return IWPP_E_ARG;
  if (im->ld != 0 && im->ld < im->W) return IWPP_E_ARG;
  const int64_t ld = im->ld ? im->ld : im->W;
  if (im->H > (int64_t(1) << 31) || im->W > (int64_t(1) << 31)) return IWPP_E_ARG;
  const int64_t es = dtype == IWPP_U8 ? 1 : 4;
  const uintptr_t m0 = (uintptr_t)im->marker, k0 = (uintptr_t)im->mask;
  const uintptr_t bytes = (uintptr_t)(((im->H - 1) * ld + im->W) * es);
  if (m0 < k0 + bytes && k0 < m0 + bytes) return IWPP_E_ARG;  // overlap
  if (dtype == IWPP_I32 && ((m0 | k0) & 3u)) return IWPP_E_ARG;
  return IWPP_OK;
}

uint32_t flip_of(uint32_t flags) { return (flags & IWPP_FLAG_EROSION) ? ~0u : 0u; }

int check_common(int dtype, int conn, uint32_t flags) {
  if (dtype != IWPP_U8 && dtype != IWPP_I32) return IWPP_E_ARG;
  if (conn != 4 && conn != 8) return IWPP_E_ARG;
  if (flags & ~(IWPP_FLAG_CLAMP_MARKER | IWPP_FLAG_EROSION)) return IWPP_E_ARG;
  return IWPP_OK;
}

DevImage make_dev_image(const iwpp_image& im, int tile_h, int64_t tile_base) {
  DevImage d{};
  d.J = im.marker;
  d.I = im.mask;
  d.H = im.H;
  d.W = im.W;
  d.ld = im.ld ? im.ld : im.W;
  d.tiles_y = (int32_t)((im.H + tile_h - 1) / tile_h);
  d.tiles_x = (int32_t)((im.W + kTileW - 1) / kTileW);
  d.tile_base = tile_base;
  return d;
}

void order_for(uint32_t seed, int64_t ntiles, uint32_t* mul, uint32_t* add) {
  *mul = 1;
  *add = 0;
  if (!seed || ntiles <= 1) return;
  static const uint32_t primes[] = {1000003u, 999983u, 7919u, 104729u, 15485863u, 2147483647u};
  for (uint32_t p : primes) {
    uint64_t a = p % (uint64_t)ntiles, b = (uint64_t)ntiles;
    while (b) {
      uint64_t t = a % b;
      a = b;
      b = t;
    }
    if (a == 1 && p % (uint64_t)ntiles != 0) {
      *mul = (uint32_t)(p % (uint64_t)ntiles);
      break;
    }
  }
  *add = (uint32_t)(((uint64_t)seed * 2654435761u) % (uint64_t)ntiles);
}

// Queue chunking: consecutive tile ids form chunks dealt round-robin to the
// per-XCD queues.  A single image uses bands of whole tile rows (up to four
// rows, at least four bands per queue when the image is tall enough); a
// batch uses short runs so that every queue gets a share of every image.
int64_t queue_chunk(int64_t ntiles, int nq, int nimg, int64_t tiles_x, int64_t tiles_y) {
  if (nimg == 1) {
    int64_t bh = tiles_y / (4 * (int64_t)nq);
    if (bh < 1) bh = 1;
    if (bh > 4) bh = 4;
    return bh * tiles_x;
  }
  int64_t c = ntiles / (8 * (int64_t)nq);
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  return c;
}

int device_grid(const Variant& v, int64_t ntiles, int want, int* grid) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  static std::map<std::tuple<int, int, int, int>, int> cache;
  int per_cu = 0, cus = 0;
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto key = std::make_tuple(dev, v.dtype, v.conn, v.tile_h);
    auto it = cache.find(key);
    if (it != cache.end()) {
      per_cu = it->second;
    } else {
      per_cu = persistent_blocks_per_cu(v);
      cache[key] = per_cu;
    }
  }
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (per_cu < 1) per_cu = 1;
  int64_t g = (int64_t)per_cu * cus;
  if (want > 0 && want < g) g = want;  // never more than can be resident
  if (g > ntiles) g = ntiles;
  if (g < 1) g = 1;
  *grid = (int)g;
  return IWPP_OK;
}

// ------------------------------------------------------------ device buffers

int Buffers::ensure(int64_t ntiles, uint32_t qcap, int nimg, bool rounds) {
  if (!ctl) {
    HIP_TRY(hipMalloc(&ctl, sizeof(DevCtl)));
    HIP_TRY(hipHostMalloc(&host_ctl, sizeof(DevCtl), hipHostMallocDefault));
    std::memset(host_ctl, 0, sizeof(DevCtl));
  }
  if (ntiles > tiles_cap) {
    (void)hipStreamSynchronize(stream_owner);
    (void)hipFree(state);
    (void)hipFree(visited);
    (void)hipFree(tile_img);
    (void)hipFree(act[0]);
    (void)hipFree(act[1]);
    state = nullptr;
    visited = nullptr;
    tile_img = nullptr;
    act[0] = act[1] = nullptr;
    int64_t cap = std::max<int64_t>(ntiles, 1024);
    HIP_TRY(hipMalloc(&state, cap * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&visited, cap));
    HIP_TRY(hipMalloc(&tile_img, cap * sizeof(int32_t)));
    tiles_cap = cap;
    act_cap = 0;
  }
  if (rounds && act_cap < ntiles) {
    (void)hipFree(act[0]);
    (void)hipFree(act[1]);
    HIP_TRY(hipMalloc(&act[0], tiles_cap));
    HIP_TRY(hipMalloc(&act[1], tiles_cap));
    HIP_TRY(hipMemset(act[0], 0, tiles_cap));
    HIP_TRY(hipMemset(act[1], 0, tiles_cap));
    act_cap = tiles_cap;
  }
  if (qcap > qcap_cap) {
    (void)hipStreamSynchronize(stream_owner);
    (void)hipFree(queue);
    queue = nullptr;
    uint32_t cap = std::max<uint32_t>(qcap, 4096u);
    HIP_TRY(hipMalloc(&queue, (size_t)cap * sizeof(int)));
    qcap_cap = cap;
  }
  if (nimg > descs_cap) {
    (void)hipStreamSynchronize(stream_owner);
    (void)hipFree(descs);
    descs = nullptr;
    int cap = std::max(nimg, 16);
    HIP_TRY(hipMalloc(&descs, (size_t)cap * sizeof(DevImage)));
    descs_cap = cap;
  }
  return IWPP_OK;
}

int Buffers::ensure_cols(int64_t bytes) {
  if (bytes <= cols_cap) return IWPP_OK;
  (void)hipStreamSynchronize(stream_owner);
  (void)hipFree(cols);
  cols = nullptr;
  cols_cap = 0;
  HIP_TRY(hipMalloc(&cols, (size_t)bytes));
  cols_cap = bytes;
  return IWPP_OK;
}

// Packed side columns of a persistent reconstruction launch, kept in the
// workspace.  Nothing fills them up front: a tile writes its own on its first
// visit, and a neighbour reads them only once that visit is complete.
static int setup_cols(Buffers& b, const Variant& v, int64_t ntiles, KParams& kp) {
  if (v.dtype == kDtypeEdt) return IWPP_OK;
  const int64_t esz = v.dtype == IWPP_U8 ? 1 : 4;
  const int64_t n = ntiles * 2 * v.tile_h;
  const int rc = b.ensure_cols_for(v.dtype, v.tile_h, ntiles);
  if (rc) return rc;
  kp.colI = b.cols;
  kp.colJ = (char*)b.cols + n * esz;
  return IWPP_OK;
}

int Buffers::ensure_bands(int64_t ntiles) {
  if (ntiles <= band_cap) return IWPP_OK;
  (void)hipStreamSynchronize(stream_owner);
  (void)hipFree(dclass);
  (void)hipFree(listed);
  (void)hipFree(list[0]);
  (void)hipFree(list[1]);
  dclass = nullptr;
  listed = nullptr;
  list[0] = list[1] = nullptr;
  const int64_t cap = std::max<int64_t>(ntiles, 1024);
  HIP_TRY(hipMalloc(&dclass, cap * sizeof(int)));
  HIP_TRY(hipMalloc(&listed, cap * sizeof(uint32_t)));
  HIP_TRY(hipMalloc(&list[0], cap * sizeof(int)));
  HIP_TRY(hipMalloc(&list[1], cap * sizeof(int)));
  if (!minmax) HIP_TRY(hipMalloc(&minmax, 2 * sizeof(int)));
  band_cap = cap;
  return IWPP_OK;
}
void Buffers::release() {
  (void)hipFree(dclass);
  (void)hipFree(listed);
  (void)hipFree(list[0]);
  (void)hipFree(list[1]);
  (void)hipFree(minmax);
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
  (void)hipFree(ctl);
  (void)hipHostFree(host_ctl);
  (void)hipFree(queue);
  (void)hipFree(state);
  (void)hipFree(visited);
  (void)hipFree(tile_img);
  (void)hipFree(cols);
  (void)hipFree(act[0]);
  (void)hipFree(act[1]);
  (void)hipFree(descs);
  *this = Buffers{};
}

// Grid, queue count, chunk and ring capacity of a persistent launch.
int plan_queues(const Variant& v, const Resolved& rp, int64_t ntiles, int nimg,
                const DevImage& one, int* grid, KParams* kp) {
  int rc = device_grid(v, ntiles, rp.grid, grid);
  if (rc) return rc;
  return plan_queues_for_grid(*grid, ntiles, nimg, one, kp);
}

// Queue count, chunk and ring capacity of a persistent launch of `grid`
// workgroups.
int plan_queues_for_grid(int grid, int64_t ntiles, int nimg, const DevImage& one, KParams* kp) {
  kp->nq = grid < kMaxQueues ? grid : kMaxQueues;
  kp->chunk = (int32_t)queue_chunk(ntiles, kp->nq, nimg, one.tiles_x, one.tiles_y);
  const int64_t nchunks = (ntiles + kp->chunk - 1) / kp->chunk;
  const int64_t per_q = (nchunks + kp->nq - 1) / kp->nq * kp->chunk;
  const int64_t qcap = per_q + grid + 64;
  if (qcap * kp->nq >= (int64_t(1) << 31)) return IWPP_E_ARG;
  kp->qcap = (uint32_t)qcap;
  return IWPP_OK;
}

// Enqueue one reconstruction of `nimg` images (descriptors either `one` or a
// device array `d_imgs`) on `st`, using buffers `b`.  The control block is
// copied to b.host_ctl at the end (stream-ordered).
// Gray-level bands (mode 2): a sequence of persistent launches over
// decreasing classes of values (the priority ordering of "Uso de Diferentes
// Estruturas de Dados", by bands of gray levels).  A launch queues only the
// activations whose class is at or above its band and lists the other tiles
// for a later launch; the next launch starts from that list at the highest
// class deferred.  Classes only decrease, so the sequence ends.
int enqueue_bands(Buffers& b, const Variant& v, const Resolved& rp, const DevImage& one,
                  const DevImage* d_imgs, int nimg, int64_t ntiles, hipStream_t st, KParams kp,
                  int64_t* launches) {
  if (nimg != 1 || d_imgs) return IWPP_E_UNSUPPORTED;
  int grid = 0;
  int rc = plan_queues(v, rp, ntiles, nimg, one, &grid, &kp);
  if (rc) return rc;
  rc = b.ensure(ntiles, kp.qcap * (uint32_t)kp.nq, nimg, false);
  if (!rc) rc = b.ensure_bands(ntiles);
  if (!rc) rc = setup_cols(b, v, ntiles, kp);
  if (rc) return rc;
  order_for(rp.order_seed, ntiles, &kp.order_mul, &kp.order_add);
  // value range of the marker, in the tile order
  int* mm = (int*)b.host_ctl;  // the pinned control copy serves as staging
  mm[0] = INT_MAX;
  mm[1] = INT_MIN;
  HIP_TRY(hipMemcpyAsync(b.minmax, mm, 2 * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_minmax(v.dtype, one.J, one.H, one.W, one.ld, rp.flip, b.minmax, st));
  HIP_TRY(hipMemcpyAsync(mm, b.minmax, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t vmin = mm[0], range = (int64_t)mm[1] - mm[0];
  const int nb = rp.bands > 0 ? rp.bands : 16;
  uint32_t shift = 0;
  while ((range >> shift) >= nb) ++shift;
  kp.band_base = (int32_t)vmin;
  kp.band_shift = shift;
  kp.band = (int32_t)(range >> shift);  // the top class: the first launch visits every tile
  kp.dclass = b.dclass;
  kp.listed = b.listed;
  kp.list_mode = 0;
  kp.list_len = 0;
  kp.list_in = nullptr;
  kp.list_out = b.list[0];
  DevCtl sum{};
  int status = 0;
  int64_t nl = 0;
  b.timed = false;
  b.rounds_ms = 0;
  if (rp.timing) {
    if (!b.ev[0]) HIP_TRY(hipEventCreate(&b.ev[0]));
    if (!b.ev[1]) HIP_TRY(hipEventCreate(&b.ev[1]));
  }
  for (int cur = 0;;) {
    HIP_TRY(launch_init(kp, b.ctl, b.queue, b.state, b.visited, nullptr, st));
    if (kp.list_mode) HIP_TRY(launch_list_mark(kp, b.state, st));
    if (rp.timing) HIP_TRY(hipEventRecord(b.ev[0], st));
    HIP_TRY(launch_persistent(v, one, d_imgs, kp, b.ctl, b.queue, b.state, b.visited, grid, st));
    if (rp.timing) HIP_TRY(hipEventRecord(b.ev[1], st));
    nl += kp.list_mode ? 3 : 2;
    HIP_TRY(hipMemcpyAsync(b.host_ctl, b.ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (rp.timing) {
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, b.ev[0], b.ev[1]));
      b.rounds_ms += ms;
    }
    const DevCtl& c = *b.host_ctl;
    sum.visits += c.visits;
    sum.sweeps += c.sweeps;
    sum.pushes += c.pushes;
    sum.overflows += c.overflows;
    sum.reproc += c.reproc;
    sum.requeued += c.requeued;
    sum.qiters += c.qiters;
    sum.t_idle += c.t_idle;
    sum.t_load += c.t_load;
    sum.t_solve += c.t_solve;
    sum.t_store += c.t_store;
    sum.t_sync += c.t_sync;
    status |= (int)c.status.v;
    const uint32_t next = c.next_len.v;
    const int maxd = (int)c.max_deferred.v;
    if ((status & (ST_INTERNAL | ST_INCOMPLETE | ST_ABORT)) || next == 0 || maxd < 0) break;
    // next launch: the list just written, at the highest class deferred
    kp.band = maxd;
    kp.list_mode = 1;
    kp.list_in = b.list[cur];
    kp.list_len = next;
    cur ^= 1;
    kp.list_out = b.list[cur];
  }
  // the totals of all launches stand in the host copy for status and stats
  sum.status.v = (uint32_t)status;
  *b.host_ctl = sum;
  if (launches) *launches = nl + 1;
  return IWPP_OK;
}

int enqueue(Buffers& b, const Variant& v, const Resolved& rp, const DevImage& one,
            const DevImage* d_imgs, int nimg, int64_t ntiles, hipStream_t st, int64_t* launches) {
  KParams kp{};
  kp.nimg = nimg;
  kp.sweeps = rp.sweeps;
  kp.ntiles = ntiles;
  kp.max_visits = rp.max_visits;
  kp.spin_limit = rp.spin_limit;
  kp.seed_queue_max = rp.seed_queue_max;
  kp.queue_waves = rp.queue_waves;
  kp.flip = rp.flip;
  kp.band = -1;
  int64_t nl = 0;
  if (rp.mode == 2) return enqueue_bands(b, v, rp, one, d_imgs, nimg, ntiles, st, kp, launches);
  if (rp.mode == 0) {
    int grid = 0;
    int rc = plan_queues(v, rp, ntiles, nimg, one, &grid, &kp);
    if (rc) return rc;
    rc = b.ensure(ntiles, kp.qcap * (uint32_t)kp.nq, nimg, false);
    if (rc) return rc;
    order_for(rp.order_seed, ntiles, &kp.order_mul, &kp.order_add);
    if (d_imgs) {
      // batches: a table of each tile's image replaces the descriptor search
      HIP_TRY(launch_tile_images(d_imgs, nimg, ntiles, b.tile_img, st));
      kp.tile_img = b.tile_img;
      if (rp.order_seed == 0) kp.phase_tx = -1;
    } else if (rp.order_seed == 0) {
      kp.phase_tx = one.tiles_x;
      kp.phase_ty = one.tiles_y;
    }
    kp.phase_diag = rp.first_pass == 2;
    rc = setup_cols(b, v, ntiles, kp);
    if (rc) return rc;
    HIP_TRY(launch_init(kp, b.ctl, b.queue, b.state, b.visited, nullptr, st));
    b.timed = false;
    if (rp.timing) {
      if (!b.ev[0]) HIP_TRY(hipEventCreate(&b.ev[0]));
      if (!b.ev[1]) HIP_TRY(hipEventCreate(&b.ev[1]));
      HIP_TRY(hipEventRecord(b.ev[0], st));
    }
    HIP_TRY(launch_persistent(v, one, d_imgs, kp, b.ctl, b.queue, b.state, b.visited, grid, st));
    if (rp.timing) {
      HIP_TRY(hipEventRecord(b.ev[1], st));
      b.timed = true;
    }
    nl = 2;
  } else {
    kp.qcap = 0;
    kp.nq = 1;
    kp.chunk = 1;
    kp.order_mul = 1;
    int rc = b.ensure(ntiles, 0, nimg, true);
    if (rc) return rc;
    HIP_TRY(launch_init(kp, b.ctl, nullptr, nullptr, b.visited, b.act[0], st));
    nl = 1;
    int cur = 0;
    b.timed = false;
    b.rounds_ms = 0;
    if (rp.timing) {
      if (!b.ev[0]) HIP_TRY(hipEventCreate(&b.ev[0]));
      if (!b.ev[1]) HIP_TRY(hipEventCreate(&b.ev[1]));
    }
    for (int64_t round = 0;; ++round) {
      HIP_TRY(launch_clear_round(b.ctl, st));
      kp.first_round = round == 0;
      if (rp.timing) HIP_TRY(hipEventRecord(b.ev[0], st));
      HIP_TRY(launch_round(v, one, d_imgs, kp, b.ctl, b.act[cur], b.act[cur ^ 1], b.visited, st));
      if (rp.timing) HIP_TRY(hipEventRecord(b.ev[1], st));
      nl += 2;
      HIP_TRY(hipMemcpyAsync(b.host_ctl, b.ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (rp.timing) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, b.ev[0], b.ev[1]));
        b.rounds_ms += ms;
      }
      if (!b.host_ctl->active_any || (b.host_ctl->status.v & ST_INTERNAL)) break;
      if (rp.max_visits > 0 && (int64_t)b.host_ctl->visits >= rp.max_visits) {
        // stop between rounds: the marker holds a valid partial result
        b.incomplete_rounds = true;
        break;
      }
      cur ^= 1;
    }
    if (b.incomplete_rounds) {
      // leave the flags clean for the next call
      HIP_TRY(hipMemsetAsync(b.act[0], 0, b.act_cap, st));
      HIP_TRY(hipMemsetAsync(b.act[1], 0, b.act_cap, st));
    }
  }
  HIP_TRY(hipMemcpyAsync(b.host_ctl, b.ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, st));
  if (launches) *launches = nl;
  return IWPP_OK;
}

int status_of(const DevCtl& c, uint32_t flags, bool incomplete_rounds) {
  const uint32_t st = c.status.v;
  if (st & ST_INTERNAL) return IWPP_E_INTERNAL;
  if ((st & ST_INCOMPLETE) || incomplete_rounds) return IWPP_E_INCOMPLETE;
  if ((st & ST_MARKER_GT_MASK) && !(flags & IWPP_FLAG_CLAMP_MARKER))
    return IWPP_E_MARKER_GT_MASK;
  return IWPP_OK;
}

void fill_stats(const DevCtl& c, int status, int nimg, int64_t ntiles, int64_t launches,
                iwpp_stats* s) {
  if (!s) return;
  std::memset(s, 0, sizeof *s);
  s->status = status;
  s->images = nimg;
  s->tiles = ntiles;
  s->tile_visits = (int64_t)c.visits;
  s->sweep_rounds = (int64_t)c.sweeps;
  s->pixels_queued = (int64_t)c.pushes;
  s->queue_overflows = (int64_t)c.overflows;
  s->reprocessed = (int64_t)c.reproc;
  s->requeued = (int64_t)c.requeued;
  s->launches = launches;
  s->queue_iterations = (int64_t)c.qiters;
  int khz = 100000;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  (void)hipGetLastError();
  s->idle_ms = (double)c.t_idle / khz;
  s->load_ms = (double)c.t_load / khz;
  s->solve_ms = (double)c.t_solve / khz;
  s->store_ms = (double)c.t_store / khz;
  s->sync_ms = (double)c.t_sync / khz;
}

double kernel_ms(Buffers& b) {
  if (b.timed) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, b.ev[0], b.ev[1]) == hipSuccess) return ms;
    (void)hipGetLastError();  // do not leave a stale error for the caller's next launch
    return 0;
  }
  return b.rounds_ms;
}

}  // namespace iwpp

// ================================================================ workspaces

namespace {

struct Workspace {
  Buffers buf;
  uint32_t flags = 0;
  int nimg = 0;
  int64_t ntiles = 0;
  int64_t launches = 0;
  int enqueue_rc = IWPP_OK;
};

std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

int get_workspace(hipStream_t st, Workspace** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_mu);
  auto key = std::make_pair(dev, st);
  auto it = g_ws.find(key);
  if (it == g_ws.end()) {
    Workspace* w = new Workspace();
    w->buf.stream_owner = st;
    it = g_ws.emplace(key, w).first;
  }
  *out = it->second;
  return IWPP_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

int iwpp_version(void) { return 10000; }

const char* iwpp_strerror(int code) {
  switch (code) {
    case IWPP_OK: return "ok";
    case IWPP_E_ARG: return "invalid argument";
    case IWPP_E_MARKER_GT_MASK: return "marker exceeds mask at some pixel";
    case IWPP_E_NOMEM: return "out of memory";
    case IWPP_E_HIP: return "HIP runtime error";
    case IWPP_E_INCOMPLETE: return "stopped at the tile-visit limit (partial result)";
    case IWPP_E_BUDGET: return "request exceeds the server memory budget";
    case IWPP_E_INTERNAL: return "internal error: a bounded device wait ran out";
    case IWPP_E_TIMEOUT: return "timed out";
    case IWPP_E_UNSUPPORTED: return "parameter combination not supported";
    case IWPP_E_SCRATCH: return "image needs more workspace than the static array holds";
    default: return "unknown status";
  }
}

const char* iwpp_last_error(void) { return g_last_error.c_str(); }

int iwpp_reconstruct_async(const iwpp_image* img, int dtype, int conn, uint32_t flags,
                           const iwpp_params* params, iwpp_stream_t stream) {
  int rc = check_common(dtype, conn, flags);
  if (!rc) rc = check_image(img, dtype);
  if (!rc) rc = check_params(params);
  if (rc) return rc;
  Resolved rp = resolve_params(params, dtype, conn, img->H, img->W);
  rp.flip = flip_of(flags);
  const Variant v{dtype, conn, rp.tile_h};
  if (!variant_supported(v)) return IWPP_E_UNSUPPORTED;
  const DevImage one = make_dev_image(*img, rp.tile_h, 0);
  const int64_t ntiles = (int64_t)one.tiles_y * one.tiles_x;
  if (ntiles >= (int64_t(1) << 30)) return IWPP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  rc = get_workspace(st, &w);
  if (rc) return rc;
  w->buf.incomplete_rounds = false;
  w->flags = flags;
  w->nimg = 1;
  w->ntiles = ntiles;
  rc = enqueue(w->buf, v, rp, one, nullptr, 1, ntiles, st, &w->launches);
  w->enqueue_rc = rc;
  return rc;
}

int iwpp_fill_holes_async(const void* image, void* out, int64_t H, int64_t W, int64_t ld,
                          int dtype, int conn, const iwpp_params* params,
                          iwpp_stream_t stream) {
  int rc = check_common(dtype, conn, 0);
  iwpp_image im{};
  im.marker = out;
  im.mask = image;
  im.H = H;
  im.W = W;
  im.ld = ld;
  if (!rc) rc = check_image(&im, dtype);
  if (!rc) rc = check_params(params);
  if (rc) return rc;
  HIP_TRY(launch_frame_marker(dtype, out, image, H, W, ld ? ld : W, (hipStream_t)stream));
  return iwpp_reconstruct_async(&im, dtype, conn, IWPP_FLAG_EROSION, params, stream);
}

int iwpp_edt_async(const void* image, int64_t ld_image, void* sites, void* dist2,
                   int64_t ld_out, int64_t H, int64_t W, int conn, const iwpp_params* params,
                   iwpp_stream_t stream) {
  if (!image || !sites) return IWPP_E_ARG;
  if (conn != 4 && conn != 8) return IWPP_E_ARG;
  if (H < 1 || W < 1 || H > 32768 || W > 32768) return IWPP_E_ARG;
  if ((ld_image != 0 && ld_image < W) || (ld_out != 0 && ld_out < W)) return IWPP_E_ARG;
  const int64_t li = ld_image ? ld_image : W, lo = ld_out ? ld_out : W;
  const uintptr_t a0 = (uintptr_t)image, s0 = (uintptr_t)sites, d0 = (uintptr_t)dist2;
  if ((s0 | d0) & 3u) return IWPP_E_ARG;
  const uintptr_t na = (uintptr_t)((H - 1) * li + W), ns = (uintptr_t)((H - 1) * lo + W) * 4;
  auto overlap = [](uintptr_t p, uintptr_t np, uintptr_t q, uintptr_t nq) {
    return p < q + nq && q < p + np;
  };
  if (overlap(a0, na, s0, ns)) return IWPP_E_ARG;
  if (dist2 && (overlap(a0, na, d0, ns) || overlap(s0, ns, d0, ns))) return IWPP_E_ARG;
  int rc = check_params(params);
  if (rc) return rc;
  Resolved rp = resolve_params(params, IWPP_I32, conn, H, W);
  if ((params && params->tile_h && params->tile_h != 32) || (params && params->mode != 0))
    return IWPP_E_UNSUPPORTED;
  rp.tile_h = 32;
  rp.mode = 0;
  rp.flip = 0;
  const Variant v{kDtypeEdt, conn, rp.tile_h};
  if (!variant_supported(v)) return IWPP_E_UNSUPPORTED;
  iwpp_image im{};
  im.marker = sites;
  im.mask = image;
  im.H = H;
  im.W = W;
  im.ld = lo;
  const DevImage one = make_dev_image(im, rp.tile_h, 0);
  const int64_t ntiles = (int64_t)one.tiles_y * one.tiles_x;
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  rc = get_workspace(st, &w);
  if (rc) return rc;
  HIP_TRY(launch_edt_init(sites, lo, image, li, H, W, st));
  w->buf.incomplete_rounds = false;
  w->flags = 0;
  w->nimg = 1;
  w->ntiles = ntiles;
  rc = enqueue(w->buf, v, rp, one, nullptr, 1, ntiles, st, &w->launches);
  if (!rc && dist2) {
    const hipError_t e = launch_edt_dist(dist2, sites, lo, H, W, st);
    if (e != hipSuccess) rc = IWPP_E_HIP;
  }
  w->enqueue_rc = rc;
  return rc;
}

int iwpp_stream_status(iwpp_stream_t stream, iwpp_stats* stats) {
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  int rc = get_workspace(st, &w);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  if (w->enqueue_rc) return w->enqueue_rc;
  if (!w->buf.host_ctl) return IWPP_E_ARG;  // nothing ran on this stream
  const DevCtl c = *w->buf.host_ctl;
  const int status = status_of(c, w->flags, w->buf.incomplete_rounds);
  fill_stats(c, status, w->nimg, w->ntiles, w->launches, stats);
  if (stats) stats->kernel_ms = kernel_ms(w->buf);
  return status;
}

int iwpp_reconstruct(void* marker, const void* mask, int64_t H, int64_t W, int dtype, int conn) {
  iwpp_image im{marker, mask, H, W, 0};
  int rc = iwpp_reconstruct_async(&im, dtype, conn, 0, nullptr, nullptr);
  if (rc) return rc;
  return iwpp_stream_status(nullptr, nullptr);
}

int iwpp_reconstruct_batched(const iwpp_image* imgs, int32_t n, int dtype, int conn,
                             uint32_t flags, const iwpp_params* params, iwpp_stream_t stream) {
  int rc = check_common(dtype, conn, flags);
  if (!rc && (!imgs || n < 1)) rc = IWPP_E_ARG;
  for (int32_t k = 0; !rc && k < n; ++k) rc = check_image(&imgs[k], dtype);
  if (!rc) rc = check_params(params);
  if (rc) return rc;
  int64_t maxpx = 0;
  for (int32_t k = 0; k < n; ++k) maxpx = std::max<int64_t>(maxpx, imgs[k].H * imgs[k].W);
  Resolved rp = resolve_params(params, dtype, conn, 1, maxpx);
  rp.flip = flip_of(flags);
  const Variant v{dtype, conn, rp.tile_h};
  if (!variant_supported(v)) return IWPP_E_UNSUPPORTED;
  std::vector<DevImage> h(n);
  int64_t base = 0;
  for (int32_t k = 0; k < n; ++k) {
    h[k] = make_dev_image(imgs[k], rp.tile_h, base);
    base += (int64_t)h[k].tiles_y * h[k].tiles_x;
  }
  if (base >= (int64_t(1) << 30)) return IWPP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  rc = get_workspace(st, &w);
  if (rc) return rc;
  // the descriptor buffer may still be read by an earlier launch
  HIP_TRY(hipStreamSynchronize(st));
  rc = w->buf.ensure(base, 0, n, false);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(w->buf.descs, h.data(), n * sizeof(DevImage), hipMemcpyHostToDevice));
  w->buf.incomplete_rounds = false;
  w->flags = flags;
  w->nimg = n;
  w->ntiles = base;
  rc = enqueue(w->buf, v, rp, h[0], w->buf.descs, n, base, st, &w->launches);
  w->enqueue_rc = rc;
  return rc;
}

int iwpp_release_workspace(void) {
  HIP_TRY(hipDeviceSynchronize());
  std::lock_guard<std::mutex> g(g_mu);
  for (auto& kv : g_ws) {
    kv.second->buf.release();
    delete kv.second;
  }
  g_ws.clear();
  return IWPP_OK;
}

int iwpp_device_copy(void* dst, const void* src, size_t bytes, iwpp_stream_t stream) {
  if (!dst || !src || bytes == 0 || (bytes & 15u)) return IWPP_E_ARG;
  HIP_TRY(launch_copy(dst, src, bytes, (hipStream_t)stream));
  return IWPP_OK;
}

// ---------------------------------------------------------------- batch plans

struct iwpp_batch {
  int device = 0;
  int dtype = 0, conn = 8;
  uint32_t flags = 0;
  Resolved rp{};
  Variant v{};
  std::vector<DevImage> h;
  int64_t ntiles = 0;
  Buffers buf;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t graph_stream = nullptr;
  hipStream_t last_stream = nullptr;
  int64_t launches = 0;
  int launch_rc = IWPP_OK;
};

int iwpp_batch_create(const iwpp_image* imgs, int32_t n, int dtype, int conn, uint32_t flags,
                      const iwpp_params* params, iwpp_batch** out) {
  if (!out) return IWPP_E_ARG;
  *out = nullptr;
  int rc = check_common(dtype, conn, flags);
  if (!rc && (!imgs || n < 1)) rc = IWPP_E_ARG;
  for (int32_t k = 0; !rc && k < n; ++k) rc = check_image(&imgs[k], dtype);
  if (!rc) rc = check_params(params);
  if (rc) return rc;
  int64_t maxpx = 0;
  for (int32_t k = 0; k < n; ++k) maxpx = std::max<int64_t>(maxpx, imgs[k].H * imgs[k].W);
  iwpp_batch* b = new iwpp_batch();
  b->dtype = dtype;
  b->conn = conn;
  b->flags = flags;
  b->rp = resolve_params(params, dtype, conn, 1, maxpx);
  b->rp.flip = flip_of(flags);
  if (b->rp.mode != 0) b->rp.mode = 0;  // plans always use the persistent kernel
  b->v = Variant{dtype, conn, b->rp.tile_h};
  if (!variant_supported(b->v)) {
    delete b;
    return IWPP_E_UNSUPPORTED;
  }
  b->h.resize(n);
  int64_t base = 0;
  for (int32_t k = 0; k < n; ++k) {
    b->h[k] = make_dev_image(imgs[k], b->rp.tile_h, base);
    base += (int64_t)b->h[k].tiles_y * b->h[k].tiles_x;
  }
  if (base >= (int64_t(1) << 30)) {
    delete b;
    return IWPP_E_ARG;
  }
  b->ntiles = base;
  hipError_t e = hipGetDevice(&b->device);
  int grid = 0;
  if (e != hipSuccess) rc = hip_fail(e, "hipGetDevice");
  KParams kp{};
  if (!rc) rc = plan_queues(b->v, b->rp, base, n, b->h[0], &grid, &kp);
  if (!rc) rc = b->buf.ensure(base, kp.qcap * (uint32_t)kp.nq, n, false);
  // sized now: a graph capture of the launch must not allocate
  if (!rc) rc = b->buf.ensure_cols_for(b->v.dtype, b->v.tile_h, base);
  if (!rc) {
    e = hipMemcpy(b->buf.descs, b->h.data(), n * sizeof(DevImage), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy(descs)");
  }
  if (rc) {
    b->buf.release();
    delete b;
    return rc;
  }
  *out = b;
  return IWPP_OK;
}

int iwpp_batch_launch(iwpp_batch* b, iwpp_stream_t stream, int use_graph) {
  if (!b) return IWPP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  b->last_stream = st;
  if (!use_graph) {
    b->launch_rc = enqueue(b->buf, b->v, b->rp, b->h[0], b->buf.descs, (int)b->h.size(),
                           b->ntiles, st, &b->launches);
    return b->launch_rc;
  }
  if (!b->exec) {
    // Capture on a private stream so the caller's stream is never in
    // capture mode; the sequence has no memset nodes (buffers are reset by
    // the init kernel).
    HIP_TRY(hipStreamCreateWithFlags(&b->graph_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->graph_stream, hipStreamCaptureModeThreadLocal));
    int64_t nl = 0;
    Resolved rp = b->rp;
    rp.timing = 0;  // timing events bracket the graph launch, not nodes inside it
    int rc = enqueue(b->buf, b->v, rp, b->h[0], b->buf.descs, (int)b->h.size(), b->ntiles,
                     b->graph_stream, &nl);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->graph_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->launches = nl;
  }
  b->buf.timed = false;
  if (b->rp.timing) {
    if (!b->buf.ev[0]) HIP_TRY(hipEventCreate(&b->buf.ev[0]));
    if (!b->buf.ev[1]) HIP_TRY(hipEventCreate(&b->buf.ev[1]));
    HIP_TRY(hipEventRecord(b->buf.ev[0], st));
  }
  HIP_TRY(hipGraphLaunch(b->exec, st));
  if (b->rp.timing) {
    HIP_TRY(hipEventRecord(b->buf.ev[1], st));
    b->buf.timed = true;
  }
  b->launch_rc = IWPP_OK;
  return IWPP_OK;
}

int iwpp_batch_status(iwpp_batch* b, iwpp_stats* stats) {
  if (!b) return IWPP_E_ARG;
  HIP_TRY(hipStreamSynchronize(b->last_stream));
  if (b->launch_rc) return b->launch_rc;
  const DevCtl c = *b->buf.host_ctl;
  const int status = status_of(c, b->flags, false);
  fill_stats(c, status, (int)b->h.size(), b->ntiles, b->launches, stats);
  if (stats) stats->kernel_ms = kernel_ms(b->buf);
  return status;
}

int iwpp_batch_destroy(iwpp_batch* b) {
  if (!b) return IWPP_E_ARG;
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->graph_stream) (void)hipStreamDestroy(b->graph_stream);
  b->buf.release();
  delete b;
  return IWPP_OK;
}

// ---------------------------------------------------------------- autotuner

int iwpp_autotune(const iwpp_image* img, int dtype, int conn, iwpp_stream_t stream,
                  iwpp_params* best) {
  int rc = check_common(dtype, conn, 0);
  if (!rc) rc = check_image(img, dtype);
  if (!rc && !best) rc = IWPP_E_ARG;
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t ld = img->ld ? img->ld : img->W;
  const size_t es = dtype == IWPP_U8 ? 1 : 4;
  const size_t bytes = (size_t)((img->H - 1) * ld + img->W) * es;
  void* scratch = nullptr;
  HIP_TRY(hipMalloc(&scratch, bytes));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // median of three timed runs (after one warm-up) from the pristine marker
  auto time_of = [&](const iwpp_params& p, float* out) -> int {
    iwpp_image im = *img;
    im.marker = scratch;
    std::vector<float> times;
    for (int rep = 0; rep < 4; ++rep) {
      (void)hipMemcpyAsync(scratch, img->marker, bytes, hipMemcpyDeviceToDevice, st);
      (void)hipEventRecord(e0, st);
      int r = iwpp_reconstruct_async(&im, dtype, conn, IWPP_FLAG_CLAMP_MARKER, &p, stream);
      (void)hipEventRecord(e1, st);
      const int s2 = iwpp_stream_status(stream, nullptr);
      if (!r && s2 != IWPP_OK) r = s2;
      if (r) return r;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep) times.push_back(ms);
    }
    std::sort(times.begin(), times.end());
    *out = times[times.size() / 2];
    return IWPP_OK;
  };
  // coordinate descent: tile height x sweeps, then the seeded-queue bound,
  // then the queue-wave bound, each stage starting from the best so far
  const std::vector<int> tiles =
      dtype == IWPP_U8 ? std::vector<int>{64, 128} : std::vector<int>{32, 64};
  float best_ms = 1e30f;
  iwpp_params bp{};
  auto consider = [&](const iwpp_params& p) -> int {
    float ms = 0;
    const int r = time_of(p, &ms);
    if (!r && ms < best_ms) {
      best_ms = ms;
      bp = p;
    }
    return r;
  };
  for (int th : tiles)
    for (int sw : {1, 2, 4, 8, 16, -1}) {
      iwpp_params p{};
      p.tile_h = th;
      p.sweeps = sw;
      if (!rc) rc = consider(p);
    }
  for (int sq : {8, 32, -1}) {
    iwpp_params p = bp;
    p.seed_queue = sq;
    if (!rc) rc = consider(p);
  }
  for (int qw : {4, 16, 64, -1}) {
    iwpp_params p = bp;
    p.queue_waves = qw;
    if (!rc) rc = consider(p);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(scratch);
  if (rc) return rc;
  *best = bp;
  std::lock_guard<std::mutex> g(g_mu);
  load_tune_cache_locked();
  g_tuned[{dtype, conn, size_class(img->H, img->W)}] = bp;
  save_tune_cache_locked();
  return IWPP_OK;
}

}  // extern "C"
