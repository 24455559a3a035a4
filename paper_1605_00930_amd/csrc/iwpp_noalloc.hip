// iwpp_noalloc.hip -- iwpp_reconstruct_noalloc: the single-image persistent
// reconstruction of iwpp_reconstruct_async for callers that cannot allocate
// (code under HIP graph capture, tight serving loops).  Its library
// workspace (control block, per-tile state and first-visit flags, tile-queue
// rings, packed side columns) lives in one file-scope device array,
// `scratch`, instead of buffers the library allocates; the device status is
// written by a small kernel into a caller-owned device word instead of a
// pinned host copy.  The kernels are the same as the existing entry point's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "iwpp.h"
#include "iwpp_internal.h"
#include "iwpp_runtime.h"

namespace iwpp {
namespace {

// Largest workspace one call may use.  Every device the library runs on
// holds this array until the process ends.
constexpr size_t kScratchBytes = IWPP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Upper bound on the persistent grid assumed when sizing a call's workspace,
// so that whether an image fits does not depend on the device.
constexpr int64_t kGridBound = 8192;

constexpr int kMaxDevices = 64;
constexpr int kVariants = 8;  // (uint8 | int32) x (4 | 8) x (two tile heights)

struct DeviceRecord {
  bool ready = false;
  uint8_t* base = nullptr;  // device address of `scratch` on this device
  int cus = 0;
  int per_cu[kVariants] = {};
};

std::mutex g_mu;
DeviceRecord g_dev[kMaxDevices];

int variant_index(const Variant& v) {
  const int th = v.dtype == IWPP_U8 ? (v.tile_h == 64 ? 0 : 1) : (v.tile_h == 32 ? 0 : 1);
  return v.dtype * 4 + (v.conn == 8 ? 2 : 0) + th;
}

// Once per device, with that device current: the device address of the
// array (in host code its name is only a host-side stand-in), the CU count
// and the resident workgroups per CU of every persistent variant.  None of
// these calls allocates.
int setup_device(int dev, DeviceRecord** out) {
  if (dev < 0 || dev >= kMaxDevices) return IWPP_E_ARG;
  std::lock_guard<std::mutex> g(g_mu);
  DeviceRecord& r = g_dev[dev];
  if (!r.ready) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return IWPP_E_HIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1) {
      (void)hipGetLastError();
      return IWPP_E_HIP;
    }
    for (int dt = 0; dt < 2; ++dt)
      for (int conn : {4, 8})
        for (int th : dt == 0 ? std::initializer_list<int>{64, 128}
                              : std::initializer_list<int>{32, 64}) {
          const Variant v{dt, conn, th};
          r.per_cu[variant_index(v)] = persistent_blocks_per_cu(v);
        }
    r.base = (uint8_t*)p;
    r.cus = cus;
    r.ready = true;
  }
  *out = &r;
  return IWPP_OK;
}

// Carves the workspace of a launch out of the array, 256-byte aligned parts;
// returns the bytes used.  With base == nullptr only the size is computed.
struct Carve {
  DevCtl* ctl;
  uint32_t* state;
  uint8_t* visited;
  int* queue;
  void* cols;
};
size_t carve(uint8_t* base, int64_t ntiles, int64_t ring_slots, int tile_h, int esize,
             Carve* c) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return (void*)p;
  };
  c->ctl = (DevCtl*)take(sizeof(DevCtl));
  c->state = (uint32_t*)take((size_t)ntiles * 4);
  c->visited = (uint8_t*)take((size_t)ntiles);
  c->queue = (int*)take((size_t)ring_slots * 4);
  c->cols = take((size_t)(2 * ntiles * 2 * tile_h) * esize);
  return off;
}

// The status the call reports, from the control block (as iwpp_stream_status
// derives it on the host for the existing entry point).
__global__ void k_write_status(const DevCtl* ctl, uint32_t flags, int32_t* out) {
  const uint32_t st = ctl->status.v;
  int32_t r = IWPP_OK;
  if (st & ST_INTERNAL)
    r = IWPP_E_INTERNAL;
  else if (st & ST_INCOMPLETE)
    r = IWPP_E_INCOMPLETE;
  else if ((st & ST_MARKER_GT_MASK) && !(flags & IWPP_FLAG_CLAMP_MARKER))
    r = IWPP_E_MARKER_GT_MASK;
  *out = r;
}

}  // namespace
}  // namespace iwpp

using namespace iwpp;

extern "C" int iwpp_reconstruct_noalloc(const iwpp_image* img, int dtype, int conn,
                                        uint32_t flags, const iwpp_params* params,
                                        int32_t* status, iwpp_stream_t stream) {
  int rc = check_common(dtype, conn, flags);
  if (!rc) rc = check_image(img, dtype);
  if (!rc) rc = check_params(params);
  if (rc) return rc;
  if (params && params->mode != 0) return IWPP_E_UNSUPPORTED;  // they wait on the host
  Resolved rp = resolve_params(params, dtype, conn, img->H, img->W, /*tuned=*/false);
  rp.flip = flip_of(flags);
  const Variant v{dtype, conn, rp.tile_h};
  if (!variant_supported(v)) return IWPP_E_UNSUPPORTED;
  const DevImage one = make_dev_image(*img, rp.tile_h, 0);
  const int64_t ntiles = (int64_t)one.tiles_y * one.tiles_x;
  const int esize = dtype == IWPP_U8 ? 1 : 4;
  // the size check comes before any device call: it is the same on every
  // device (ring slots sized for the largest grid)
  {
    KParams kb{};
    const int gb = (int)(ntiles < kGridBound ? ntiles : kGridBound);
    if (plan_queues_for_grid(gb, ntiles, 1, one, &kb)) return IWPP_E_ARG;
    Carve c{};
    if (carve(nullptr, ntiles, (int64_t)kb.nq * kb.qcap, rp.tile_h, esize, &c) > kScratchBytes)
      return IWPP_E_SCRATCH;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return IWPP_E_HIP;
  }
  DeviceRecord* r = nullptr;
  rc = setup_device(dev, &r);
  if (rc) return rc;
  int64_t grid = (int64_t)(r->per_cu[variant_index(v)] > 0 ? r->per_cu[variant_index(v)] : 1) *
                 r->cus;
  if (rp.grid > 0 && rp.grid < grid) grid = rp.grid;
  if (grid > ntiles) grid = ntiles;
  if (grid > kGridBound) grid = kGridBound;
  KParams kp{};
  kp.nimg = 1;
  kp.sweeps = rp.sweeps;
  kp.ntiles = ntiles;
  kp.max_visits = rp.max_visits;
  kp.spin_limit = rp.spin_limit;
  kp.seed_queue_max = rp.seed_queue_max;
  kp.queue_waves = rp.queue_waves;
  kp.flip = rp.flip;
  kp.band = -1;
  rc = plan_queues_for_grid((int)grid, ntiles, 1, one, &kp);
  if (rc) return rc;
  order_for(rp.order_seed, ntiles, &kp.order_mul, &kp.order_add);
  if (rp.order_seed == 0) {
    kp.phase_tx = one.tiles_x;
    kp.phase_ty = one.tiles_y;
  }
  kp.phase_diag = rp.first_pass == 2;
  Carve c{};
  carve(r->base, ntiles, (int64_t)kp.nq * kp.qcap, rp.tile_h, esize, &c);
  const int64_t ncol = ntiles * 2 * rp.tile_h;
  kp.colI = c.cols;
  kp.colJ = (uint8_t*)c.cols + ncol * esize;
  hipStream_t st = (hipStream_t)stream;
  // the init kernel resets the control block, tile states, first-visit
  // flags and queue rings (the previous call's contents stay otherwise);
  // packed columns are written before they are read
  if (launch_init(kp, c.ctl, c.queue, c.state, c.visited, nullptr, st) != hipSuccess ||
      launch_persistent(v, one, nullptr, kp, c.ctl, c.queue, c.state, c.visited, (int)grid, st) !=
          hipSuccess) {
    (void)hipGetLastError();
    return IWPP_E_HIP;
  }
  if (status) {
    hipLaunchKernelGGL(k_write_status, dim3(1), dim3(1), 0, st, (const DevCtl*)c.ctl, flags,
                       status);
    if (hipGetLastError() != hipSuccess) return IWPP_E_HIP;
  }
  return IWPP_OK;
}
