// iwpp_runtime.h -- host-side pieces shared by the C-ABI implementation files
// (iwpp_api.cpp, iwpp_server.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "iwpp.h"
#include "iwpp_internal.h"

namespace iwpp {

// Parameters after defaults, tuned values and user overrides.
struct Resolved {
  int tile_h;
  int sweeps;
  int mode;
  int grid;
  int64_t max_visits;
  uint32_t order_seed;
  uint32_t spin_limit;
  int timing;
  int seed_queue_max;
  uint32_t queue_waves;
  uint32_t flip;  // 0 dilation, ~0u erosion (from IWPP_FLAG_EROSION)
  int bands;      // mode 2: number of gray-level classes
  int first_pass; // 1 first-visit groups by rows of the group grid, 2 diagonal groups first
};

// Device buffers of one launch context (a stream workspace, a batch plan or a
// server slot).  Grown on demand; release() frees everything.
struct Buffers {
  DevCtl* ctl = nullptr;
  DevCtl* host_ctl = nullptr;  // pinned copy of the control block
  int* queue = nullptr;
  uint32_t* state = nullptr;
  uint8_t* visited = nullptr;
  uint8_t* act[2] = {nullptr, nullptr};
  DevImage* descs = nullptr;
  int32_t* tile_img = nullptr;  // batches: image index per tile (tiles_cap entries)
  void* cols = nullptr;         // packed side columns of I and J
  int64_t cols_cap = 0;         // bytes
  int64_t tiles_cap = 0;
  int64_t act_cap = 0;
  uint32_t qcap_cap = 0;
  int descs_cap = 0;
  hipStream_t stream_owner = nullptr;
  bool incomplete_rounds = false;
  hipEvent_t ev[2] = {nullptr, nullptr};  // kernel timing (created on demand)
  bool timed = false;                     // last enqueue recorded ev[0..1]
  double rounds_ms = 0;                   // host-driven rounds: summed kernel time
  // gray-level bands
  int* dclass = nullptr;
  uint32_t* listed = nullptr;
  int* list[2] = {nullptr, nullptr};
  int* minmax = nullptr;
  int64_t band_cap = 0;
  int ensure(int64_t ntiles, uint32_t qcap, int nimg, bool rounds);
  int ensure_bands(int64_t ntiles);
  int ensure_cols(int64_t bytes);
  // ensure_cols for a reconstruction launch of `ntiles` tiles of variant v
  int ensure_cols_for(int dtype, int tile_h, int64_t ntiles) {
    return ensure_cols(2 * ntiles * 2 * tile_h * (dtype == 0 ? 1 : 4));
  }
  void release();
};

Resolved resolve_params(const iwpp_params* user, int dtype, int conn, int64_t H, int64_t W,
                        bool tuned = true);
int check_params(const iwpp_params* p);
int check_image(const iwpp_image* im, int dtype);
int check_common(int dtype, int conn, uint32_t flags);
DevImage make_dev_image(const iwpp_image& im, int tile_h, int64_t tile_base);
int device_grid(const Variant& v, int64_t ntiles, int want, int* grid);
int plan_queues(const Variant& v, const Resolved& rp, int64_t ntiles, int nimg,
                const DevImage& one, int* grid, KParams* kp);
int plan_queues_for_grid(int grid, int64_t ntiles, int nimg, const DevImage& one, KParams* kp);
uint32_t flip_of(uint32_t flags);
void order_for(uint32_t seed, int64_t ntiles, uint32_t* mul, uint32_t* add);
int enqueue(Buffers& b, const Variant& v, const Resolved& rp, const DevImage& one,
            const DevImage* d_imgs, int nimg, int64_t ntiles, hipStream_t st, int64_t* launches);
int status_of(const DevCtl& c, uint32_t flags, bool incomplete_rounds);
void fill_stats(const DevCtl& c, int status, int nimg, int64_t ntiles, int64_t launches,
                iwpp_stats* s);
double kernel_ms(Buffers& b);

}  // namespace iwpp
