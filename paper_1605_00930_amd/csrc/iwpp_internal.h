// iwpp_internal.h -- device-side data layout shared by the HIP kernels and
// the host runtime of the reconstruction library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iwpp {

// One image of a launch.  Tiles of all images of a launch are numbered
// consecutively: image k owns tile ids [tile_base, tile_base + tiles_y*tiles_x).
struct DevImage {
  void* J;           // marker, reconstructed in place (device)
  const void* I;     // mask (device)
  int64_t H, W, ld;  // rows, columns, row pitch in elements
  int32_t tiles_y, tiles_x;
  int64_t tile_base;
};

// Control block of one launch (device memory, zeroed by the init kernel).
struct DevCtl {
  uint32_t q_head;   // next queue slot to claim
  uint32_t q_tail;   // next queue slot to fill
  int32_t pending;   // tiles queued or running
  int32_t status;    // ST_* bits
  uint64_t visits;   // tile visits (first visits, re-visits, in-place reprocessing)
  uint64_t sweeps;   // rounds of the four directional passes
  uint64_t pushes;   // entries written to tile queues
  uint64_t overflows;
  uint64_t reproc;   // in-place reprocessing after a neighbour changed mid-visit
  uint32_t q_high;   // queue high-water mark
  int32_t active_any;  // host-driven rounds: some tile was activated
  uint64_t launches;   // filled by the host
};

enum : int32_t {
  ST_MARKER_GT_MASK = 1,  // some marker pixel exceeded its mask pixel
  ST_INCOMPLETE = 2,      // stopped at the tile-visit cap
  ST_INTERNAL = 4,        // a bounded wait or in-tile loop hit its limit
  ST_ABORT = 8,           // workers must stop
};

// Per-tile state word (persistent mode).
enum : uint32_t {
  TS_PENDING = 1u,  // needs a (re)visit: queued, or re-run by its current owner
  TS_RUNNING = 2u,  // owned by a workgroup
};

struct KParams {
  int32_t nimg;
  int32_t sweeps;       // max rounds of directional passes before the queue
  int64_t ntiles;
  int64_t max_visits;   // 0 = unlimited
  uint32_t qcap;        // global queue capacity (slots)
  uint32_t spin_limit;  // bounded waits (iterations)
  int32_t first_round;  // host-driven rounds: this is the first round
  int32_t pad;
};

// Host-side launchers (iwpp_kernels.hip).  dtype: 0 = u8, 1 = i32.
// Return hipSuccess or the launch error.
struct Variant {
  int dtype, conn, tile_h;
};
bool variant_supported(const Variant& v);
hipError_t launch_init(const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                       uint8_t* visited, uint8_t* active, uint32_t order_mul,
                       uint32_t order_add, hipStream_t st);
hipError_t launch_persistent(const Variant& v, const DevImage& one, const DevImage* imgs,
                             const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                             uint8_t* visited, int grid, hipStream_t st);
hipError_t launch_round(const Variant& v, const DevImage& one, const DevImage* imgs,
                        const KParams& kp, DevCtl* ctl, uint8_t* act_cur, uint8_t* act_next,
                        uint8_t* visited, hipStream_t st);
hipError_t launch_clear_round(DevCtl* ctl, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
int persistent_blocks_per_cu(const Variant& v);

constexpr int kTileW = 64;     // one wavefront spans a tile row
constexpr int kThreads = 256;  // four wavefronts per workgroup

}  // namespace iwpp
