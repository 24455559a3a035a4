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

// Control block of one launch (device memory, reset by the init kernel).
// Words that many wavefronts hit with atomics sit on their own 128-byte
// lines.
constexpr int kMaxQueues = 8;  // one tile queue per XCD
struct alignas(128) HotWord {
  uint32_t v;
  uint32_t pad[31];
};
struct DevCtl {
  HotWord fphead[kMaxQueues];  // next first-pass chunk of each queue
  HotWord head[kMaxQueues];    // next ring ticket of each queue
  HotWord tail[kMaxQueues];    // next fill position of each queue
  HotWord pending;           // tiles queued or running (int32)
  HotWord status;            // ST_* bits (int32)
  HotWord done;              // set once no more work can arrive
  HotWord visits_cap;        // visit counter, only used with a visit limit
  HotWord next_len;          // gray-level bands: tiles appended to the next launch's list
  HotWord max_deferred;      // gray-level bands: highest class deferred (int32, -1 none)
  uint64_t visits;     // tile visits (first visits, re-visits, in-place reprocessing)
  uint64_t sweeps;     // rounds of the four directional passes
  uint64_t pushes;     // entries processed by tile queues
  uint64_t overflows;  // tile-queue overflows
  uint64_t reproc;     // in-place reprocessing after a neighbour changed mid-visit
  uint64_t requeued;   // tiles put back on a queue after their first visit
  uint64_t qiters;     // queue-loop iterations (identify + propagate pairs)
  int32_t active_any;  // host-driven rounds: some tile was activated
  int32_t pad0;
  // wavefront time (wall_clock64 ticks, summed over workers) spent waiting
  // for work, loading tiles, solving tiles, storing them and publishing them
  // (release fence + tile-state updates)
  uint64_t t_idle, t_load, t_solve, t_store, t_sync;
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
  uint32_t qcap;        // ring capacity of each tile queue (slots)
  uint32_t spin_limit;  // bounded waits (iterations)
  int32_t first_round;  // host-driven rounds: this is the first round
  int32_t seed_queue_max;  // re-visits with at most this many halo receivers skip the scans
  uint32_t queue_waves;    // queue waves before a tile falls back to sweep rounds
  uint32_t flip;           // 0: dilation; ~0u: erosion (values complemented in the tile)
  // Gray-level bands (mode 2): activations whose value class
  // (value - band_base) >> band_shift is below `band` are deferred to a later
  // launch instead of being queued.  band < 0: no bands.
  int32_t band;
  int32_t band_base;
  uint32_t band_shift;
  int32_t list_mode;       // the first pass is list_in[0 .. list_len) (else all tiles)
  int64_t list_len;
  const int* list_in;
  int* list_out;           // tiles with deferred work for the next launch
  int* dclass;             // per tile: highest deferred class, -1 none
  uint32_t* listed;        // per tile: already in list_out
  int32_t nq;           // tile queues in use (1..kMaxQueues)
  int32_t chunk;        // consecutive tile ids per queue chunk: tile t is in queue (t / chunk) % nq
  uint32_t order_mul, order_add;  // first-pass order: tile = (i * mul + add) mod ntiles
  // four-phase first pass (see phase_tile): the tile grid of a single image,
  // or phase_tx = -1 for a batch, each image on its own (0: off); phase_diag
  // takes the two diagonal groups first
  int32_t phase_tx, phase_ty;
  int32_t phase_diag;
  const int32_t* tile_img;  // batches: image index of every tile (or null)
  // packed side columns of I and J (column 0 and TW - 1 of every tile, row
  // after row), written by each tile from its first visit on (null: halo
  // columns are read from the image)
  const void* colI;
  void* colJ;
};

// Host-side launchers (iwpp_kernels.hip).  dtype: 0 = u8, 1 = i32.
// Return hipSuccess or the launch error.
struct Variant {
  int dtype, conn, tile_h;
};
bool variant_supported(const Variant& v);
hipError_t launch_tile_images(const DevImage* imgs, int nimg, int64_t ntiles, int32_t* out,
                              hipStream_t st);

hipError_t launch_init(const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                       uint8_t* visited, uint8_t* active, hipStream_t st);
hipError_t launch_persistent(const Variant& v, const DevImage& one, const DevImage* imgs,
                             const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                             uint8_t* visited, int grid, hipStream_t st);
hipError_t launch_round(const Variant& v, const DevImage& one, const DevImage* imgs,
                        const KParams& kp, DevCtl* ctl, uint8_t* act_cur, uint8_t* act_next,
                        uint8_t* visited, hipStream_t st);
hipError_t launch_clear_round(DevCtl* ctl, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// Gray-level bands: mark the tiles of kp.list_in pending; min / max of the
// marker (tile order) into out[0], out[1] (which the caller initialises).
hipError_t launch_list_mark(const KParams& kp, uint32_t* state, hipStream_t st);
hipError_t launch_minmax(int dtype, const void* J, int64_t H, int64_t W, int64_t ld,
                         uint32_t flip, int* out, hipStream_t st);
// out <- image on the 1-pixel frame, the highest value inside (fill-holes marker).
hipError_t launch_frame_marker(int dtype, void* out, const void* img, int64_t H, int64_t W,
                               int64_t ld, hipStream_t st);
int persistent_blocks_per_cu(const Variant& v);

// Distance transform (iwpp_edt.hip).  Its variants use dtype kDtypeEdt.
constexpr int kDtypeEdt = 2;
bool edt_variant_supported(int conn, int tile_h);
hipError_t launch_persistent_edt(int conn, int tile_h, const DevImage& one, const KParams& kp,
                                 DevCtl* ctl, int* queue, uint32_t* state, uint8_t* visited,
                                 int grid, hipStream_t st);
int persistent_edt_blocks_per_cu(int conn, int tile_h);
// sites <- own position (background, image value 0) or none (object)
hipError_t launch_edt_init(void* sites, int64_t ld_out, const void* img, int64_t ld_img,
                           int64_t H, int64_t W, hipStream_t st);
// dist <- squared distance of each pixel to its site (-1: none)
hipError_t launch_edt_dist(void* dist, const void* sites, int64_t ld_out, int64_t H, int64_t W,
                           hipStream_t st);

constexpr int kTileW = 64;    // one lane per tile column
constexpr int kThreads = 64;  // one wavefront per workgroup, one tile per wavefront

}  // namespace iwpp
