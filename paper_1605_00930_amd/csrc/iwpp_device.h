// iwpp_device.h -- device-side pieces shared by the tile kernels: memory
// primitives, per-visit and per-worker counters, the persistent tile queue
// (tickets, ring slots, single-owner tile states, termination) and the
// persistent worker loop, which is generic over the tile policy that loads,
// solves and writes back one tile.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "iwpp_internal.h"

namespace iwpp {

constexpr int TW = kTileW;  // 64: one lane per tile column
static_assert(kThreads == 64, "one wavefront per tile");

// ------------------------------------------------------------ primitives

__device__ __forceinline__ uint32_t ld_rlx_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_rlx_i32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Marker pixels cross workgroups that may sit on different XCDs, each with
// its own L2.  They are only ever read and written with agent-scope relaxed
// atomic accesses: on gfx950 such a load is served coherently for the whole
// device and such a store writes through, so no L2 write-back or invalidate
// (what an agent-scope fence costs) is needed to hand a tile from one
// workgroup to another.  Ordering comes from drain_memory() below.
template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ T ld_coherent(gptr<const T> p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coherent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coherent(__attribute__((address_space(1))) T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sixteen bytes per lane through a buffer resource over `bytes` bytes from
// `base`: ld_coherent_b128 with the cache policy an agent-scope relaxed load
// gets on gfx950 (sc1), for marker rows; ld_plain_b128 without it, for the
// mask, which nothing writes during a launch.  One instruction then carries
// four rows of a 64-column int32 tile where dword loads carry one.
typedef int int4v __attribute__((ext_vector_type(4)));
constexpr int kPolicySc1 = 16;  // cache-policy bit of a buffer access: sc1
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const void* base, uint32_t bytes) {
  // word 3: 32-bit data format (a raw buffer access needs a non-zero one)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ int4v ld_coherent_b128(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                  uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kPolicySc1);
}
__device__ __forceinline__ int4v ld_plain_b128(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                               uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}

// Wait until every memory access this wavefront has issued is complete (an
// agent-scope store is then visible to the whole device), and keep the
// compiler from moving memory accesses across the wait.  Used after the
// marker write-back, before the tile is published, and after a tile is
// taken, before its marker is read.
__device__ __forceinline__ void drain_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Orders this wavefront's LDS accesses before and after the call (a
// one-wavefront workgroup barrier; the compiler keeps its memory fences).
__device__ __forceinline__ void wsync() { __syncthreads(); }

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// OR of v over the wavefront, as a scalar: an inclusive OR-scan within each
// row of 16 lanes (row_shr 1, 2, 4, 8), then rows joined by the row
// broadcasts of lane 15 (into rows 1 and 3) and lane 31 (into rows 2 and
// 3), so that lane 63 holds the OR of all lanes.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

__device__ __forceinline__ uint64_t now() { return wall_clock64(); }

// Per-visit work counters, kept by the wavefront (uniform values).
struct VisitStats {
  uint32_t pushes = 0, rounds = 0, iters = 0, ovf = 0;
};

// ------------------------------------------------------------ helpers

__device__ __forceinline__ int find_image(const DevImage* imgs, int nimg, int64_t t) {
  int lo = 0, hi = nimg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (imgs[mid].tile_base <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// The image of tile t of a batch: from the per-tile table when there is one.
__device__ __forceinline__ int image_of(const KParams& kp, const DevImage* imgs, int64_t t) {
  return kp.tile_img ? kp.tile_img[t] : find_image(imgs, kp.nimg, t);
}

__device__ __forceinline__ void add64(uint64_t* p, uint64_t v) {
  if (v) atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

// Per-worker totals, flushed once when the worker exits.
// 32-bit counts are enough for one worker within one launch (the wall clock
// runs at 100 MHz, 43 s before a per-worker timer wraps).
struct WorkerStats {
  uint32_t pushes = 0, rounds = 0, iters = 0, ovf = 0, visits = 0, reproc = 0, requeued = 0;
  uint32_t t_idle = 0, t_load = 0, t_solve = 0, t_store = 0, t_sync = 0;
  __device__ void add(const VisitStats& v) {
    pushes += v.pushes;
    rounds += v.rounds;
    iters += v.iters;
    ovf += v.ovf;
  }
  __device__ void flush(DevCtl* ctl) const {
    add64(&ctl->pushes, pushes);
    add64(&ctl->sweeps, rounds);
    add64(&ctl->qiters, iters);
    add64(&ctl->overflows, ovf);
    add64(&ctl->visits, visits);
    add64(&ctl->reproc, reproc);
    add64(&ctl->requeued, requeued);
    add64(&ctl->t_idle, t_idle);
    add64(&ctl->t_load, t_load);
    add64(&ctl->t_solve, t_solve);
    add64(&ctl->t_store, t_store);
    add64(&ctl->t_sync, t_sync);
  }
};

// ------------------------------------------------------------ persistent
//
// Tile queues.  Tile t belongs to queue (t / chunk) % nq; workgroup w
// serves queue w % nq (workgroups are dealt to the 8 XCDs in turn, so a
// queue's tiles are handled under one L2, and chunks of neighbouring tiles
// are spread over all queues).  A pop is one atomicAdd on the queue head:
// ticket h.  Tickets below the queue's first-pass length map directly to
// the tiles of the initial pass (no ring traffic); later tickets wait on
// their ring slot until a producer fills it.  The worker that brings the
// pending count to zero marks the launch done and writes a stop value into
// every slot a waiter may hold.

constexpr int kSlotEmpty = -1;
constexpr int kSlotStop = -3;

__device__ __forceinline__ int queue_of(const KParams& kp, int64_t t) {
  return (int)((t / kp.chunk) % kp.nq);
}

// Number of tiles of queue q's first pass: chunks q, q + nq, ...
__device__ __forceinline__ int64_t first_pass_len(const KParams& kp, int q) {
  // list mode: entry i of the list belongs to queue i % nq
  if (kp.list_mode) return q < kp.list_len ? (kp.list_len - 1 - q) / kp.nq + 1 : 0;
  const int64_t nchunks = (kp.ntiles + kp.chunk - 1) / kp.chunk;
  if (q >= nchunks) return 0;
  const int64_t nc = (nchunks - 1 - q) / kp.nq + 1;
  int64_t len = nc * kp.chunk;
  if (q + (nc - 1) * kp.nq == nchunks - 1) len -= nchunks * kp.chunk - kp.ntiles;
  return len;
}

// Four-phase first pass of one image: the tiles fall into four groups by
// the parity of their row and column, group g holding rows of parity g >> 1
// and columns of parity g & 1, and position i of the pass goes to the
// groups one after the other, each in raster order.  No two tiles of a group
// touch, so tiles that run at the same time are seldom neighbours (each
// would otherwise load the other's border before it changes and ask for a
// re-visit).  The groups go in the order 0, 1, 2, 3, or with `diag` in the
// order 0, 3, 1, 2: the two diagonal groups first, so that every tile of the
// last two groups, half the image, starts with all four edge neighbours
// finished.
__device__ __forceinline__ uint32_t phase_tile(uint32_t tx, uint32_t ty, uint32_t i, bool diag) {
  const uint32_t ex = (tx + 1) / 2, ox = tx / 2, ey = (ty + 1) / 2, oy = ty / 2;
  auto size = [&](int g) { return ((g >> 1) ? oy : ey) * ((g & 1) ? ox : ex); };
  const int g1 = diag ? 3 : 1, g2 = diag ? 1 : 2, g3 = diag ? 2 : 3;
  // the group sizes, compared one after the other (no indexed array: that
  // would live in scratch memory)
  int p = 0;
  if (i >= size(0)) {
    i -= size(0);
    p = g1;
    if (i >= size(g1)) {
      i -= size(g1);
      p = g2;
      if (i >= size(g2)) {
        i -= size(g2);
        p = g3;
      }
    }
  }
  const uint32_t w = (p & 1) ? ox : ex;
  return (2 * (i / w) + (p >> 1)) * tx + 2 * (i % w) + (p & 1);
}

__device__ __forceinline__ int64_t first_pass_tile(const KParams& kp, const DevImage* imgs,
                                                   int q, int64_t i) {
  if (kp.list_mode) return kp.list_in[i * kp.nq + q];
  const uint32_t ii = (uint32_t)i, ch = (uint32_t)kp.chunk;
  const uint32_t c = (ii / ch) * (uint32_t)kp.nq + (uint32_t)q;
  const uint32_t t = c * ch + ii % ch;
  if (kp.phase_tx > 0)
    return phase_tile((uint32_t)kp.phase_tx, (uint32_t)kp.phase_ty, t, kp.phase_diag != 0);
  if (kp.phase_tx < 0) {
    // a batch: the pass covers the images one after the other (tile ids),
    // each in its own four phases
    const DevImage& im = imgs[kp.tile_img[t]];
    return im.tile_base + phase_tile((uint32_t)im.tiles_x, (uint32_t)im.tiles_y,
                                     t - (uint32_t)im.tile_base, kp.phase_diag != 0);
  }
  if (kp.order_mul == 1 && kp.order_add == 0) return t;
  return (int64_t)(((uint64_t)t * kp.order_mul + kp.order_add) % (uint64_t)kp.ntiles);
}

__device__ __forceinline__ int* ring_slot(int* queue, const KParams& kp, int q, int64_t pos,
                                          int64_t len) {
  return &queue[(int64_t)q * kp.qcap + (pos - len) % (int64_t)kp.qcap];
}

// No more work: tell every waiter.  Executed by a whole wavefront.
static __device__ void stop_all(DevCtl* ctl, int* queue, const KParams& kp, int grid) {
  __hip_atomic_store(&ctl->done.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int q = 0; q < kp.nq; ++q) {
    const int64_t len = first_pass_len(kp, q);
    const int64_t h = ld_rlx_u32(&ctl->head[q].v);
    int64_t t = ld_rlx_u32(&ctl->tail[q].v);
    if (t < len) t = len;
    // waiters hold tickets in [tail, head); a worker that passed the `done`
    // check but has not taken its ticket yet lands within `grid` more
    const int64_t hi = (h > t ? h : t) + grid;
    for (int64_t pos = t + threadIdx.x; pos < hi; pos += 64)
      __hip_atomic_store(ring_slot(queue, kp, q, pos, len), kSlotStop, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

static __device__ void abort_launch(DevCtl* ctl, int* queue, const KParams& kp, int grid, int bits) {
  atomicOr((int*)&ctl->status.v, bits | ST_ABORT);
  __hip_atomic_store(&ctl->done.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int q = 0; q < kp.nq; ++q) {  // one lane: this path only ends a failed launch
    const int64_t len = first_pass_len(kp, q);
    const int64_t h = ld_rlx_u32(&ctl->head[q].v);
    int64_t t = ld_rlx_u32(&ctl->tail[q].v);
    if (t < len) t = len;
    const int64_t hi = (h > t ? h : t) + grid;
    for (int64_t pos = t; pos < hi; ++pos)
      __hip_atomic_store(ring_slot(queue, kp, q, pos, len), kSlotStop, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Per-worker state of the queue protocol.
//  - First pass: the positions of queue q's first pass are taken in chunks
//    of kFpChunk positions, one ticket (an atomic on the queue's first-pass
//    head) per chunk, and the next chunk's ticket is taken when the last
//    position of the current one is, so its round trip overlaps a visit.
//    With m workers serving the queue, ticket h holds positions
//    (h / m) m K + h % m + j m, j < K: the workers that took neighbouring
//    tickets walk neighbouring positions in step, so the tiles in flight at
//    one time stay a compact band of the pass's order (as one ticket per
//    position would keep them), while there is one atomic per K positions.
//    Tickets keep the first pass dynamic: a worker that is not resident yet
//    (other work on the device) holds no positions.
//  - Ring tickets (re-activated tiles) come from the ring head, which starts
//    at the first pass's length.
//  - Pending count: a release of a tile is not taken off the launch's
//    pending count at once.  It becomes this worker's credit, which covers
//    the next tile it activates; the rest is taken off only when the worker
//    is about to wait for work.  The count then never falls below the number
//    of tiles queued or running (a tile is counted before it is queued), and
//    it reaches zero exactly when every worker waits with no credit left: the
//    worker whose subtraction brings it there ends the launch.  A visit thus
//    touches the one pending word only when it activates more tiles than its
//    credit covers, instead of on every visit (a single hot word serialises
//    its atomics device-wide).
constexpr uint32_t kNoTicket = 0xFFFFFFFFu;
constexpr int kLaunchDone = -2;  // take_tile: this worker's credit ended the launch
constexpr uint32_t kFpChunk = 8;

struct QState {
  uint32_t fp_next, fp_left;  // lane 0: next position of the current chunk, positions left
  uint32_t fp_step;           // workers serving the queue (m)
  uint32_t fp_pre;            // lane 0: the next chunk's ticket, taken ahead, or kNoTicket
  bool fp_done;              // lane 0: the queue's first pass has no chunk left
  uint32_t pre;              // lane 0: a ring ticket taken ahead of time, or kNoTicket
  uint32_t credit;           // wave-uniform: releases not yet taken off the pending count
  bool backlog;              // lane 0: its last ring slot was already filled when it looked
};

__device__ __forceinline__ QState init_qstate(const KParams& kp, int grid) {
  QState s;
  const int q = blockIdx.x % kp.nq;
  s.fp_next = s.fp_left = 0;
  s.fp_step = (uint32_t)((grid - q + kp.nq - 1) / kp.nq);
  s.fp_pre = kNoTicket;
  s.fp_done = false;
  s.pre = kNoTicket;
  s.credit = 0;
  s.backlog = false;
  return s;
}

// Take a ticket of queue head *p (one lane).  The compiler combines the lanes
// of an atomic with a wavefront-uniform address into one atomic and waits
// for its result at once, to hand each lane its share; an address offset
// that it cannot prove uniform (a zero written by an asm move) keeps the
// plain atomic, whose round trip then overlaps the work before the ticket
// is used.
__device__ __forceinline__ uint32_t take_ticket(uint32_t* p) {
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return atomicAdd(p + z, 1u);
}

// Lane 0: this worker's next position in queue q's first pass (of length
// len), or -1 once the first pass has none left.
__device__ __forceinline__ int64_t next_first_pass(DevCtl* ctl, int q, int64_t len, QState& qs) {
  if (qs.fp_left == 0 || qs.fp_next >= len) {
    if (qs.fp_done) return -1;
    const uint32_t h = qs.fp_pre != kNoTicket ? qs.fp_pre : take_ticket(&ctl->fphead[q].v);
    qs.fp_pre = kNoTicket;
    const uint32_t m = qs.fp_step;
    const int64_t a = (int64_t)(h / m) * m * kFpChunk + h % m;
    if (a >= len) {
      qs.fp_done = true;
      return -1;
    }
    qs.fp_next = (uint32_t)a;
    qs.fp_left = kFpChunk;
  }
  const int64_t pos = qs.fp_next;
  qs.fp_next += qs.fp_step;
  qs.fp_left--;
  return pos;
}

// Lane 0, after next_first_pass: once this worker's chunk is used up, the
// ticket of its next chunk is taken ahead (its round trip then overlaps a
// visit).  A separate step, so that callers can issue it after the
// arithmetic that maps the position to a tile.
__device__ __forceinline__ void refill_first_pass(DevCtl* ctl, int q, int64_t len, QState& qs) {
  if ((qs.fp_left == 0 || qs.fp_next >= len) && qs.fp_pre == kNoTicket && !qs.fp_done)
    qs.fp_pre = take_ticket(&ctl->fphead[q].v);
}

// Lane 0: the next tile of queue q for this worker, -1 when the launch is
// over, or kLaunchDone when this worker's credit brought the pending count
// to zero (the caller then ends the launch).  `first_pass` tells whether it
// came from the first pass; `ready` whether it did not wait; `vbits` holds
// the tile's first-visit bit (bit 0) and whether the packed side columns of
// the tiles on either side are written (bits 1, 2).  Waits use relaxed
// loads only: an acquire on gfx950 invalidates the L2 of the XCD, which a
// waiting worker must not do to the tiles others are working on.
static __device__ __forceinline__ int take_tile(DevCtl* ctl, int* queue, const KParams& kp,
                                                uint32_t* state, const uint8_t* visited,
                                                const DevImage* imgs, int q, int grid,
                                                QState& qs, bool& first_pass, bool& ready,
                                                int& vbits) {
  const int64_t len = first_pass_len(kp, q);
  first_pass = false;
  ready = false;
  vbits = 0;
  int v;
  const int64_t pos = qs.pre == kNoTicket ? next_first_pass(ctl, q, len, qs) : -1;
  if (pos >= 0) {
    first_pass = ready = true;
    v = (int)first_pass_tile(kp, imgs, q, pos);
    refill_first_pass(ctl, q, len, qs);
  } else {
    uint32_t h = qs.pre;
    qs.pre = kNoTicket;
    if (h == kNoTicket) {
      if (ld_rlx_u32(&ctl->done.v)) return -1;
      h = take_ticket(&ctl->head[q].v);
    }
    int* slot = ring_slot(queue, kp, q, h, len);
    uint32_t nap = 1;
    for (uint32_t w = 0;; ++w) {
      v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v >= 0) {
        ready = w == 0;
        break;
      }
      if (v == kSlotStop) return -1;
      if (w == 0 && qs.credit) {
        // about to wait: this worker's releases come off the pending count
        const uint32_t c = qs.credit;
        qs.credit = 0;
        if (atomicSub(&ctl->pending.v, c) == c) return kLaunchDone;
      }
      if ((w & 63) == 63 && ld_rlx_u32(&ctl->done.v)) return -1;
      if (w > kp.spin_limit) {
        abort_launch(ctl, queue, kp, grid, ST_INTERNAL);
        return -1;
      }
      for (uint32_t k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(2);
      if (nap < 16) nap <<= 1;
    }
    __hip_atomic_store(slot, kSlotEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (kp.max_visits > 0) {
    const uint32_t nv = atomicAdd(&ctl->visits_cap.v, 1u);
    if ((int64_t)nv >= kp.max_visits) {
      abort_launch(ctl, queue, kp, grid, ST_INCOMPLETE);
      return -1;
    }
  }
  // pending -> running.  A neighbour that asked for this visit finished its
  // marker stores before its request reached the state word, so once the
  // exchange is complete, the marker reads that follow see them.  The
  // visited flags of the tile (written by its last owner before it released
  // it) and of the tiles on either side (whether their packed side columns
  // are written yet) are read in the same round trip.
  __hip_atomic_exchange(&state[v], TS_RUNNING, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint8_t seen = ld_coherent(&visited[v]);
  uint8_t sl = 0, sr = 0;
  if (kp.colJ) {
    if (v > 0) sl = ld_coherent(&visited[v - 1]);
    if (v + 1 < kp.ntiles) sr = ld_coherent(&visited[v + 1]);
  }
  drain_memory();
  vbits = (seen == 0 ? 1 : 0) | (sl ? 2 : 0) | (sr ? 4 : 0);
  return v;
}

// Whole wavefront: take the next tile (lane 0 does the work; the result,
// the flags and the credit are broadcast).  Returns the tile, -1 when the
// launch is over (after ending it, if this worker's credit did).
static __device__ __forceinline__ int next_tile(DevCtl* ctl, int* queue, const KParams& kp,
                                                uint32_t* state, const uint8_t* visited,
                                                const DevImage* imgs, int q, int grid,
                                                QState& qs, bool& first_pass, int& vbits) {
  int t = 0, fp = 0, fv = 0;
  if (threadIdx.x == 0) {
    bool f = false, ready = false;
    t = take_tile(ctl, queue, kp, state, visited, imgs, q, grid, qs, f, ready, fv);
    qs.backlog = !f && ready;
    fp = f ? 1 : 0;
  }
  t = __builtin_amdgcn_readfirstlane(t);
  qs.credit = __builtin_amdgcn_readfirstlane(qs.credit);
  first_pass = __builtin_amdgcn_readfirstlane(fp) != 0;
  vbits = __builtin_amdgcn_readfirstlane(fv);
  if (t == kLaunchDone) {
    stop_all(ctl, queue, kp, grid);
    return -1;
  }
  return t;
}

// Mid-visit requests.  peek_request() reads the state word of the tile a
// wavefront is visiting (lane 0; the result is used later, so the read's
// round trip overlaps work); take_request() with that value returns true if
// a neighbour asked for the tile since it was taken.  The request is then
// consumed (pending -> running, as when a tile is taken) and, once the
// exchange is complete, the neighbour's marker stores are visible, so the
// caller re-reads its halo and goes on.  A request that lands after the
// read is seen by the release at the end of the visit as before.
__device__ __forceinline__ uint32_t peek_request(const uint32_t* word) {
  uint32_t v = 0;
  if (threadIdx.x == 0) v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}
__device__ __forceinline__ bool take_request(uint32_t* word, uint32_t peeked) {
  const uint32_t v = __builtin_amdgcn_readfirstlane(peeked);
  if (!(v & TS_PENDING)) return false;
  if (threadIdx.x == 0)
    __hip_atomic_exchange(word, TS_RUNNING, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  drain_memory();
  return true;
}

// Gray-level bands: remember that tile t has work of class c for a later
// launch (one lane; its class is already recorded).  The tile enters the
// next launch's list once.
static __device__ void defer_tile(DevCtl* ctl, const KParams& kp, int t, int c) {
  if (atomicExch(&kp.listed[t], 1u) == 0u) {
    const uint32_t i = atomicAdd(&ctl->next_len.v, 1u);
    __hip_atomic_store(&kp.list_out[i], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  atomicMax((int*)&ctl->max_deferred.v, c);
}

// Once this worker's share of the first pass is done: if its last ring slot
// was already filled when it looked (a backlog), the next ring ticket is
// taken before the current tile is solved, so its round trip overlaps useful
// work (lane 0).  Decided without reading anything: a read here would stall
// the wavefront before its solve.  A ticket taken after the launch ended
// still returns: the slot wait checks the done flag.
static __device__ __forceinline__ void prefetch_ring_ticket(DevCtl* ctl, const KParams& kp, int q,
                                                            QState& qs) {
  if (qs.pre == kNoTicket && qs.backlog && qs.fp_done) qs.pre = take_ticket(&ctl->head[q].v);
}

// Lane d < 9: the neighbour tile in direction d (3 x 3 grid index) of tile
// (ty, tx) of image im if `act` asks for it, else -1 (every other lane -1).
__device__ __forceinline__ int neighbour_request(const DevImage& im, int64_t ty, int64_t tx,
                                                 uint32_t act) {
  const int d = threadIdx.x;
  int n = -1;
  if (d < 9 && ((act >> d) & 1u)) {
    const int64_t ny = ty + d / 3 - 1, nx = tx + d % 3 - 1;
    if (ny >= 0 && ny < im.tiles_y && nx >= 0 && nx < im.tiles_x)
      n = (int)(im.tile_base + ny * im.tiles_x + nx);
  }
  return n;
}

// Publish the end of a visit of tile t (whole wavefront, once the tile's
// marker write-back is complete).  Lanes 0..8 ask the neighbours they name
// in `n` (neighbour_request) for a visit while lane 9 tries to release t
// (one round trip).  A release
// adds to the worker's credit (QState); the neighbours that were idle are
// covered by that credit, and only what it does not cover is added to the
// pending count, together with their queue reservations (a second round
// trip, only when there are such neighbours).  The queue slots are filled
// once both have landed, so a queued tile is always already counted.
// Returns 1 if t must be run again (a neighbour asked while it ran), else 0.
// With `release` false (a visit that publishes its border and goes on) t
// stays running and only the requests go out.  With `requeue`, a tile that a
// neighbour asked for while it ran goes back on its queue instead of being
// run again by this worker (it stays counted as pending, and its state word
// keeps the request until the next owner takes it).
static __device__ __forceinline__ int publish_requests(DevCtl* ctl, int* queue,
                                                       const KParams& kp, uint32_t* state,
                                                       int t, int n, int cls, WorkerStats& ws,
                                                       uint32_t& credit, bool release,
                                                       bool requeue) {
  const int d = threadIdx.x;
  bool fresh = false;  // was idle: this wavefront enqueues it
  bool released = false;
  bool again = false;  // lane 9: t goes back on its queue
  if (n >= 0) {
    // with bands every request records its class on the tile, so that a
    // listed tile whose first-pass visit is still ahead knows it has work
    // at this band; below the band a later launch takes it
    if (kp.band >= 0) atomicMax(&kp.dclass[n], cls);
    if (kp.band >= 0 && cls < kp.band)
      defer_tile(ctl, kp, n, cls);
    else
      fresh = __hip_atomic_fetch_or(&state[n], TS_PENDING, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) == 0u;
  }
  if (d == 9 && release) {
    uint32_t expect = TS_RUNNING;
    released = __hip_atomic_compare_exchange_strong(
        &state[t], &expect, 0u, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!released && requeue) {
      again = true;
      n = t;
    }
  }
  const int nfresh = __popcll(__ballot(fresh));
  const bool rel = __ballot(released) != 0;
  const bool req = __ballot(again) != 0;
  // count the new tiles (what the credit does not cover) and reserve their
  // queue positions
  uint32_t cr = credit + (rel ? 1u : 0u);
  uint32_t add = 0;
  if ((uint32_t)nfresh > cr) {
    add = (uint32_t)nfresh - cr;
    cr = 0;
  } else {
    cr -= (uint32_t)nfresh;
  }
  credit = cr;
  if (d == 0 && add) atomicAdd(&ctl->pending.v, add);
  uint32_t pos = 0;
  int q = 0;
  if (fresh || again) {
    q = queue_of(kp, n);
    pos = atomicAdd(&ctl->tail[q].v, 1u);
  }
  // the count has landed before any slot is filled
  if (add) drain_memory();
  int res = 0;
  if (fresh || again)
    __hip_atomic_store(ring_slot(queue, kp, q, pos, first_pass_len(kp, q)), n, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  ws.requeued += nfresh + (req ? 1 : 0);
  if (req) ws.reproc++;
  if (release && !rel && !req) {
    // running | pending: take the request and run again (the failed release
    // already saw the request, so the halo reads that follow see the
    // neighbour's new border)
    if (d == 0)
      __hip_atomic_exchange(&state[t], TS_RUNNING, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    drain_memory();
    ws.reproc++;
    ws.visits++;
    res = 1;
  }
  return res;
}

// publish() for the requests of mask `act` of tile (ty, tx).
static __device__ __forceinline__ int publish(DevCtl* ctl, int* queue, const KParams& kp, uint32_t* state, int t,
                       const DevImage& im, int64_t ty, int64_t tx, uint32_t act, int cls,
                       WorkerStats& ws, uint32_t& credit, bool release = true,
                       bool requeue = false) {
  return publish_requests(ctl, queue, kp, state, t, neighbour_request(im, ty, tx, act), cls, ws,
                          credit, release, requeue);
}

// Geometry of tile t: its image and the origin of the tile in it.
struct TilePos {
  DevImage im;
  int64_t ty, tx, y0, x0;
};
template <int TH>
__device__ __forceinline__ TilePos tile_pos(const DevImage& one, const DevImage* imgs,
                                            const KParams& kp, int t) {
  TilePos p;
  // two plain assignments: a select between the two sources would make the
  // compiler copy `one` to scratch and read either through a flat pointer
  if (imgs)
    p.im = imgs[image_of(kp, imgs, t)];
  else
    p.im = one;
  const int64_t tl = (int64_t)t - p.im.tile_base;
  p.ty = tl / p.im.tiles_x;
  p.tx = tl % p.im.tiles_x;
  p.y0 = p.ty * TH;
  p.x0 = p.tx * TW;
  return p;
}

// The persistent worker of a tile policy that prefetches (TP::kPrefetch).
// Along its share of the first pass a worker keeps three tiles in flight:
// the tile t it solves; the next tile n, whose loads it issues into
// registers once t is solved and its activation mask taken, before t is
// written back, so that their round trip overlaps the write-back (for int32
// tiles the loads and stores together stay within the 63 memory operations
// a wavefront can have outstanding; a tile at the image edge is loaded at
// its visit instead, see Tile::prefetchable); and the
// tile after n, whose state word goes pending -> running (its flags read in
// the same round trip) right after t's solve.  t is published only after
// n's solve: by then its stores have completed, and the drain before the
// publication costs nothing.  A tile that a neighbour asks for while it
// runs (or waits for its publication) goes back on its queue (the registers
// already hold the next tile) instead of being run again in place.  Only
// plain launches use it: no gray-level bands, no visit limit.
template <typename TP>
__device__ __forceinline__ void prefetch_worker(DevImage one, const DevImage* __restrict__ imgs,
                                                const KParams& kp, DevCtl* ctl, int* queue,
                                                uint32_t* state, uint8_t* visited) {
  constexpr int TH = TP::kTH;
  __shared__ typename TP::L s;
  const bool lead = threadIdx.x == 0;
  const int q = blockIdx.x % kp.nq;
  const int grid = gridDim.x;
  WorkerStats ws;
  typename TP::Pre P;
  QState qs = init_qstate(kp, grid);
  const int64_t fp_len = first_pass_len(kp, q);
  // Lead: the tile after the next one, if this worker's share of the first
  // pass has one (-1 otherwise): its state word goes pending -> running and
  // its flags are read now, and the results are used after the next solve.
  // Taken right after the drain that follows a solve, when no memory
  // operation is outstanding, so that nothing in here waits for one (a
  // register hazard in its index arithmetic would otherwise wait for all of
  // them); its round trip overlaps the publication that follows.  The first
  // call of a run is made once that run's first tile has been issued.
  int nx = -1;
  uint8_t f0 = 0, f1 = 0, f2 = 0;
  uint32_t ended = 0;  // the launch was stopped (an abort): take no next tile
  auto take_next = [&]() {
    nx = -1;
    f0 = f1 = f2 = 0;
    ended = 0;
    if (lead) {
      // the arithmetic first, then the memory operations
      const int64_t pos = qs.pre == kNoTicket ? next_first_pass(ctl, q, fp_len, qs) : -1;
      if (pos >= 0) nx = (int)first_pass_tile(kp, imgs, q, pos);
      ended = ld_rlx_u32(&ctl->done.v);
      if (pos >= 0) {
        refill_first_pass(ctl, q, fp_len, qs);
        __hip_atomic_exchange(&state[nx], TS_RUNNING, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        f0 = ld_coherent(&visited[nx]);
        if (kp.colJ) {
          if (nx > 0) f1 = ld_coherent(&visited[nx - 1]);
          if (nx + 1 < kp.ntiles) f2 = ld_coherent(&visited[nx + 1]);
        }
      } else {
        prefetch_ring_ticket(ctl, kp, q, qs);
      }
    }
  };
  // Outer loop: take a tile the plain way (this worker's share of the first
  // pass is done, or a ring ticket was taken ahead); its visit loads it.
  // Inner loop: visit it; while the first pass has a next position for this
  // worker, that tile's loads are issued once the current tile is solved,
  // and its visit follows.  The registers of the next tile are written on
  // every path into the write-back (zeros when there is none), so the
  // compiler never keeps them live across a solve.
  // A first-pass tile the inner loop could not prefetch (see
  // Tile::prefetchable) comes back here as `carry` with its flags; the tile
  // after it is already taken (nx).
  int carry = -1, carry_fv = 0;
  for (;;) {
    uint32_t c0 = (uint32_t)now();
    bool first_pass = false;
    int fv = 0;
    int t;
    const bool carried = carry >= 0;
    if (carried) {
      t = carry;
      fv = carry_fv;
      carry = -1;
    } else {
      t = next_tile(ctl, queue, kp, state, visited, imgs, q, grid, qs, first_pass, fv);
      if (t < 0) break;
    }
    TilePos tp = tile_pos<TH>(one, imgs, kp, t);
    // a re-visit stages its seams (load_seam); anything else is issued into
    // the registers and committed at once
    bool seam = false;
    if constexpr (TP::kSeamVisits) seam = !(fv & 1) && kp.colJ;
    if (!seam) TP::issue(P, tp.im, tp.y0, tp.x0, kp, t, tp.tx, fv >> 1);
    if (!carried) take_next();  // the tile after t
    // the tile written back before this one, awaiting its publication
    // (dt < 0: none): its neighbour requests (lanes 0..8) and whether it was
    // a first visit
    int dt = -1, dn = -1;
    bool dfirst = false;
    for (;;) {
      uint32_t c1 = (uint32_t)now();
      ws.t_idle += c1 - c0;
      ws.visits++;
      const bool first = (fv & 1) != 0;
      const int sides = fv >> 1;
      bool viol = false;
      if (seam)
        TP::load_seam(s, tp.im, tp.y0, tp.x0, kp, t, tp.tx, sides);
      else
        viol = TP::commit(s, P, first, kp);
      uint32_t c2 = (uint32_t)now();
      ws.t_load += c2 - c1;
      VisitStats vs;
      bool hit = false;
      TP::template solve<TP::kSeamVisits>(s, tp.y0, tp.x0, kp.sweeps, !first, kp.seed_queue_max,
                                          kp.queue_waves, kp.spin_limit, vs, hit, &state[t],
                                          tp.im, kp, t, tp.tx, sides, false, false);
      uint32_t c3 = (uint32_t)now();
      ws.t_solve += c3 - c2;
      // the previous tile's write-back had this solve to complete, and the
      // next tile's exchange and flag reads are complete before its loads
      // are issued (as at a pop)
      drain_memory();
      int nt = __builtin_amdgcn_readfirstlane(nx);
      if (__builtin_amdgcn_readfirstlane(ended)) nt = -1;
      int nfv = 0;
      if (nt >= 0) {
        nfv = __builtin_amdgcn_readfirstlane((f0 == 0 ? 1 : 0) | (f1 ? 2 : 0) | (f2 ? 4 : 0));
        take_next();  // the tile after nt
      }
      if (dt >= 0) {
        if (lead && dfirst) st_coherent(&visited[dt], (uint8_t)1);
        publish_requests(ctl, queue, kp, state, dt, dn, 0, ws, qs.credit, true, true);
      }
      uint32_t c4 = (uint32_t)now();
      ws.t_sync += c4 - c3;
      // the activation mask reads the tile before its stores are issued
      int amax = 0;
      const uint32_t act = TP::activation_mask(s, tp.y0, tp.x0, false, amax);
      TilePos np = tp;
      bool nissued = false;
      if (nt >= 0) {
        np = tile_pos<TH>(one, imgs, kp, nt);
        nissued = TP::prefetchable(np.im, np.y0, np.x0);
      }
      if (nissued)
        TP::issue_prefetch(P, np.im, np.y0, np.x0, kp, nt, np.tx, nfv >> 1);
      else
        TP::clear_pre(P);
      TP::store(s, tp.im, tp.y0, tp.x0, kp, t, first);
      const int n = neighbour_request(tp.im, tp.ty, tp.tx, act);
      c0 = (uint32_t)now();
      ws.t_store += c0 - c4;
      ws.add(vs);
      if (lead) {
        if (viol) atomicOr((int*)&ctl->status.v, ST_MARKER_GT_MASK);
        if (hit) abort_launch(ctl, queue, kp, grid, ST_INTERNAL);
      }
      if (!nissued) {
        // no next tile, or one the outer loop loads: publish this one now
        // (its write-back and packed side columns complete first)
        drain_memory();
        if (lead && first) st_coherent(&visited[t], (uint8_t)1);
        publish_requests(ctl, queue, kp, state, t, n, 0, ws, qs.credit, true, true);
        uint32_t c5 = (uint32_t)now();
        ws.t_sync += c5 - c0;
        c0 = c5;
        if (nt >= 0) {
          carry = nt;
          carry_fv = nfv;
        }
        break;
      }
      dt = t;
      dn = n;
      dfirst = first;
      t = nt;
      fv = nfv;
      tp = np;
      seam = false;
    }
  }
  if (lead) ws.flush(ctl);
}

// The body of a persistent tile worker, for any tile policy TP (the
// reconstruction tile, the distance-transform tile): take tiles from the
// queues, load, solve, write back, publish, until the launch ends.
template <typename TP>
__device__ __forceinline__ void persistent_worker(DevImage one, const DevImage* __restrict__ imgs,
                                                  KParams kp, DevCtl* ctl, int* queue,
                                                  uint32_t* state, uint8_t* visited) {
  constexpr int TH = TP::kTH;
  __shared__ typename TP::L s;
  const bool lead = threadIdx.x == 0;
  const int q = blockIdx.x % kp.nq;
  const int grid = gridDim.x;
  WorkerStats ws;
  QState qs = init_qstate(kp, grid);
  for (;;) {
    uint32_t c0 = (uint32_t)now();
    bool fp = false;
    int fv = 0;
    const int t = next_tile(ctl, queue, kp, state, visited, imgs, q, grid, qs, fp, fv);
    uint32_t c1 = (uint32_t)now();
    ws.t_idle += c1 - c0;
    if (t < 0) break;
    const TilePos tp = tile_pos<TH>(one, imgs, kp, t);
    const DevImage& im = tp.im;
    const int64_t ty = tp.ty, tx = tp.tx, y0 = tp.y0, x0 = tp.x0;
    if (kp.band >= 0) {
      // gray-level bands: this visit takes the tile's deferred work (the
      // halo it loads holds it).  A list entry with nothing at or above the
      // band goes back to the next launch's list without a visit.
      int dc = -1;
      if (lead)
        dc = __hip_atomic_exchange(&kp.dclass[t], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      dc = __builtin_amdgcn_readfirstlane(dc);
      if (kp.list_mode && fp && dc < kp.band) {
        if (lead && dc >= 0) {
          atomicMax(&kp.dclass[t], dc);
          defer_tile(ctl, kp, t, dc);
        }
        drain_memory();
        const int res = publish(ctl, queue, kp, state, t, im, ty, tx, 0u, 0, ws, qs.credit);
        if (res != 1) continue;
        ws.visits--;  // a neighbour asked for the tile meanwhile: visit it after all
      }
    }
    ws.visits++;
    const bool first = (fv & 1) != 0;
    // packed side columns of the left / right neighbour are written (bit 0 / 1)
    const int sides = fv >> 1;
    VisitStats vs;
    bool hit = false;
    const bool viol = TP::load(s, im, y0, x0, first, kp, t, tx, sides);
    uint32_t c2 = (uint32_t)now();
    ws.t_load += c2 - c1;
    if (lead) prefetch_ring_ticket(ctl, kp, q, qs);
    // one solve and one publication site: a visit may go round this loop
    // after publishing its border early (streaming tiles) or after a
    // release that found a neighbour's request (re-run with the new halo)
    bool seeded = !first, resume = false, early = TP::kStreaming;
    uint32_t c3 = c2;
    for (;;) {
      const bool more = TP::solve(s, y0, x0, kp.sweeps, seeded, kp.seed_queue_max,
                                  kp.queue_waves, kp.spin_limit, vs, hit, &state[t], im, kp, t,
                                  tx, sides, resume, early);
      uint32_t c3a = (uint32_t)now();
      ws.t_solve += c3a - c3;
      TP::store(s, im, y0, x0, kp, t, first);
      int amax = 0;
      const uint32_t act = TP::activation_mask(s, y0, x0, kp.band >= 0, amax);
      int cls = 0;
      if (kp.band >= 0) {
        cls = (amax - kp.band_base) >> kp.band_shift;
        if (cls < 0) cls = 0;
      }
      uint32_t c3b = (uint32_t)now();
      ws.t_store += c3b - c3a;
      ws.add(vs);
      vs = VisitStats();
      if (lead) {
        if (viol) atomicOr((int*)&ctl->status.v, ST_MARKER_GT_MASK);
        if (hit) abort_launch(ctl, queue, kp, grid, ST_INTERNAL);
      }
      hit = false;
      // the write-back is complete before anyone is told about it
      drain_memory();
      // ... and, with it, this tile's packed side columns: only now may a
      // neighbour see the visited flag and read them
      if (lead && first) st_coherent(&visited[t], (uint8_t)1);
      // with `more` the border raised a neighbour before the tile's fixed
      // point: the requests go out now and the rounds go on
      const bool release = !(TP::kStreaming && more);
      const int res =
          publish(ctl, queue, kp, state, t, im, ty, tx, act, cls, ws, qs.credit, release);
      uint32_t c4 = (uint32_t)now();
      ws.t_sync += c4 - c3b;
      c3 = c4;
      if constexpr (TP::kStreaming) {
        if (!release) {
          TP::clear_dirty(s);
          TP::snapshot_border(s);
          wsync();
          seeded = false;
          resume = true;
          early = false;
          continue;
        }
      }
      if (res != 1) break;
      // a neighbour changed while this tile ran: reload the halo, continue
      TP::reload_halo(s, im, y0, x0, kp, t, tx, sides);
      c3 = (uint32_t)now();
      ws.t_load += c3 - c4;
      seeded = true;
      resume = false;
      early = TP::kStreaming;
    }
  }
  if (lead) ws.flush(ctl);
}

}  // namespace iwpp
