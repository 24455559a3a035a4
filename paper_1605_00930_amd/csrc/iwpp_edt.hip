// iwpp_edt.hip -- Euclidean distance transform as an irregular wavefront
// propagation (IWPP chapter, "Transformada de Distancia Euclidiana", the
// distance-transform algorithm in IWPP form), on the same persistent tile
// queue as the reconstruction.
//
// Method: every background pixel (value 0) is its own site; every object
// pixel starts with no site.  A pixel q takes the site of a neighbour p
// whenever that site is strictly closer to q than q's own site (squared
// Euclidean distance), until no pixel changes.  The distance map is then the
// distance from each pixel to its site.  Like the paper's algorithm this is
// the vector-propagation approximation of the exact transform: a pixel's
// site is the best among the sites its neighbours hold, so a few pixels can
// end a fraction of a pixel farther than the exact nearest background pixel.
//
// GPU mapping: one 64-lane wavefront per 64 x 32 tile, as for the
// reconstruction.  Sites (packed y << 16 | x) and their squared distances
// are staged in LDS; rounds of four directional passes (down, up, right,
// left) offer each pixel the sites of the three pixels on the incoming side,
// the diagonal ones through DPP lane shifts, until a round changes nothing.
// A changed border site that is closer to a halo pixel than that pixel's own
// site activates the neighbouring tile.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "iwpp_device.h"
#include "iwpp_internal.h"

namespace iwpp {

namespace {

constexpr uint32_t kNoSite = 0xFFFFFFFFu;
constexpr uint32_t kFar = 0xFFFFFFFFu;  // distance of "no site"

__device__ __forceinline__ uint32_t pack_site(int64_t y, int64_t x) {
  return ((uint32_t)y << 16) | (uint32_t)x;
}

// Squared Euclidean distance from pixel (py, px) to site s.  Coordinates are
// below 2^15, so each square and the sum fit in 32 bits; "no site" is kFar.
__device__ __forceinline__ uint32_t dist2(int py, int px, uint32_t s) {
  const int dy = py - (int)(s >> 16), dx = px - (int)(s & 0xFFFFu);
  const uint32_t ay = (uint32_t)(dy < 0 ? -dy : dy), ax = (uint32_t)(dx < 0 ? -dx : dx);
  const uint32_t d = __umul24(ay, ay) + __umul24(ax, ax);
  return s == kNoSite ? kFar : d;
}

template <int TH>
struct EdtGeo {
  static constexpr int P = 67;  // odd pitch in words: one-lane-per-row passes are conflict free
  static constexpr int ROWS = TH + 2;
  static constexpr int RING = 2 * TW + 2 * (TH - 2);
  static constexpr int HALO = 2 * (TW + 2) + 2 * TH;
  __device__ static constexpr int at(int y, int x) { return (y + 1) * P + (x + 1); }
};

template <int TH>
struct EdtLds {
  using G = EdtGeo<TH>;
  uint32_t S[G::ROWS * G::P];  // sites of the tile and its halo
  uint32_t D[G::ROWS * G::P];  // squared distance of each tile pixel to its site
  uint32_t b_top[TW], b_bot[TW], b_left[TH], b_right[TH];  // border sites as loaded
  uint8_t rowdirty[TH];
};

template <int CONN, int TH>
struct EdtTile {
  using G = EdtGeo<TH>;
  using L = EdtLds<TH>;
  static constexpr int kTH = TH;
  static constexpr int B = 16;
  static_assert(TH == 32 || TH == 64, "one lane per row in the horizontal passes");

  __device__ static int lane() { return threadIdx.x; }

  // ---------------------------------------------------------- load / store
  // Stage the sites of the tile and its halo (coherent loads: neighbours on
  // other XCDs write them); pixels outside the image have no site.
  __device__ static bool load(L& s, const DevImage& im, int64_t y0, int64_t x0, bool,
                              const KParams&, int64_t, int64_t, int) {
    const gptr<const uint32_t> gS = (gptr<const uint32_t>)im.J;
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    for (int e = lane(); e < G::ROWS * (TW + 2); e += 64) {
      const int y = e / (TW + 2) - 1, x = e % (TW + 2) - 1;
      const int64_t gy = y0 + y, gx = x0 + x;
      uint32_t v = kNoSite;
      if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) v = ld_coherent(&gS[gy * im.ld + gx]);
      s.S[G::at(y, x)] = v;
    }
    wsync();
    // a tile pixel outside the image (ragged last tiles) gets distance 0, so
    // it never takes a site: it would change on every visit (it is never
    // written back) and re-activate its neighbours without end
    for (int e = lane(); e < TH * TW; e += 64) {
      const int y = e / TW, x = e % TW;
      const bool inside = y0 + y < im.H && x0 + x < im.W;
      s.D[G::at(y, x)] = inside ? dist2((int)(y0 + y), (int)(x0 + x), s.S[G::at(y, x)]) : 0u;
    }
    snapshot_border(s);
    wsync();
    return false;
  }

  __device__ static void snapshot_border(L& s) {
    s.b_top[lane()] = s.S[G::at(0, lane())];
    s.b_bot[lane()] = s.S[G::at(TH - 1, lane())];
    for (int y = lane(); y < TH; y += 64) {
      s.b_left[y] = s.S[G::at(y, 0)];
      s.b_right[y] = s.S[G::at(y, TW - 1)];
    }
  }

  __device__ __forceinline__ static void reload_halo(L& s, const DevImage& im, int64_t y0, int64_t x0,
                                     const KParams&, int64_t, int64_t, int) {
    const gptr<const uint32_t> gS = (gptr<const uint32_t>)im.J;
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    for (int e = lane(); e < G::HALO; e += 64) {
      int y, x;
      if (e < TW + 2) {
        y = -1;
        x = e - 1;
      } else if (e < 2 * (TW + 2)) {
        y = TH;
        x = e - (TW + 2) - 1;
      } else if (e < 2 * (TW + 2) + TH) {
        y = e - 2 * (TW + 2);
        x = -1;
      } else {
        y = e - 2 * (TW + 2) - TH;
        x = TW;
      }
      const int64_t gy = y0 + y, gx = x0 + x;
      if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W)
        s.S[G::at(y, x)] = ld_coherent(&gS[gy * im.ld + gx]);
    }
    wsync();
    snapshot_border(s);
    wsync();
  }

  __device__ __forceinline__ static void store(const L& s, const DevImage& im, int64_t y0, int64_t x0,
                               const KParams&, int64_t, bool) {
    const gptr<uint32_t> gS = (gptr<uint32_t>)im.J;
    const int64_t gx = x0 + lane();
    const bool col_in = gx < im.W;
    for (int g = 0; g < TH; g += 64) {
      unsigned long long rows = __ballot(g + lane() < TH && s.rowdirty[g + lane()]);
      while (rows) {
        const int y = g + __builtin_ctzll(rows);
        rows &= rows - 1;
        const int64_t gy = y0 + y;
        if (gy < im.H && col_in) st_coherent(&gS[gy * im.ld + gx], s.S[G::at(y, lane())]);
      }
    }
  }

  // ---------------------------------------------------------- passes
  // Offer site c to the pixel at (py, px) whose best so far is (bs, bd):
  // it wins only if strictly closer (the paper's propagation condition).
  __device__ static void offer(int py, int px, uint32_t c, uint32_t& bs, uint32_t& bd) {
    const uint32_t d = dist2(py, px, c);
    if (d < bd) {
      bd = d;
      bs = c;
    }
  }

  // Down (DIR = +1) or up (DIR = -1) pass, one lane per column.  Lane 0
  // takes its left diagonal from the halo column on the left and lane 63 its
  // right diagonal from the halo column on the right (`fprev`).
  template <int DIR>
  __device__ static void pass_vert(L& s, int64_t y0, int64_t x0, uint64_t& d0) {
    const int x = lane();
    const int px = (int)x0 + x;
    const int ys = DIR > 0 ? 0 : TH - 1;
    const int fx = x == 0 ? -1 : TW;
    uint32_t prev = s.S[G::at(ys - DIR, x)];
    uint32_t fprev = s.S[G::at(ys - DIR, fx)];
#pragma unroll 1
    for (int kb = 0; kb < TH; kb += B) {
      uint32_t ss[B], dd[B], ff[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int y = ys + DIR * (kb + k);
        ss[k] = s.S[G::at(y, x)];
        dd[k] = s.D[G::at(y, x)];
        if (CONN == 8) ff[k] = s.S[G::at(y, fx)];
      }
      bool changed = false;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int py = (int)y0 + ys + DIR * (kb + k);
        uint32_t bs = ss[k], bd = dd[k];
        offer(py, px, prev, bs, bd);
        if (CONN == 8) {
          offer(py, px, (uint32_t)__builtin_amdgcn_update_dpp((int)fprev, (int)prev, 0x138, 0xF,
                                                              0xF, false),
                bs, bd);
          offer(py, px, (uint32_t)__builtin_amdgcn_update_dpp((int)fprev, (int)prev, 0x130, 0xF,
                                                              0xF, false),
                bs, bd);
          fprev = ff[k];
        }
        changed = changed || bs != ss[k];
        ss[k] = bs;
        dd[k] = bd;
        prev = bs;
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int y = ys + DIR * (kb + k);
        s.S[G::at(y, x)] = ss[k];
        s.D[G::at(y, x)] = dd[k];
      }
      if (__ballot(changed)) {
        const int yb = DIR > 0 ? kb : TH - kb - B;
        d0 |= ((1ull << B) - 1) << yb;
      }
    }
  }

  // Right (DIR = +1) or left (DIR = -1) pass, one lane per row.  Lane 0
  // takes its upper diagonal from the halo row above, the last tile row its
  // lower one from the halo row below.  In 32-row tiles lanes 32..63 replay
  // the halo row below with distance 0, so they only hand its stored sites to
  // lane 31 and never change or write anything.
  template <int DIR>
  __device__ static void pass_horz(L& s, int64_t y0, int64_t x0, uint64_t& d0) {
    const bool live = lane() < TH;
    const int yc = live ? lane() : TH;
    const int py = (int)y0 + yc;
    const int xs = DIR > 0 ? 0 : TW - 1;
    const int fy = lane() == 0 ? -1 : TH;
    uint32_t prev = s.S[G::at(yc, xs - DIR)];
    uint32_t fprev = s.S[G::at(fy, xs - DIR)];
    bool dirty = false;
#pragma unroll 1
    for (int kb = 0; kb < TW; kb += B) {
      uint32_t ss[B], dd[B], ff[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int x = xs + DIR * (kb + k);
        ss[k] = s.S[G::at(yc, x)];
        dd[k] = live ? s.D[G::at(yc, x)] : 0u;
        if (CONN == 8) ff[k] = s.S[G::at(fy, x)];
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int px = (int)x0 + xs + DIR * (kb + k);
        uint32_t bs = ss[k], bd = dd[k];
        offer(py, px, prev, bs, bd);
        if (CONN == 8) {
          offer(py, px, (uint32_t)__builtin_amdgcn_update_dpp((int)fprev, (int)prev, 0x138, 0xF,
                                                              0xF, false),
                bs, bd);
          offer(py, px, (uint32_t)__builtin_amdgcn_update_dpp((int)fprev, (int)prev, 0x130, 0xF,
                                                              0xF, false),
                bs, bd);
          fprev = ff[k];
        }
        dirty = dirty || bs != ss[k];
        ss[k] = bs;
        dd[k] = bd;
        prev = bs;
      }
      if (live) {
#pragma unroll
        for (int k = 0; k < B; ++k) {
          const int x = xs + DIR * (kb + k);
          s.S[G::at(yc, x)] = ss[k];
          s.D[G::at(yc, x)] = dd[k];
        }
      }
    }
    d0 |= __ballot(live && dirty);
  }

  // Pass p of a round (0 down, 1 up, 2 right, 3 left); true if it changed
  // a pixel.  The rows it changed are marked in rowdirty.
  __device__ static bool run_pass(L& s, int64_t y0, int64_t x0, int p) {
    uint64_t d0 = 0;
    if (p == 0)
      pass_vert<+1>(s, y0, x0, d0);
    else if (p == 1)
      pass_vert<-1>(s, y0, x0, d0);
    else if (p == 2)
      pass_horz<+1>(s, y0, x0, d0);
    else
      pass_horz<-1>(s, y0, x0, d0);
    wsync();
    for (int y = lane(); y < TH; y += 64)
      if ((d0 >> y) & 1ull) s.rowdirty[y] = 1;
    return d0 != 0;
  }

  // No streaming publication and no prefetch of the next tile.
  static constexpr bool kStreaming = false;
  static constexpr bool kPrefetch = false;
  struct Pre {};
  __device__ static void issue(Pre&, const DevImage&, int64_t, int64_t, const KParams&, int64_t,
                               int64_t, int) {}
  __device__ static bool commit(L&, const Pre&, bool, const KParams&) { return false; }
  __device__ static void clear_pre(Pre&) {}
  static constexpr bool kSeamVisits = false;
  __device__ static void load_seam(L&, const DevImage&, int64_t, int64_t, const KParams&, int64_t,
                                   int64_t, int) {}

  // Rounds until one changes nothing: the tile is then at a fixed point of
  // the propagation for its halo (the reconstruction tile's scan-round and
  // queue parameters do not apply).
  template <bool SEAM = false>
  __device__ static bool solve(L& s, int64_t y0, int64_t x0, int, bool, int, uint32_t,
                               uint32_t iter_limit, VisitStats& vs, bool& hit_limit, uint32_t*,
                               const DevImage&, const KParams&, int64_t, int64_t, int, bool, bool) {
    // passes down, up, right, left, round after round, until four in a row
    // change nothing: those four saw the same tile in every direction
    int quiet = 0;
    for (uint32_t k = 0; quiet < 4; ++k) {
      if (run_pass(s, y0, x0, (int)(k & 3u)))
        quiet = 0;
      else
        ++quiet;
      if ((k & 3u) == 3u) vs.rounds++;
      if (k >= 4u * iter_limit) {
        hit_limit = true;
        return false;
      }
    }
    return false;
  }

  // Neighbour tiles (3x3 grid index) with a halo pixel to which a changed
  // border site is strictly closer than the halo pixel's own site.
  __device__ static void ring_pos(int e, int& y, int& x) {
    if (e < TW) {
      y = 0;
      x = e;
    } else if (e < 2 * TW) {
      y = TH - 1;
      x = e - TW;
    } else if (e < 2 * TW + TH - 2) {
      y = e - 2 * TW + 1;
      x = 0;
    } else {
      y = e - 2 * TW - (TH - 2) + 1;
      x = TW - 1;
    }
  }
  __device__ __forceinline__ static uint32_t activation_mask(const L& s, int64_t y0, int64_t x0, bool,
                                             int& amax) {
    amax = 0;  // no gray-level bands for distances
    uint32_t m = 0;
    for (int base = 0; base < G::RING; base += 64) {
      const int e = base + lane();
      if (e >= G::RING) continue;
      int y, x;
      ring_pos(e, y, x);
      const uint32_t v = s.S[G::at(y, x)];
      uint32_t v0;
      if (e < TW)
        v0 = s.b_top[x];
      else if (e < 2 * TW)
        v0 = s.b_bot[x];
      else if (e < 2 * TW + TH - 2)
        v0 = s.b_left[y];
      else
        v0 = s.b_right[y];
      if (v == v0) continue;
      for (int d = 0; d < 9; ++d) {
        const int dy = d / 3 - 1, dx = d % 3 - 1;
        if (d == 4 || (CONN == 4 && dy != 0 && dx != 0)) continue;
        const int hy = y + dy, hx = x + dx;
        const int cy = hy < 0 ? 0 : (hy >= TH ? 2 : 1);
        const int cx = hx < 0 ? 0 : (hx >= TW ? 2 : 1);
        if (cy == 1 && cx == 1) continue;
        const int py = (int)y0 + hy, px = (int)x0 + hx;
        if (dist2(py, px, v) < dist2(py, px, s.S[G::at(hy, hx)])) m |= 1u << (cy * 3 + cx);
      }
    }
    uint32_t all = 0;
    for (int d = 0; d < 9; ++d)
      if (__ballot((m >> d) & 1u)) all |= 1u << d;
    return all;
  }
};

template <int CONN, int TH>
__global__ __launch_bounds__(64) void k_persistent_edt(DevImage one,
                                                       const DevImage* __restrict__ imgs,
                                                       KParams kp, DevCtl* ctl, int* queue,
                                                       uint32_t* state, uint8_t* visited) {
  persistent_worker<EdtTile<CONN, TH>>(one, imgs, kp, ctl, queue, state, visited);
}

// Initial sites: a background pixel (0) is its own site, an object pixel has
// none (the initialisation phase of the distance-transform algorithm).
__global__ __launch_bounds__(256) void k_edt_init(uint32_t* __restrict__ sites, int64_t ld_out,
                                                  const uint8_t* __restrict__ img,
                                                  int64_t ld_img, int64_t H, int64_t W) {
  for (int64_t y = blockIdx.y; y < H; y += gridDim.y)
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < W;
         x += (int64_t)gridDim.x * 256)
      sites[y * ld_out + x] = img[y * ld_img + x] == 0 ? pack_site(y, x) : kNoSite;
}

// Distance map: squared distance of each pixel to its site, -1 where no
// site was found (an image without background).
__global__ __launch_bounds__(256) void k_edt_dist(int32_t* __restrict__ dist,
                                                  const uint32_t* __restrict__ sites,
                                                  int64_t ld_out, int64_t H, int64_t W) {
  for (int64_t y = blockIdx.y; y < H; y += gridDim.y)
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < W;
         x += (int64_t)gridDim.x * 256) {
      const uint32_t s = sites[y * ld_out + x];
      dist[y * ld_out + x] = s == kNoSite ? -1 : (int32_t)dist2((int)y, (int)x, s);
    }
}

dim3 plane_grid(int64_t H, int64_t W) {
  int64_t gx = (W + 255) / 256, gy = H;
  if (gx > 64) gx = 64;
  if (gy > 65535) gy = 65535;
  return dim3((unsigned)gx, (unsigned)gy);
}

}  // namespace

#define IWPP_EDT_VARIANTS(X) \
  X(4, 32)                   \
  X(8, 32)

bool edt_variant_supported(int conn, int tile_h) {
#define X(C, H) \
  if (conn == C && tile_h == H) return true;
  IWPP_EDT_VARIANTS(X)
#undef X
  return false;
}

hipError_t launch_persistent_edt(int conn, int tile_h, const DevImage& one, const KParams& kp,
                                 DevCtl* ctl, int* queue, uint32_t* state, uint8_t* visited,
                                 int grid, hipStream_t st) {
#define X(C, H)                                                                              \
  if (conn == C && tile_h == H) {                                                            \
    hipLaunchKernelGGL((k_persistent_edt<C, H>), dim3(grid), dim3(kThreads), 0, st, one,     \
                       (const DevImage*)nullptr, kp, ctl, queue, state, visited);            \
    return hipGetLastError();                                                                \
  }
  IWPP_EDT_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int persistent_edt_blocks_per_cu(int conn, int tile_h) {
  int nb = 0;
#define X(C, H)                                                                                \
  if (conn == C && tile_h == H) {                                                              \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent_edt<C, H>, kThreads, 0) \
        != hipSuccess)                                                                         \
      return 0;                                                                                \
    return nb;                                                                                 \
  }
  IWPP_EDT_VARIANTS(X)
#undef X
  return 0;
}

hipError_t launch_edt_init(void* sites, int64_t ld_out, const void* img, int64_t ld_img,
                           int64_t H, int64_t W, hipStream_t st) {
  hipLaunchKernelGGL(k_edt_init, plane_grid(H, W), dim3(256), 0, st, (uint32_t*)sites, ld_out,
                     (const uint8_t*)img, ld_img, H, W);
  return hipGetLastError();
}

hipError_t launch_edt_dist(void* dist, const void* sites, int64_t ld_out, int64_t H, int64_t W,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_edt_dist, plane_grid(H, W), dim3(256), 0, st, (int32_t*)dist,
                     (const uint32_t*)sites, ld_out, H, W);
  return hipGetLastError();
}

}  // namespace iwpp
