// iwpp_kernels.hip -- HIP kernels (gfx950) for grayscale morphological
// reconstruction by dilation, organised as an irregular wavefront propagation
// (IWPP) over image tiles.
//
// Method (Gomes & Teodoro): the reconstruction R of mask I from marker J <= I
// is the fixed point of J <- dilate(J) ^ I (reconstruction Equation).  The
// paper computes it in two phases: raster / anti-raster scans propagate most
// values, then the pixels that can still raise a neighbour seed a queue that
// runs to stability (the IWPP reconstruction algorithm).  Its many-core
// redesign (the atomic-free two-phase algorithm of "Algoritmo Proposto")
// splits each wave of the queue into an identification phase, which collects
// the pixels that will receive a value, and a propagation phase in which each
// receiver only updates itself.
//
// GPU mapping:
//  * One workgroup (4 wavefronts of 64 lanes) owns one 64-wide tile at a time.
//    The tile and a 1-pixel halo of I and J are staged in LDS with coalesced
//    row loads (a tile row is one wavefront).
//  * Scan phase: rounds of four directional passes (down, up, right, left).
//    A vertical pass walks rows with one lane per column; a horizontal pass
//    walks columns with one lane per row.  Each pass takes every pixel to
//    min(I, max(J, the three neighbours on the side it comes from)), so one
//    round pulls from all eight neighbours.  Each pixel has a single writer
//    per pass; reads across band borders may see old or new values, which is
//    harmless because values only grow and are re-checked.
//  * Seed detection: one lane per pixel tests whether a neighbour can still
//    raise it; receivers are compacted into an LDS queue with a wavefront
//    ballot + mbcnt prefix and one LDS atomic per wavefront (the role of the
//    paper's popcnt / prefix-sum / scatter insertion).
//  * Queue phase (two-phase IWPP): propagate -- each receiver pulls
//    min(I, max(J, max of its neighbours)) and writes only itself; identify --
//    the receivers that changed find their neighbours that can be raised and
//    append them to the other LDS queue.  No pixel atomics.  A queue overflow
//    falls back to another scan round, which is always correct.
//  * Cross-tile propagation: after write-back, a tile activates each
//    neighbour tile into which one of its changed border pixels can propagate.
//    Persistent workgroups take tile ids from a global work queue; a per-tile
//    state word keeps every tile single-owner (a tile activated while running
//    is re-run in place by its owner after reloading its halo).  The launch
//    ends when no tile is queued or running.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "iwpp_internal.h"

namespace iwpp {

constexpr int NT = kThreads;
constexpr int NW = NT / 64;
constexpr int TW = kTileW;

// ------------------------------------------------------------ atomics

__device__ __forceinline__ uint32_t ld_acq_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_rlx_i32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup-wide OR.  The leading barrier orders all earlier LDS and global
// accesses of the workgroup before the reduction's own synchronisation.
__device__ __forceinline__ int block_any(bool p) {
  __syncthreads();
  return __syncthreads_or(p);
}

// ------------------------------------------------------------ pixel types

template <typename T>
struct Lowest;
template <>
struct Lowest<uint8_t> {
  static constexpr int v = 0;
};
template <>
struct Lowest<int32_t> {
  static constexpr int v = INT_MIN;
};

// LDS image of one tile plus a 1-pixel halo.  Interior pixel (y, x),
// 0 <= y < TH, 0 <= x < TW, lives at (y + 1) * P + (x + 1).  The pitch is
// odd in 32-bit words so that one-lane-per-row passes hit distinct banks.
template <typename T, int TH>
struct Geo {
  static constexpr int P = sizeof(T) == 1 ? TW + 4 : TW + 3;
  static constexpr int ROWS = TH + 2;
  static constexpr int NPIX = TH * TW;
  static constexpr int QCAP = TH * TW;
  static constexpr int RING = 2 * TW + 2 * TH;            // interior border positions
  static constexpr int HALO = 2 * (TW + 2) + 2 * TH;      // halo positions
  __device__ static constexpr int at(int y, int x) { return (y + 1) * P + (x + 1); }
};

template <typename T, int TH>
struct Lds {
  using G = Geo<T, TH>;
  T J[G::ROWS * G::P];
  T I[G::ROWS * G::P];
  uint16_t q[2][G::QCAP];
  T b_top[TW], b_bot[TW], b_left[TH], b_right[TH];  // border as loaded
  uint8_t rowdirty[TH];
  int qn[2];
  int act[9];
  int viol;
  int tile;
  int cmd;
  int npush;
  int nround;
  int novf;
};

// Queue entries are 15-bit pixel indices y * TW + x; bit 15 marks an entry
// whose pixel rose during the propagation phase.
constexpr uint16_t kRose = 0x8000u;

template <typename T, int CONN, int TH>
struct Tile {
  using G = Geo<T, TH>;
  using L = Lds<T, TH>;
  static constexpr int LO = Lowest<T>::v;
  static constexpr int RG = TH / 64;  // 64-row groups (horizontal passes)
  static constexpr int NS = NW / RG;  // column strips (horizontal passes)
  static constexpr int SW = TW / NS;  // strip width
  static constexpr int BAND = TH / NW;  // rows per wavefront (vertical passes)
  static_assert(TH % 64 == 0 && NW % RG == 0 && TH / 64 <= NW, "tile height");
  static_assert(G::NPIX <= 32768, "queue entries are 15-bit");
  static_assert(G::NPIX % NT == 0, "whole wavefronts per scan");

  __device__ static int jv(const L& s, int y, int x) { return (int)s.J[G::at(y, x)]; }
  __device__ static int iv(const L& s, int y, int x) { return (int)s.I[G::at(y, x)]; }

  // ---------------------------------------------------------- compaction
  // Append `val` for every lane with `pred` to queue `which`.  All 64 lanes
  // of the wavefront must call it together.
  __device__ static void push(L& s, int which, bool pred, int val) {
    const unsigned long long b = __ballot(pred);
    if (b == 0) return;
    const int n = __popcll(b);
    int base = 0;
    if ((threadIdx.x & 63) == 0) base = atomicAdd(&s.qn[which], n);
    base = __builtin_amdgcn_readfirstlane(base);
    const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32),
                                              __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
    if (pred && base + off < G::QCAP) s.q[which][base + off] = (uint16_t)val;
  }

  // ---------------------------------------------------------- load / store
  // Stage tile (ty, tx) and its halo.  Pixels outside the image become the
  // lowest value in both I and J: they can neither give nor take a value.
  // J is clamped to I on load; a first visit reports interior J > I.
  __device__ static void load(L& s, const DevImage& im, int64_t y0, int64_t x0, bool first) {
    const T* __restrict__ gJ = (const T*)im.J;
    const T* __restrict__ gI = (const T*)im.I;
    bool viol = false;
    constexpr int RW = TW + 2;
    if (threadIdx.x < TH) s.rowdirty[threadIdx.x] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < G::ROWS * RW; e += NT) {
      const int yy = e / RW, xx = e - yy * RW;  // padded coordinates
      const int64_t gy = y0 + yy - 1, gx = x0 + xx - 1;
      int j = LO, i = LO;
      if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) {
        const int64_t o = gy * im.ld + gx;
        j = (int)gJ[o];
        i = (int)gI[o];
        if (j > i) {
          if (yy >= 1 && yy <= TH && xx >= 1 && xx <= TW) {
            viol = viol || first;
            s.rowdirty[yy - 1] = 1;  // the clamped value must reach memory
          }
          j = i;
        }
      }
      s.J[yy * G::P + xx] = (T)j;
      s.I[yy * G::P + xx] = (T)i;
    }
    if (threadIdx.x < 9) s.act[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      s.npush = 0;
      s.nround = 0;
      s.novf = 0;
    }
    const int any = block_any(viol);
    if (any && threadIdx.x == 0) s.viol = 1;
    snapshot_border(s);
    __syncthreads();
  }

  __device__ static void snapshot_border(L& s) {
    for (int e = threadIdx.x; e < TW; e += NT) {
      s.b_top[e] = s.J[G::at(0, e)];
      s.b_bot[e] = s.J[G::at(TH - 1, e)];
    }
    for (int e = threadIdx.x; e < TH; e += NT) {
      s.b_left[e] = s.J[G::at(e, 0)];
      s.b_right[e] = s.J[G::at(e, TW - 1)];
    }
  }

  // Re-read the halo of J (the tile's own pixels in LDS are current because
  // this workgroup is their only writer).
  __device__ static void reload_halo(L& s, const DevImage& im, int64_t y0, int64_t x0) {
    const T* __restrict__ gJ = (const T*)im.J;
    for (int e = threadIdx.x; e < G::HALO; e += NT) {
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
      if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) {
        const int i = iv(s, y, x);
        const int j = (int)gJ[gy * im.ld + gx];
        s.J[G::at(y, x)] = (T)(j < i ? j : i);
      }
    }
    if (threadIdx.x < TH) s.rowdirty[threadIdx.x] = 0;
    if (threadIdx.x < 9) s.act[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      s.npush = 0;
      s.nround = 0;
      s.novf = 0;
    }
    snapshot_border(s);
    __syncthreads();
  }

  __device__ static void store(const L& s, const DevImage& im, int64_t y0, int64_t x0) {
    T* __restrict__ gJ = (T*)im.J;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int y = wave; y < TH; y += NW) {
      if (!s.rowdirty[y]) continue;
      const int64_t gy = y0 + y, gx = x0 + lane;
      if (gy < im.H && gx < im.W) gJ[gy * im.ld + gx] = s.J[G::at(y, lane)];
    }
  }

  // ---------------------------------------------------------- scans
  // Vertical pass, downward (D = +1) or upward (D = -1).  Wavefront w owns
  // rows [w*BAND, (w+1)*BAND); lane = column.
  template <int D>
  __device__ static bool pass_vert(L& s) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = lane;
    const int ybeg = D > 0 ? wave * BAND : wave * BAND + BAND - 1;
    const int yprev = ybeg - D;
    int pc = jv(s, yprev, x);
    int pl = LO, pr = LO;
    if (CONN == 8) {
      pl = jv(s, yprev, x - 1);
      pr = jv(s, yprev, x + 1);
    }
    bool any = false;
#pragma unroll 2
    for (int k = 0; k < BAND; ++k) {
      const int y = ybeg + D * k;
      const int a = G::at(y, x);
      const int j = (int)s.J[a], i = (int)s.I[a];
      int m = j > pc ? j : pc;
      if (CONN == 8) {
        const int d = pl > pr ? pl : pr;
        m = m > d ? m : d;
      }
      const int v = m < i ? m : i;
      const bool c = v != j;
      if (c) s.J[a] = (T)v;
      if (__ballot(c)) {
        if (lane == 0) s.rowdirty[y] = 1;
        any = true;
      }
      pc = v;
      if (CONN == 8) {
        pl = __shfl_up(v, 1);
        pr = __shfl_down(v, 1);
        if (x == 0) pl = jv(s, y, -1);
        if (x == TW - 1) pr = jv(s, y, TW);
      }
    }
    return any;
  }

  // Horizontal pass, rightward (D = +1) or leftward (D = -1).  Wavefront w
  // owns a strip of SW columns of one 64-row group; lane = row.
  template <int D>
  __device__ static bool pass_horz(L& s) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rg = wave % RG, strip = wave / RG;
    const int y = rg * 64 + lane;
    const int xbeg = D > 0 ? strip * SW : strip * SW + SW - 1;
    const int xprev = xbeg - D;
    int pc = jv(s, y, xprev);
    int pu = LO, pd = LO;
    if (CONN == 8) {
      pu = jv(s, y - 1, xprev);
      pd = jv(s, y + 1, xprev);
    }
    bool dirty = false;
#pragma unroll 2
    for (int k = 0; k < SW; ++k) {
      const int x = xbeg + D * k;
      const int a = G::at(y, x);
      const int j = (int)s.J[a], i = (int)s.I[a];
      int m = j > pc ? j : pc;
      if (CONN == 8) {
        const int d = pu > pd ? pu : pd;
        m = m > d ? m : d;
      }
      const int v = m < i ? m : i;
      if (v != j) {
        s.J[a] = (T)v;
        dirty = true;
      }
      pc = v;
      if (CONN == 8) {
        pu = __shfl_up(v, 1);
        pd = __shfl_down(v, 1);
        if (lane == 0) pu = jv(s, y - 1, x);
        if (lane == 63) pd = jv(s, y + 1, x);
      }
    }
    if (dirty) s.rowdirty[y] = 1;
    return __ballot(dirty) != 0;
  }

  // One round of the four passes; true if any pixel of the tile rose.
  __device__ static bool sweep_round(L& s) {
    bool c = pass_vert<+1>(s);
    __syncthreads();
    c |= pass_vert<-1>(s);
    __syncthreads();
    c |= pass_horz<+1>(s);
    __syncthreads();
    c |= pass_horz<-1>(s);
    if (threadIdx.x == 0) s.nround++;
    return block_any(c) != 0;
  }

  // ---------------------------------------------------------- seeds
  // Largest J over the neighbourhood of interior pixel (y, x), halo included.
  __device__ static int nbr_max(const L& s, int y, int x) {
    const int a = G::at(y, x);
    constexpr int P = G::P;
    int m = (int)s.J[a - P];
    int t = (int)s.J[a + P];
    m = m > t ? m : t;
    t = (int)s.J[a - 1];
    m = m > t ? m : t;
    t = (int)s.J[a + 1];
    m = m > t ? m : t;
    if (CONN == 8) {
      t = (int)s.J[a - P - 1];
      m = m > t ? m : t;
      t = (int)s.J[a - P + 1];
      m = m > t ? m : t;
      t = (int)s.J[a + P - 1];
      m = m > t ? m : t;
      t = (int)s.J[a + P + 1];
      m = m > t ? m : t;
    }
    return m;
  }

  // Every pixel some neighbour can still raise goes to queue 0.
  __device__ static void scan_receivers(L& s) {
    if (threadIdx.x == 0) s.qn[0] = 0;
    __syncthreads();
#pragma unroll 1
    for (int base = 0; base < G::NPIX; base += NT) {
      const int idx = base + threadIdx.x;
      const int y = idx / TW, x = idx % TW;
      const int a = G::at(y, x);
      const int j = (int)s.J[a], i = (int)s.I[a];
      bool r = false;
      if (j < i) r = nbr_max(s, y, x) > j;
      push(s, 0, r, idx);
    }
    __syncthreads();
  }

  // Border pixels that a (new) halo value can raise go to queue 0.
  __device__ static void halo_receivers(L& s) {
    if (threadIdx.x == 0) s.qn[0] = 0;
    __syncthreads();
    for (int base = 0; base < G::RING; base += NT) {
      const int e = base + threadIdx.x;
      bool r = false;
      int idx = 0;
      if (e < G::RING) {
        int y, x;
        ring_pos(e, y, x);
        idx = y * TW + x;
        const int j = jv(s, y, x), i = iv(s, y, x);
        if (j < i) {
          for (int dy = -1; dy <= 1 && !r; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (dy == 0 && dx == 0) continue;
              if (CONN == 4 && dy != 0 && dx != 0) continue;
              const int hy = y + dy, hx = x + dx;
              if (hy >= 0 && hy < TH && hx >= 0 && hx < TW) continue;
              if (jv(s, hy, hx) > j) {
                r = true;
                break;
              }
            }
        }
      }
      push(s, 0, r, idx);
    }
    __syncthreads();
  }

  __device__ static void ring_pos(int e, int& y, int& x) {
    if (e < TW) {
      y = 0;
      x = e;
    } else if (e < 2 * TW) {
      y = TH - 1;
      x = e - TW;
    } else if (e < 2 * TW + TH) {
      y = e - 2 * TW;
      x = 0;
    } else {
      y = e - 2 * TW - TH;
      x = TW - 1;
    }
  }

  // ---------------------------------------------------------- queue phase
  // Two-phase queue loop on queue 0 (receivers).  Returns false when the
  // queue ran dry (the tile is at a fixed point), true on overflow.
  __device__ static bool queue_loop(L& s, uint32_t iter_limit, bool& hit_limit) {
    int cur = 0;
    for (uint32_t iter = 0;; ++iter) {
      const int n = s.qn[cur];
      const int nxt = cur ^ 1;
      if (n > G::QCAP) {
        if (threadIdx.x == 0) s.novf++;
        __syncthreads();
        return true;
      }
      if (n == 0) return false;
      if (iter >= iter_limit) {
        hit_limit = true;
        return false;
      }
      if (threadIdx.x == 0) s.npush += n;
      // propagation: each receiver updates only itself
      for (int e = threadIdx.x; e < n; e += NT) {
        const int idx = s.q[cur][e];
        const int y = idx / TW, x = idx % TW;
        const int a = G::at(y, x);
        const int j = (int)s.J[a], i = (int)s.I[a];
        int v = nbr_max(s, y, x);
        v = v < i ? v : i;
        if (v > j) {
          s.J[a] = (T)v;
          s.rowdirty[y] = 1;
          s.q[cur][e] = (uint16_t)(idx | kRose);
        }
      }
      if (threadIdx.x == 0) s.qn[nxt] = 0;
      __syncthreads();
      // identification: neighbours of risen pixels that can now be raised
#pragma unroll 1
      for (int base = 0; base < n; base += NT) {
        const int e = base + threadIdx.x;
        int idx = 0, jp = LO;
        bool live = false;
        if (e < n) {
          const int q = s.q[cur][e];
          if (q & kRose) {
            live = true;
            idx = q & ~kRose;
            jp = (int)s.J[G::at(idx / TW, idx % TW)];
          }
        }
        const int y = idx / TW, x = idx % TW;
#pragma unroll
        for (int d = 0; d < 9; ++d) {
          const int dy = d / 3 - 1, dx = d % 3 - 1;
          if (d == 4) continue;
          if (CONN == 4 && dy != 0 && dx != 0) continue;
          const int yy = y + dy, xx = x + dx;
          bool r = false;
          if (live && yy >= 0 && yy < TH && xx >= 0 && xx < TW) {
            const int a = G::at(yy, xx);
            const int jq = (int)s.J[a];
            r = jq < jp && jq < (int)s.I[a];
          }
          push(s, nxt, r, yy * TW + xx);
        }
      }
      __syncthreads();
      cur = nxt;
    }
  }

  // ---------------------------------------------------------- full visit
  // Bring the tile to a fixed point given its (fixed) halo.
  __device__ static void solve(L& s, int sweeps, bool seeded, uint32_t iter_limit,
                               bool& hit_limit) {
    int budget = sweeps;
    if (seeded) {
      // The tile was at a fixed point for its previous halo: only border
      // pixels next to a changed halo pixel can be raised at first.
      halo_receivers(s);
      if (!queue_loop(s, iter_limit, hit_limit)) return;
      if (budget < 1) budget = 1;
    }
    for (uint32_t guard = 0;; ++guard) {
      bool ch = true;
      for (int r = 0; r < budget; ++r) {
        ch = sweep_round(s);
        if (!ch) break;
      }
      if (!ch) return;  // a round that changed nothing: fixed point
      scan_receivers(s);
      if (s.qn[0] == 0) return;
      if (!queue_loop(s, iter_limit, hit_limit)) return;
      if (budget < 1) budget = 1;
      if (guard >= iter_limit) {
        hit_limit = true;
        return;
      }
    }
  }

  // Mark the neighbour tiles (3x3 grid index) that a changed border pixel
  // can propagate into.  Halo values are the ones seen at load time; they
  // never exceed the current ones, so no needed activation is missed.
  __device__ static void activation_flags(L& s) {
    for (int e = threadIdx.x; e < G::RING; e += NT) {
      int y, x;
      ring_pos(e, y, x);
      const int j = jv(s, y, x);
      int j0;
      if (e < TW)
        j0 = (int)s.b_top[x];
      else if (e < 2 * TW)
        j0 = (int)s.b_bot[x];
      else if (e < 2 * TW + TH)
        j0 = (int)s.b_left[y];
      else
        j0 = (int)s.b_right[y];
      if (j == j0) continue;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (dy == 0 && dx == 0) continue;
          if (CONN == 4 && dy != 0 && dx != 0) continue;
          const int hy = y + dy, hx = x + dx;
          const int cy = hy < 0 ? 0 : (hy >= TH ? 2 : 1);
          const int cx = hx < 0 ? 0 : (hx >= TW ? 2 : 1);
          if (cy == 1 && cx == 1) continue;
          const int jh = jv(s, hy, hx);
          if (j > jh && jh < iv(s, hy, hx)) s.act[cy * 3 + cx] = 1;
        }
    }
  }

  // Load, solve and write back tile t of image im.
  __device__ static void visit(L& s, const DevImage& im, int64_t t_local, bool first,
                               int sweeps, uint32_t iter_limit, bool& hit_limit) {
    const int64_t ty = t_local / im.tiles_x, tx = t_local % im.tiles_x;
    const int64_t y0 = ty * TH, x0 = tx * TW;
    load(s, im, y0, x0, first);
    solve(s, sweeps, !first, iter_limit, hit_limit);
    store(s, im, y0, x0);
    activation_flags(s);
  }
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

__device__ __forceinline__ void flush_stats(DevCtl* ctl, int npush, int nround, int novf) {
  if (npush) atomicAdd((unsigned long long*)&ctl->pushes, (unsigned long long)npush);
  if (nround) atomicAdd((unsigned long long*)&ctl->sweeps, (unsigned long long)nround);
  if (novf) atomicAdd((unsigned long long*)&ctl->overflows, (unsigned long long)novf);
}

// ------------------------------------------------------------ persistent

// Enqueue tile n (caller has just moved it from idle to pending).
__device__ void queue_push(DevCtl* ctl, int* queue, uint32_t qcap, int n) {
  const uint32_t slot = atomicAdd(&ctl->q_tail, 1u);
  __hip_atomic_store(&queue[slot % qcap], n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t head = ld_acq_u32(&ctl->q_head);
  const uint32_t depth = slot + 1 - head;
  if ((int32_t)depth > 0) atomicMax(&ctl->q_high, depth);
}

// Take a tile id, or -1 when the launch is over (or aborted).
__device__ int queue_pop(DevCtl* ctl, int* queue, const KParams& kp, uint32_t* state) {
  for (uint32_t spin = 0;; ++spin) {
    if (ld_rlx_i32(&ctl->status) & ST_ABORT) return -1;
    const uint32_t h = ld_acq_u32(&ctl->q_head);
    const uint32_t tl = ld_acq_u32(&ctl->q_tail);
    if ((int32_t)(tl - h) > 0) {
      uint32_t expect = h;
      if (!__hip_atomic_compare_exchange_strong(&ctl->q_head, &expect, h + 1u, __ATOMIC_ACQ_REL,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        continue;
      int* slot = &queue[h % kp.qcap];
      int v = -1;
      for (uint32_t w = 0;; ++w) {
        v = __hip_atomic_load(slot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (v >= 0) break;
        if (w > kp.spin_limit) {
          atomicOr(&ctl->status, ST_INTERNAL | ST_ABORT);
          return -1;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __hip_atomic_store(slot, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long nv = atomicAdd((unsigned long long*)&ctl->visits, 1ull);
      if (kp.max_visits > 0 && (long long)nv >= kp.max_visits) {
        atomicOr(&ctl->status, ST_INCOMPLETE | ST_ABORT);
        return -1;
      }
      // pending -> running (acquire: the tile and its halo become visible)
      __hip_atomic_exchange(&state[v], TS_RUNNING, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      return v;
    }
    if (__hip_atomic_load(&ctl->pending, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0)
      return -1;
    if (spin > kp.spin_limit) {
      atomicOr(&ctl->status, ST_INTERNAL | ST_ABORT);
      return -1;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Ask for neighbour n to be (re)visited.
__device__ void activate(DevCtl* ctl, int* queue, uint32_t qcap, uint32_t* state, int n) {
  const uint32_t old =
      __hip_atomic_fetch_or(&state[n], TS_PENDING, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  if (old == 0u) {  // was idle: this workgroup enqueues it
    __hip_atomic_fetch_add(&ctl->pending, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    queue_push(ctl, queue, qcap, n);
  }
}

// Release tile t.  Returns true if a neighbour asked for it while it ran, in
// which case the caller keeps ownership and must run it again.
__device__ bool finish(DevCtl* ctl, uint32_t* state, int t) {
  uint32_t expect = TS_RUNNING;
  if (__hip_atomic_compare_exchange_strong(&state[t], &expect, 0u, __ATOMIC_ACQ_REL,
                                           __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) {
    __hip_atomic_fetch_add(&ctl->pending, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  // running | pending: clear the request and run again
  __hip_atomic_exchange(&state[t], TS_RUNNING, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  atomicAdd((unsigned long long*)&ctl->reproc, 1ull);
  atomicAdd((unsigned long long*)&ctl->visits, 1ull);
  return true;
}

template <typename T, int CONN, int TH>
__global__ __launch_bounds__(NT) void k_persistent(DevImage one, const DevImage* __restrict__ imgs,
                                                   KParams kp, DevCtl* ctl, int* queue,
                                                   uint32_t* state, uint8_t* visited) {
  using TP = Tile<T, CONN, TH>;
  __shared__ typename TP::L s;
  const uint32_t iter_limit = kp.spin_limit;
  for (;;) {
    if (threadIdx.x == 0) {
      s.tile = queue_pop(ctl, queue, kp, state);
      s.viol = 0;
    }
    __syncthreads();
    const int t = s.tile;
    if (t < 0) break;
    const int k = imgs ? find_image(imgs, kp.nimg, t) : 0;
    const DevImage im = imgs ? imgs[k] : one;
    const int64_t tl = (int64_t)t - im.tile_base;
    const int64_t ty = tl / im.tiles_x, tx = tl % im.tiles_x;
    const int64_t y0 = ty * TH, x0 = tx * TW;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool first = visited[t] == 0;
    bool hit = false;
    TP::visit(s, im, tl, first, kp.sweeps, iter_limit, hit);
    for (;;) {
      // publish the tile before anyone is told about it
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const int hit_any = block_any(hit);
      if (threadIdx.x == 0) {
        if (first) visited[t] = 1;
        if (s.viol) atomicOr(&ctl->status, ST_MARKER_GT_MASK);
        if (hit_any) atomicOr(&ctl->status, ST_INTERNAL | ST_ABORT);
        flush_stats(ctl, s.npush, s.nround, s.novf);
        for (int d = 0; d < 9; ++d) {
          if (!s.act[d]) continue;
          const int64_t ny = ty + d / 3 - 1, nx = tx + d % 3 - 1;
          if (ny < 0 || ny >= im.tiles_y || nx < 0 || nx >= im.tiles_x) continue;
          activate(ctl, queue, kp.qcap, state, (int)(im.tile_base + ny * im.tiles_x + nx));
        }
        s.cmd = finish(ctl, state, t) ? 1 : 0;
        s.viol = 0;
      }
      __syncthreads();
      if (!s.cmd) break;
      // a neighbour changed while this tile ran: reload the halo and continue
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      TP::reload_halo(s, im, y0, x0);
      hit = false;
      TP::solve(s, kp.sweeps, true, iter_limit, hit);
      TP::store(s, im, y0, x0);
      TP::activation_flags(s);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ host-driven rounds

// One round: every active tile is visited once; tiles it activates are
// flagged for the next round.  Workgroups are mapped so that each XCD (the
// dispatcher deals workgroups to the 8 XCDs in turn) gets a contiguous run
// of tiles, keeping neighbouring tiles under one L2.
template <typename T, int CONN, int TH>
__global__ __launch_bounds__(NT) void k_round(DevImage one, const DevImage* __restrict__ imgs,
                                              KParams kp, DevCtl* ctl, uint8_t* act_cur,
                                              uint8_t* act_next, uint8_t* visited) {
  using TP = Tile<T, CONN, TH>;
  __shared__ typename TP::L s;
  const int64_t per = (kp.ntiles + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= kp.ntiles || !act_cur[t]) return;
  const int k = imgs ? find_image(imgs, kp.nimg, t) : 0;
  const DevImage im = imgs ? imgs[k] : one;
  const int64_t tl = t - im.tile_base;
  const int64_t ty = tl / im.tiles_x, tx = tl % im.tiles_x;
  const bool first = visited[t] == 0;
  if (threadIdx.x == 0) s.viol = 0;
  bool hit = false;
  TP::visit(s, im, tl, first, kp.sweeps, kp.spin_limit, hit);
  const int hit_any = block_any(hit);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctl->visits, 1ull);
    if (s.viol) atomicOr(&ctl->status, ST_MARKER_GT_MASK);
    if (hit_any) atomicOr(&ctl->status, ST_INTERNAL);
    flush_stats(ctl, s.npush, s.nround, s.novf);
    bool any = false;
    for (int d = 0; d < 9; ++d) {
      if (!s.act[d]) continue;
      const int64_t ny = ty + d / 3 - 1, nx = tx + d % 3 - 1;
      if (ny < 0 || ny >= im.tiles_y || nx < 0 || nx >= im.tiles_x) continue;
      act_next[im.tile_base + ny * im.tiles_x + nx] = 1;
      any = true;
    }
    if (any) atomicOr(&ctl->active_any, 1);
    act_cur[t] = 0;
    visited[t] = 1;
  }
}

// ------------------------------------------------------------ small kernels

// Reset the control block and per-tile state; the queue receives every tile
// in the order slot -> (slot * mul + add) mod ntiles (mul coprime to ntiles).
__global__ void k_init(KParams kp, DevCtl* ctl, int* queue, uint32_t* state, uint8_t* visited,
                       uint8_t* active, uint32_t mul, uint32_t add) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = gid; i < kp.ntiles; i += stride) {
    if (state) state[i] = TS_PENDING;
    visited[i] = 0;
    if (active) active[i] = 1;
  }
  if (queue) {
    for (int64_t i = gid; i < (int64_t)kp.qcap; i += stride) {
      int v = -1;
      if (i < kp.ntiles)
        v = (int)(((unsigned long long)i * mul + add) % (unsigned long long)kp.ntiles);
      queue[i] = v;
    }
  }
  if (gid == 0) {
    DevCtl c = {};
    c.q_head = 0;
    c.q_tail = queue ? (uint32_t)kp.ntiles : 0u;
    c.pending = state ? (int32_t)kp.ntiles : 0;
    c.q_high = c.q_tail;
    *ctl = c;
  }
}

__global__ void k_clear_round(DevCtl* ctl) { ctl->active_any = 0; }

// Plain streaming copy (bandwidth reference for the profiler counters).
__global__ __launch_bounds__(256) void k_copy(uint4* __restrict__ dst,
                                              const uint4* __restrict__ src, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

// ------------------------------------------------------------ dispatch

#define IWPP_VARIANTS(X) \
  X(uint8_t, 4, 64)      \
  X(uint8_t, 8, 64)      \
  X(uint8_t, 4, 128)     \
  X(uint8_t, 8, 128)     \
  X(int32_t, 4, 64)      \
  X(int32_t, 8, 64)

static int dtype_of(uint8_t*) { return 0; }
static int dtype_of(int32_t*) { return 1; }

bool variant_supported(const Variant& v) {
#define X(T, C, H) \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) return true;
  IWPP_VARIANTS(X)
#undef X
  return false;
}

hipError_t launch_persistent(const Variant& v, const DevImage& one, const DevImage* imgs,
                             const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                             uint8_t* visited, int grid, hipStream_t st) {
#define X(T, C, H)                                                                              \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) {                       \
    hipLaunchKernelGGL((k_persistent<T, C, H>), dim3(grid), dim3(NT), 0, st, one, imgs, kp, ctl, \
                       queue, state, visited);                                                  \
    return hipGetLastError();                                                                   \
  }
  IWPP_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_round(const Variant& v, const DevImage& one, const DevImage* imgs,
                        const KParams& kp, DevCtl* ctl, uint8_t* act_cur, uint8_t* act_next,
                        uint8_t* visited, hipStream_t st) {
  const int64_t per = (kp.ntiles + 7) / 8;
  const unsigned grid = (unsigned)(per * 8);
#define X(T, C, H)                                                                           \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) {                    \
    hipLaunchKernelGGL((k_round<T, C, H>), dim3(grid), dim3(NT), 0, st, one, imgs, kp, ctl, \
                       act_cur, act_next, visited);                                          \
    return hipGetLastError();                                                                \
  }
  IWPP_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int persistent_blocks_per_cu(const Variant& v) {
  int nb = 0;
#define X(T, C, H)                                                                      \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) {               \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<T, C, H>, NT, 0) \
        != hipSuccess)                                                                  \
      return 0;                                                                         \
    return nb;                                                                          \
  }
  IWPP_VARIANTS(X)
#undef X
  return 0;
}

hipError_t launch_init(const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                       uint8_t* visited, uint8_t* active, uint32_t order_mul, uint32_t order_add,
                       hipStream_t st) {
  int64_t work = kp.ntiles > (int64_t)kp.qcap ? kp.ntiles : (int64_t)kp.qcap;
  int64_t blocks = (work + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, st, kp, ctl, queue, state,
                     visited, active, order_mul, order_add);
  return hipGetLastError();
}

hipError_t launch_clear_round(DevCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_round, dim3(1), dim3(1), 0, st, ctl);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)dst,
                     (const uint4*)src, n16);
  return hipGetLastError();
}

}  // namespace iwpp
