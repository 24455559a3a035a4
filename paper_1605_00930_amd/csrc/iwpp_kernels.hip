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
// GPU mapping (one 64-lane wavefront owns one tile 64 columns wide):
//  * The tile and a 1-pixel halo of I and J are staged in LDS; a tile row is
//    one wavefront-wide coalesced load.
//  * Scan phase: rounds of four directional passes over the whole tile.  The
//    downward / upward passes walk rows with one lane per column; the
//    rightward / leftward passes walk columns with one lane per row.  Each
//    step takes a pixel to min(I, max(J, the three neighbours on the side the
//    pass comes from)); the previous line lives in registers and the diagonal
//    neighbours arrive by DPP lane shifts, so one round pulls from all eight
//    neighbours and carries a value across the whole tile.
//  * Seed detection: one lane per pixel tests whether a neighbour can still
//    raise it; receivers are compacted into an LDS queue with a wavefront
//    ballot + mbcnt prefix (the role of the paper's popcnt / prefix-sum /
//    scatter insertion).  The wavefront keeps the queue length in a scalar
//    register, so no LDS counter is needed.
//  * Queue phase (two-phase IWPP): propagate -- each receiver pulls
//    min(I, max(J, max of its neighbours)) and writes only itself; identify --
//    receivers that rose find the neighbours they can raise.  A neighbour
//    claims its place in the next queue through a bit in an LDS bitmap, so a
//    pixel is queued at most once per wave of the queue; winners are
//    compacted with ballot + mbcnt.  No pixel atomics.
//  * Cross-tile propagation: after write-back a tile activates each neighbour
//    tile into which one of its changed border pixels can propagate.
//    Persistent wavefronts take tile ids from a global work queue; a per-tile
//    state word keeps every tile single-owner (a tile activated while running
//    is re-run in place by its owner after reloading its halo).  The launch
//    ends when no tile is queued or running.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "iwpp_device.h"
#include "iwpp_internal.h"

namespace iwpp {

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
template <typename T>
struct Highest;
template <>
struct Highest<uint8_t> {
  static constexpr uint8_t v = 255;
};
template <>
struct Highest<int32_t> {
  static constexpr int32_t v = INT_MAX;
};

// LDS image of one tile plus a 1-pixel halo.  Interior pixel (y, x),
// 0 <= y < TH, 0 <= x < TW, lives at (y + 1) * P + (x + 1).  The pitch is
// odd in 32-bit words so that one-lane-per-row passes hit distinct banks.
template <typename T, int TH>
struct Geo {
  static constexpr int P = sizeof(T) == 1 ? TW + 4 : TW + 3;
  static constexpr int ROWS = TH + 2;
  static constexpr int NPIX = TH * TW;
  // Queue capacity: a fraction of the tile, so that eight tiles fit in a
  // CU's LDS; an overflowing queue falls back to rounds of passes.
  static constexpr int QCAP = sizeof(T) == 1 ? NPIX / 4 : NPIX / 8;
  static constexpr int NWORDS = NPIX / 32;
  static constexpr int HALO = 2 * (TW + 2) + 2 * TH;  // halo pixels
  __device__ static constexpr int at(int y, int x) { return (y + 1) * P + (x + 1); }
};

template <typename T, int TH>
struct Lds {
  using G = Geo<T, TH>;
  alignas(16) T J[G::ROWS * G::P];
  alignas(16) T I[G::ROWS * G::P];
  uint16_t q[2][G::QCAP];
  uint32_t claim[G::NWORDS];  // pixels already in the next queue
  T b_top[TW], b_bot[TW], b_left[TH], b_right[TH];  // border as loaded
  uint8_t rowdirty[TH];
  // seam visits (Tile::load_seam): tile rows staged so far (bit y, tiles of
  // at most 32 rows) and the rows the next queue wave needs
  uint32_t loaded, need;
};

// Queue entries are 15-bit pixel indices y * TW + x; bit 15 marks an entry
// whose pixel rose during the propagation phase.
constexpr uint16_t kRose = 0x8000u;

// Issued halo rows of a tile, one int per row and lane (Q false), or four
// consecutive rows to a quad (Q true), so that a 16-byte load of four
// columns fills a quad in place (see Tile::issue_t).
template <int ROWS, bool Q>
struct PreRows {
  int j[ROWS], i[ROWS];
  __device__ __forceinline__ int gj(int k) const { return j[k]; }
  __device__ __forceinline__ int gi(int k) const { return i[k]; }
  __device__ __forceinline__ void set(int k, int a, int b) {
    j[k] = a;
    i[k] = b;
  }
};
template <int ROWS>
struct PreRows<ROWS, true> {
  static constexpr int NQ = ROWS / 4;  // rows past the quads: one int each
  int4v jq[NQ], iq[NQ];
  int jt[ROWS - 4 * NQ], it[ROWS - 4 * NQ];
  __device__ __forceinline__ int gj(int k) const {
    return k < 4 * NQ ? jq[k >> 2][k & 3] : jt[k - 4 * NQ];
  }
  __device__ __forceinline__ int gi(int k) const {
    return k < 4 * NQ ? iq[k >> 2][k & 3] : it[k - 4 * NQ];
  }
  __device__ __forceinline__ void set(int k, int a, int b) {
    if (k < 4 * NQ) {
      jq[k >> 2][k & 3] = a;
      iq[k >> 2][k & 3] = b;
    } else {
      jt[k - 4 * NQ] = a;
      it[k - 4 * NQ] = b;
    }
  }
};

template <typename T, int CONN, int TH>
struct Tile {
  using G = Geo<T, TH>;
  using L = Lds<T, TH>;
  static constexpr int LO = Lowest<T>::v;
  static constexpr int kTH = TH;
  static_assert(TH % 32 == 0 && G::NPIX <= 32768, "queue entries are 15-bit");

  __device__ static int lane() { return threadIdx.x; }
  // Memory <-> tile value.  `flip` is 0 for reconstruction by dilation and
  // all ones for reconstruction by erosion: bitwise NOT reverses the order of
  // both pixel types, so the tile holds the complemented images and the
  // dilation machinery computes the erosion (duality).
  __device__ static int in(T raw, uint32_t flip) { return (int)(T)(raw ^ (T)flip); }
  __device__ static T out(T v, uint32_t flip) { return (T)(v ^ (T)flip); }
  __device__ static int jv(const L& s, int y, int x) { return (int)s.J[G::at(y, x)]; }
  __device__ static int iv(const L& s, int y, int x) { return (int)s.I[G::at(y, x)]; }

  // Append `val` for every lane with `pred` to queue `which`, whose length is
  // the wave-uniform `n`.  Entries past the capacity are dropped; the caller
  // sees n > QCAP.
  __device__ static void push(L& s, int which, int& n, bool pred, int val) {
    const unsigned long long b = __ballot(pred);
    const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32),
                                              __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
    if (pred && n + off < G::QCAP) s.q[which][n + off] = (uint16_t)val;
    n += __popcll(b);
  }

  // ---------------------------------------------------------- load / store
  // Packed side columns.  A launch that keeps them (kp.colJ, kp.colI) holds,
  // for every tile t, its column 0 and its column TW - 1 row after row:
  // entry (t * 2 + side) * TH + r.  A tile reads its halo columns from its
  // neighbours' entries (one contiguous run per side) instead of one pixel
  // from each of TH rows, which costs a whole cache line per row; its owner
  // rewrites them with the tile's dirty rows.  Entries hold memory values
  // (before the complement of an erosion), like the image.
  __device__ static int64_t side_at(int64_t t, int side) { return (t * 2 + side) * TH; }

  // Stage the tile at (y0, x0) (tile t, column tx of its image's tile grid)
  // and its halo.  Pixels outside the image become the lowest value in both
  // I and J: they can neither give nor take a value.  J is clamped to I on
  // load (a clamped pixel's row is marked dirty so that the clamp reaches
  // memory); returns true if a first visit saw J > I inside the tile.
  __device__ __forceinline__ static bool load(L& s, const DevImage& im, int64_t y0, int64_t x0,
                                              bool first, const KParams& kp, int64_t t,
                                              int64_t tx, int sides) {
    // almost every tile lies inside the image with its halo: its loads need
    // no bounds checks and its two row batches are unrolled
    const bool inner = y0 >= 1 && y0 + TH < im.H && x0 >= 1 && x0 + TW < im.W;
    return inner ? load_t<true>(s, im, y0, x0, first, kp, t, tx, sides)
                 : load_t<false>(s, im, y0, x0, first, kp, t, tx, sides);
  }

  // Halo side entry e of a tile: e < TH the left halo column of row e,
  // e < 2 TH the right one of row e - TH, then the four corners (top left,
  // top right, bottom left, bottom right), at (y, x) in halo coordinates
  // (-1 .. TH, -1 .. TW).
  __device__ __forceinline__ static void side_pos(int e, int& y, int& x) {
    if (e < 2 * TH) {
      y = e >= TH ? e - TH : e;
      x = e >= TH ? TW : -1;
    } else {
      y = ((e - 2 * TH) & 2) ? TH : -1;
      x = ((e - 2 * TH) & 1) ? TW : -1;
    }
  }
  // Loads side entry e: returns whether the pixel lies in the image; the raw
  // J and I values go to j and i.  A halo column comes from the neighbour's
  // packed side column when `sides` says it is written (bit 0 left, bit 1
  // right: the neighbour's first visit is complete), else from the image.
  template <bool INNER>
  __device__ __forceinline__ static bool side_load(const DevImage& im, int64_t y0, int64_t x0,
                                                   const KParams& kp, int64_t t, int64_t tx,
                                                   int sides, int e, int& j, int& i) {
    const gptr<const T> gJ = (gptr<const T>)im.J;
    const gptr<const T> gI = (gptr<const T>)im.I;
    int y, x;
    side_pos(e, y, x);
    if (e < 2 * TH) {
      const int side = e >= TH;
      const bool nb = side ? tx + 1 < im.tiles_x : tx > 0;
      if (!(INNER || (nb && y0 + y < im.H))) return false;
      if ((sides >> side) & 1) {
        // the neighbour's own side facing this tile
        const int64_t k = side_at(side ? t + 1 : t - 1, side ? 0 : 1) + y;
        // both written during the launch, possibly under another XCD's L2:
        // coherent loads, like the marker
        j = (int)ld_coherent(&((gptr<const T>)kp.colJ)[k]);
        i = (int)ld_coherent(&((gptr<const T>)kp.colI)[k]);
      } else {
        const int64_t a = (y0 + y) * im.ld + x0 + x;
        j = (int)ld_coherent(&gJ[a]);
        i = (int)gI[a];
      }
      return true;
    }
    const int64_t gy = y0 + y, gx = x0 + x;
    if (!(INNER || (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W))) return false;
    j = (int)ld_coherent(&gJ[gy * im.ld + gx]);
    i = (int)gI[gy * im.ld + gx];
    return true;
  }

  template <bool INNER>
  __device__ __forceinline__ static bool load_t(L& s, const DevImage& im, int64_t y0, int64_t x0,
                                                bool first, const KParams& kp, int64_t t,
                                                int64_t tx, int sides) {
    const uint32_t flip = kp.flip;
    // image rows live in global memory: address-space-1 pointers give
    // global_load instructions, which (unlike flat ones) leave the LDS
    // counter alone
    const gptr<const T> gJ = (gptr<const T>)im.J;
    const gptr<const T> gI = (gptr<const T>)im.I;
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    wsync();
    bool viol = false;
    // raw values are loaded under the bounds checks and complemented after
    // the batch, so no load waits for its own data; a pixel outside the image
    // starts as the raw encoding of LO
    const int lo_raw = in((T)LO, flip);
    // Rows -1 .. TH of the tile's own columns, one lane per column, B rows
    // per batch (each row is whole cache lines of this tile).  The halo
    // columns and corners (side entries, see side_load) are spread over the
    // lanes and issued with the first batch.  Two batches cover a tile of
    // up to 64 rows; taller tiles take batches of 22 rows (registers).
    constexpr int B = G::ROWS <= 66 ? G::ROWS / 2 + 1 : 22;
    constexpr int NE = 2 * TH + 4;
    constexpr int K = (NE + 63) / 64;
    const int64_t gx = x0 + lane();
    const bool c_in = gx < im.W;
    int ej[K], ei[K];
    auto batch = [&](const int yb) {
      int j[B], i[B];
      const int64_t gy0 = y0 + yb - 1;
      const gptr<const T> pj = gJ + gy0 * im.ld + gx;
      const gptr<const T> pi = gI + gy0 * im.ld + gx;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int64_t gy = gy0 + k;
        j[k] = i[k] = lo_raw;
        if (yb + k < G::ROWS && (INNER || (gy >= 0 && gy < im.H && c_in))) {
          j[k] = (int)ld_coherent(&pj[k * im.ld]);
          i[k] = (int)pi[k * im.ld];
        }
      }
      if (yb == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int e = lane() + 64 * k;
          ej[k] = ei[k] = lo_raw;
          if (e < NE) side_load<INNER>(im, y0, x0, kp, t, tx, sides, e, ej[k], ei[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int yy = yb + k;
        if (yy >= G::ROWS) continue;
        int a = in((T)j[k], flip);
        const int b = in((T)i[k], flip);
        if (a > b) {
          if (yy >= 1 && yy <= TH) {
            viol = viol || first;
            s.rowdirty[yy - 1] = 1;  // the clamped value must reach memory
          }
          a = b;
        }
        s.J[yy * G::P + lane() + 1] = (T)a;
        s.I[yy * G::P + lane() + 1] = (T)b;
      }
    };
    if (INNER && G::ROWS <= 2 * B) {
#pragma unroll
      for (int yb = 0; yb < G::ROWS; yb += B) batch(yb);
    } else {
#pragma unroll 1
      for (int yb = 0; yb < G::ROWS; yb += B) batch(yb);
    }
    // side entries: halo pixels only, clamped but never dirty
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = lane() + 64 * k;
      if (e >= NE) continue;
      int y, x;
      side_pos(e, y, x);
      const int b = in((T)ei[k], flip);
      const int a = imin(in((T)ej[k], flip), b);
      s.J[G::at(y, x)] = (T)a;
      s.I[G::at(y, x)] = (T)b;
    }
    if constexpr (kSeamVisits) {
      if (lane() == 0) s.loaded = kAllRows;
    }
    wsync();
    snapshot_border(s);
    wsync();
    return __ballot(viol) != 0;
  }

  // ---------------------------------------------------------- prefetch
  // int32 tiles of 32 rows can hold the raw values of a whole tile and its
  // halo in registers (two per row and lane, plus the side entries), so a
  // worker issues the loads of its next tile before it writes back the
  // current one: their round trip then overlaps the write-back, its drain and
  // the publication, instead of following them.  issue() starts the loads;
  // commit() stages the values in LDS as load() does.
  static constexpr bool kPrefetch = sizeof(T) == 4 && TH == 32;
  static constexpr int kSideEntries = 2 * TH + 4;
  static constexpr int kSideRegs = (kSideEntries + 63) / 64;
  // int32 tiles of 32 rows load halo rows 0 .. 31 sixteen bytes to a lane:
  // eight instructions per array instead of 32, so that the next tile's
  // loads and the current tile's stores stay under the 63 memory operations
  // a wavefront can have outstanding (past that the issue waits a whole
  // round trip).
  static constexpr bool kWideRows = sizeof(T) == 4 && TH == 32;
  // Issued values of a tile: halo row k of J and I for this lane's column
  // (r.gj(k), r.gi(k)), except that int32 tiles of 32 rows (kWideRows) hold
  // rows 0 .. 31 four columns to a lane (quad q: columns 4 (l % 16) .. + 3
  // of row 4 q + l / 16).
  struct Pre {
    PreRows<G::ROWS, kWideRows> r;
    int ej[kSideRegs], ei[kSideRegs];
  };
  __device__ __forceinline__ static bool wide_rows_ok(const DevImage& im) {
    return kWideRows && (((uintptr_t)im.J | (uintptr_t)im.I) % 16) == 0 && im.ld % 4 == 0 &&
           im.ld <= (1 << 24);
  }

  // FAST: the caller has checked prefetchable() (inner tile, and for int32
  // rows that allow 16-byte loads), so only that load path is compiled.
  template <bool INNER, bool FAST = false>
  __device__ __forceinline__ static void issue_t(Pre& p, const DevImage& im, int64_t y0,
                                                 int64_t x0, const KParams& kp, int64_t t,
                                                 int64_t tx, int sides) {
    const gptr<const T> gJ = (gptr<const T>)im.J;
    const gptr<const T> gI = (gptr<const T>)im.I;
    const int lo_raw = in((T)LO, kp.flip);
    // the lane index through an empty asm: values derived from it are then
    // computed here, not kept in registers for the whole launch
    int ln = lane();
    asm volatile("" : "+v"(ln));
    const int64_t gx = x0 + ln;
    const bool c_in = gx < im.W;
    int k0 = 0;
    if constexpr (kWideRows) {
      // halo rows 0 .. 31 (image rows y0 - 1 .. y0 + 30), four columns to a
      // lane: quad q holds columns 4 (l % 16) .. + 3 of row 4 q + l / 16
      static_assert(G::ROWS == 34, "two rows follow the 32 of the quads");
      const int rr = ln >> 4, cq = 4 * (ln & 15);
      if (FAST || (INNER && wide_rows_ok(im))) {
        // sixteen bytes to a lane, one instruction per quad
        const uint32_t row_b = (uint32_t)im.ld * 4u;
        const int64_t o = (y0 - 1) * im.ld + x0;
        const __amdgpu_buffer_rsrc_t rj = rows_rsrc((const void*)(gJ + o), 32u * row_b);
        const __amdgpu_buffer_rsrc_t ri = rows_rsrc((const void*)(gI + o), 32u * row_b);
        const uint32_t voff = (uint32_t)rr * row_b + 4u * (uint32_t)cq;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          p.r.jq[q] = ld_coherent_b128(rj, voff, 4u * (uint32_t)q * row_b);
          p.r.iq[q] = ld_plain_b128(ri, voff, 4u * (uint32_t)q * row_b);
        }
      } else if constexpr (!FAST) {
        // edge tiles and unaligned images: the same layout, a pixel at a time
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int64_t gy = y0 - 1 + 4 * q + rr;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t gxe = x0 + cq + e;
            int a = lo_raw, b = lo_raw;
            if (INNER || (gy >= 0 && gy < im.H && gxe < im.W)) {
              a = (int)ld_coherent(&gJ[gy * im.ld + gxe]);
              b = (int)gI[gy * im.ld + gxe];
            }
            p.r.jq[q][e] = a;
            p.r.iq[q][e] = b;
          }
        }
      }
      k0 = 32;
    }
#pragma unroll
    for (int k = 0; k < G::ROWS; ++k) {
      if (k < k0) continue;
      const int64_t gy = y0 - 1 + k;
      if (INNER || (gy >= 0 && gy < im.H && c_in))
        p.r.set(k, (int)ld_coherent(&gJ[gy * im.ld + gx]), (int)gI[gy * im.ld + gx]);
      else
        p.r.set(k, lo_raw, lo_raw);
    }
#pragma unroll
    for (int k = 0; k < kSideRegs; ++k) {
      const int e = ln + 64 * k;
      p.ej[k] = p.ei[k] = lo_raw;
      if (e < kSideEntries) side_load<INNER>(im, y0, x0, kp, t, tx, sides, e, p.ej[k], p.ei[k]);
    }
  }
  __device__ __forceinline__ static void issue(Pre& p, const DevImage& im, int64_t y0, int64_t x0,
                                               const KParams& kp, int64_t t, int64_t tx,
                                               int sides) {
    const bool inner = y0 >= 1 && y0 + TH < im.H && x0 >= 1 && x0 + TW < im.W;
    if (inner)
      issue_t<true>(p, im, y0, x0, kp, t, tx, sides);
    else
      issue_t<false>(p, im, y0, x0, kp, t, tx, sides);
  }
  // The persistent worker's next-tile prefetch takes only tiles with a
  // single load path: inside the image with their halo and, for int32, rows
  // that allow 16-byte loads.  With several paths the compiler's wait counts
  // follow each of them into the block after, and the first register write
  // of the fast path then waits for every memory operation in flight (the
  // previous publication's atomics among them).  Other tiles load at their
  // visit (load()).
  __device__ __forceinline__ static bool prefetchable(const DevImage& im, int64_t y0,
                                                      int64_t x0) {
    const bool inner = y0 >= 1 && y0 + TH < im.H && x0 >= 1 && x0 + TW < im.W;
    return inner && (!kWideRows || wide_rows_ok(im));
  }
  __device__ __forceinline__ static void issue_prefetch(Pre& p, const DevImage& im, int64_t y0,
                                                        int64_t x0, const KParams& kp, int64_t t,
                                                        int64_t tx, int sides) {
    issue_t<true, true>(p, im, y0, x0, kp, t, tx, sides);
  }
  __device__ __forceinline__ static void clear_pre(Pre& p) {
#pragma unroll
    for (int k = 0; k < G::ROWS; ++k) p.r.set(k, 0, 0);
#pragma unroll
    for (int k = 0; k < kSideRegs; ++k) p.ej[k] = p.ei[k] = 0;
  }
  // Stage the issued values: J clamped to I (a clamped pixel's row is marked
  // dirty), the complement of an erosion applied; returns true if a first
  // visit saw J > I inside the tile.
  __device__ __forceinline__ static bool commit(L& s, const Pre& p, bool first,
                                                const KParams& kp) {
    const uint32_t flip = kp.flip;
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    wsync();
    bool viol = false;
    int y_lane = 0;  // halo rows before this one are already staged
    if constexpr (kWideRows) {
      {
        // rows 0 .. 31, four columns to a lane (issue_t)
        const int rr = lane() >> 4, c = 4 * (lane() & 15) + 1;
        uint32_t clamped = 0;  // bit q: this lane clamped a pixel of quad q
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int yy = 4 * q + rr;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int a = in((T)p.r.jq[q][e], flip);
            const int b = in((T)p.r.iq[q][e], flip);
            clamped |= (uint32_t)(a > b) << q;
            s.J[yy * G::P + c + e] = (T)imin(a, b);
            s.I[yy * G::P + c + e] = (T)b;
          }
        }
        // a clamped pixel's row goes back to memory; inside the tile (halo
        // row 0 is the row above it) it means J > I on a first visit
        clamped &= rr == 0 ? ~1u : ~0u;
        for (uint32_t m = clamped; m; m &= m - 1) {
          s.rowdirty[4 * __builtin_ctz(m) + rr - 1] = 1;
          viol = viol || first;
        }
        y_lane = 32;
      }
    }
#pragma unroll
    for (int yy = 0; yy < G::ROWS; ++yy) {
      if (yy < y_lane) continue;
      int a = in((T)p.r.gj(yy), flip);
      const int b = in((T)p.r.gi(yy), flip);
      if (a > b) {
        if (yy >= 1 && yy <= TH) {
          viol = viol || first;
          s.rowdirty[yy - 1] = 1;
        }
        a = b;
      }
      s.J[yy * G::P + lane() + 1] = (T)a;
      s.I[yy * G::P + lane() + 1] = (T)b;
    }
#pragma unroll
    for (int k = 0; k < kSideRegs; ++k) {
      const int e = lane() + 64 * k;
      if (e >= kSideEntries) continue;
      int y, x;
      side_pos(e, y, x);
      const int b = in((T)p.ei[k], flip);
      const int a = imin(in((T)p.ej[k], flip), b);
      s.J[G::at(y, x)] = (T)a;
      s.I[G::at(y, x)] = (T)b;
    }
    if constexpr (kSeamVisits) {
      if (lane() == 0) s.loaded = kAllRows;
    }
    wsync();
    snapshot_border(s);
    wsync();
    return __ballot(viol) != 0;
  }

  // ---------------------------------------------------------- seam visits
  // A re-visit starts from a tile at its fixed point for an older halo: only
  // pixels next to the seams can rise at first, and typically only a few do,
  // a pixel or two deep.  load_seam() stages just the seam ring -- the rows
  // above, at the top of, at the bottom of and below the tile, the tile's
  // own first and last columns (its packed side columns, written from its
  // first visit on), the neighbours' facing columns and the corners -- and
  // the queue then stages further rows only as its waves reach them
  // (ensure_rows).  A visit that needs the whole tile (rounds of passes)
  // stages the rest first.  Rows that are not staged are never read: queue
  // entries and their neighbours lie on staged rows, the write-back covers
  // dirty rows only, and the activation reads the ring.
  static constexpr bool kSeamVisits = sizeof(T) == 4 && TH <= 32;
  static constexpr uint32_t kAllRows = TH >= 32 ? 0xFFFFFFFFu : ((1u << TH) - 1);

  __device__ __forceinline__ static void load_seam(L& s, const DevImage& im, int64_t y0,
                                                   int64_t x0, const KParams& kp, int64_t t,
                                                   int64_t tx, int sides) {
    const uint32_t flip = kp.flip;
    const gptr<const T> gJ = (gptr<const T>)im.J;
    const gptr<const T> gI = (gptr<const T>)im.I;
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    wsync();
    const int lo_raw = in((T)LO, flip);
    const int64_t gx = x0 + lane();
    const bool c_in = gx < im.W;
    // halo row, first row, last row, halo row (halo coordinates)
    constexpr int ring[4] = {0, 1, TH, TH + 1};
    int j[4], i[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t gy = y0 + ring[k] - 1;
      j[k] = i[k] = lo_raw;
      if (gy >= 0 && gy < im.H && c_in) {
        j[k] = (int)ld_coherent(&gJ[gy * im.ld + gx]);
        i[k] = (int)gI[gy * im.ld + gx];
      }
    }
    // the tile's own first and last columns: entry e < TH is column 0 of
    // row e, the next TH column TW - 1
    constexpr int KO = (2 * TH + 63) / 64;
    int oj[KO], oi[KO];
#pragma unroll
    for (int k = 0; k < KO; ++k) {
      const int e = lane() + 64 * k;
      const int side = e >= TH, r = side ? e - TH : e, x = side ? TW - 1 : 0;
      oj[k] = oi[k] = lo_raw;
      if (e < 2 * TH && y0 + r < im.H && x0 + x < im.W) {
        oj[k] = (int)ld_coherent(&((gptr<const T>)kp.colJ)[side_at(t, side) + r]);
        oi[k] = (int)ld_coherent(&((gptr<const T>)kp.colI)[side_at(t, side) + r]);
      }
    }
    constexpr int NE = 2 * TH + 4;
    constexpr int K = (NE + 63) / 64;
    int ej[K], ei[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = lane() + 64 * k;
      ej[k] = ei[k] = lo_raw;
      if (e < NE) side_load<false>(im, y0, x0, kp, t, tx, sides, e, ej[k], ei[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = in((T)i[k], flip);
      int a = in((T)j[k], flip);
      if (a > b) {
        if (ring[k] >= 1 && ring[k] <= TH) s.rowdirty[ring[k] - 1] = 1;
        a = b;
      }
      s.J[ring[k] * G::P + lane() + 1] = (T)a;
      s.I[ring[k] * G::P + lane() + 1] = (T)b;
    }
#pragma unroll
    for (int k = 0; k < KO; ++k) {
      const int e = lane() + 64 * k;
      if (e >= 2 * TH) continue;
      const int side = e >= TH, r = side ? e - TH : e, x = side ? TW - 1 : 0;
      const int b = in((T)oi[k], flip);
      s.J[G::at(r, x)] = (T)imin(in((T)oj[k], flip), b);
      s.I[G::at(r, x)] = (T)b;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = lane() + 64 * k;
      if (e >= NE) continue;
      int y, x;
      side_pos(e, y, x);
      const int b = in((T)ei[k], flip);
      s.J[G::at(y, x)] = (T)imin(in((T)ej[k], flip), b);
      s.I[G::at(y, x)] = (T)b;
    }
    if (lane() == 0) {
      s.loaded = 1u | (1u << (TH - 1));
      s.need = 0;
    }
    wsync();
    snapshot_border(s);
    wsync();
  }

  // Stage the tile rows in `need` (bit y) that are not staged yet, four at
  // a time (their loads in flight together), and record them.
  __device__ __forceinline__ static void ensure_rows(L& s, const DevImage& im, int64_t y0,
                                                     int64_t x0, const KParams& kp,
                                                     uint32_t need) {
    uint32_t missing = need & ~__builtin_amdgcn_readfirstlane(s.loaded);
    if (!missing) return;
    const uint32_t flip = kp.flip;
    const gptr<const T> gJ = (gptr<const T>)im.J;
    const gptr<const T> gI = (gptr<const T>)im.I;
    const int lo_raw = in((T)LO, flip);
    const int64_t gx = x0 + lane();
    const bool c_in = gx < im.W;
    const uint32_t got = missing;
    while (missing) {
      constexpr int R = 4;
      int r[R], j[R], i[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        r[k] = missing ? __builtin_ctz(missing) : -1;
        missing &= missing - 1;
        j[k] = i[k] = lo_raw;
        const int64_t gy = y0 + r[k];
        if (r[k] >= 0 && gy < im.H && c_in) {
          j[k] = (int)ld_coherent(&gJ[gy * im.ld + gx]);
          i[k] = (int)gI[gy * im.ld + gx];
        }
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (r[k] < 0) continue;
        const int b = in((T)i[k], flip);
        int a = in((T)j[k], flip);
        if (a > b) {
          s.rowdirty[r[k]] = 1;
          a = b;
        }
        s.J[G::at(r[k], lane())] = (T)a;
        s.I[G::at(r[k], lane())] = (T)b;
      }
    }
    if (lane() == 0) s.loaded |= got;
    wsync();
  }
  __device__ __forceinline__ static void ensure_all_rows(L& s, const DevImage& im, int64_t y0,
                                                         int64_t x0, const KParams& kp) {
    if constexpr (kSeamVisits)
      ensure_rows(s, im, y0, x0, kp, kAllRows);
  }

  __device__ __forceinline__ static void snapshot_border(L& s) {
    s.b_top[lane()] = s.J[G::at(0, lane())];
    s.b_bot[lane()] = s.J[G::at(TH - 1, lane())];
    for (int y = lane(); y < TH; y += 64) {
      s.b_left[y] = s.J[G::at(y, 0)];
      s.b_right[y] = s.J[G::at(y, TW - 1)];
    }
  }

  // Re-read the halo of J for a re-run after a release that found a
  // request; the tile's own pixels in LDS are current because this
  // wavefront is their only writer.
  __device__ __forceinline__ static void reload_halo(L& s, const DevImage& im, int64_t y0,
                                                     int64_t x0, const KParams& kp, int64_t t,
                                                     int64_t tx, int sides) {
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    refresh_halo(s, im, y0, x0, kp, t, tx, sides);
    snapshot_border(s);
    wsync();
  }

  // Re-read the halo of J (and nothing else): the rows above and below the
  // tile's own columns, then the side entries.
  __device__ __forceinline__ static void refresh_halo(L& s, const DevImage& im, int64_t y0,
                                                      int64_t x0, const KParams& kp, int64_t t,
                                                      int64_t tx, int sides) {
    const gptr<const T> gJ = (gptr<const T>)im.J;
    constexpr int NE = 2 * TH + 4;
    const int64_t gx = x0 + lane();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int y = h ? TH : -1;
      const int64_t gy = y0 + y;
      if (gy >= 0 && gy < im.H && gx < im.W) {
        const int j = in(ld_coherent(&gJ[gy * im.ld + gx]), kp.flip);
        s.J[G::at(y, lane())] = (T)imin(j, iv(s, y, lane()));
      }
    }
    for (int e = lane(); e < NE; e += 64) {
      int y, x, j, i;
      side_pos(e, y, x);
      if (side_load<false>(im, y0, x0, kp, t, tx, sides, e, j, i))
        s.J[G::at(y, x)] = (T)imin(in((T)j, kp.flip), iv(s, y, x));
    }
    wsync();
  }

  // Write back the dirty rows, and their side pixels into the packed side
  // columns when the launch keeps them: every row's on the tile's first
  // visit (nothing wrote them before), with the side pixels of I.
  __device__ __forceinline__ static void store(const L& s, const DevImage& im, int64_t y0,
                                               int64_t x0, const KParams& kp, int64_t t,
                                               bool first) {
    const uint32_t flip = kp.flip;
    const bool col_in = x0 + lane() < im.W;
    constexpr int NR = TH < 64 ? TH : 64;
    // side entry e: column 0 of row e (e < TH), column TW - 1 of row e - TH;
    // read before the first store, like the rows (see below)
    constexpr int KS = (2 * TH + 63) / 64;
    int sv[KS];
    bool sw[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int e = lane() + 64 * k;
      const int side = e >= TH, r = side ? e - TH : e, x = side ? TW - 1 : 0;
      sw[k] = kp.colJ && e < 2 * TH && (first || s.rowdirty[r]) && y0 + r < im.H &&
              x0 + x < im.W;
      sv[k] = sw[k] ? (int)s.J[G::at(r, x)] : 0;
      if (first && sw[k])
        st_coherent(&((gptr<T>)kp.colI)[side_at(t, side) + r], out(s.I[G::at(r, x)], flip));
    }
    // uint8 rows are written four pixels to a lane when the image allows
    // 4-byte accesses there (a 64-byte row is then 16 lanes, four rows to an
    // instruction) instead of one byte per lane and row
    // (64-row tiles; taller ones keep within their register budget with bytes)
    const bool wide = sizeof(T) == 1 && TH <= 64 && ((uintptr_t)im.J % 4) == 0 &&
                      (im.ld % 4) == 0 && x0 + TW <= im.W;
    for (int g = 0; g < TH; g += 64) {
      // lane k reports row g + k; the set bits are the rows to write back
      const unsigned long long rows = __ballot(g + lane() < TH && s.rowdirty[g + lane()]);
      if (!rows) continue;
      if constexpr (sizeof(T) == 1) {
        if (TH <= 64 && wide) {
          // lane l: columns 4 (l % 16) .. + 3 of rows 4 q + l / 16, eight
          // quads of rows at a time
          constexpr int NQ = NR / 4;
          const int c4 = (lane() & 15) * 4, rs = lane() >> 4;
          gptr<uint32_t> row = (gptr<uint32_t>)((gptr<T>)im.J + (y0 + g + rs) * im.ld + x0 + c4);
          const uint32_t fw = flip ? 0xFFFFFFFFu : 0u;
          // this lane's rows: bit q for row 4 q + rs, dirty and inside the image
          const int64_t rows_in = im.H - (y0 + g);
          uint32_t mine = 0;
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            mine |= (uint32_t)(((rows >> (4 * q)) >> rs) & 1ull & (4 * q + rs < rows_in)) << q;
#pragma unroll
          for (int q0 = 0; q0 < NQ; q0 += 8) {
            uint32_t w[8];
            // the four pixels start one byte past a 4-byte boundary in LDS
            // (the halo column comes first): two aligned words and a shift
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const uint32_t* a = (const uint32_t*)&s.J[G::at(g + 4 * (q0 + q) + rs, c4) - 1];
              w[q] = __builtin_amdgcn_alignbyte(a[1], a[0], 1);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              if ((mine >> (q0 + q)) & 1u) st_coherent(row, w[q] ^ fw);
              row = (gptr<uint32_t>)((gptr<T>)row + 4 * im.ld);
              asm volatile("" : "+v"(row));
            }
          }
          continue;
        }
        // other uint8 rows (a pitch or base that is not a multiple of 4, or a
        // tile past the right edge): one byte per lane and row
        gptr<T> row = (gptr<T>)im.J + (y0 + g) * im.ld + x0 + lane();
        const int64_t rows_in = im.H - (y0 + g);
#pragma unroll 1
        for (int k = 0; k < NR; ++k) {
          if (((rows >> k) & 1ull) && k < rows_in && col_in)
            st_coherent(row, out(s.J[G::at(g + k, lane())], flip));
          row += im.ld;
        }
        continue;
      }
      if constexpr (sizeof(T) == 4) {
        // int32 rows are written two pixels to a lane (8-byte stores, two
        // rows to an instruction) when the image allows 8-byte accesses there
        const bool wide4 = TH <= 32 && (im.ld % 2) == 0 && ((uintptr_t)im.J % 8) == 0 &&
                           x0 + TW <= im.W;
        if (wide4) {
          constexpr int NQ = NR / 2;
          const int c2 = 2 * (lane() & 31), rs = lane() >> 5;
          const int64_t rows_in = im.H - (y0 + g);
          // every value is read from LDS before the first store (see below)
          uint64_t w[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int a = G::at(g + 2 * q + rs, c2);
            w[q] = (uint64_t)(uint32_t)out(s.J[a], flip) |
                   ((uint64_t)(uint32_t)out(s.J[a + 1], flip) << 32);
          }
          // this lane's rows: bit q for row 2 q + rs, dirty and inside the image
          uint32_t mine = 0;
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            mine |= (uint32_t)(((rows >> (2 * q)) >> rs) & 1ull & (2 * q + rs < rows_in)) << q;
          gptr<uint64_t> row = (gptr<uint64_t>)((gptr<T>)im.J + (y0 + g + rs) * im.ld + x0 + c2);
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if ((mine >> q) & 1u) st_coherent(row, w[q]);
            row = (gptr<uint64_t>)((gptr<T>)row + 2 * im.ld);
            asm volatile("" : "+v"(row));
          }
          continue;
        }
      }
      // Every row's value is read from LDS before the first store: an LDS
      // read into a register that an outstanding store still reads would
      // make the store wait for completion (a store reads its registers
      // after it issues), so reads between stores serialize them.
      int v[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) v[k] = (int)s.J[G::at(g + k, lane())];
      // one pointer, stepped row by row (the empty asm keeps the compiler
      // from holding every row's address in registers at once)
      gptr<T> row = (gptr<T>)im.J + (y0 + g) * im.ld + x0 + lane();
      const int64_t rows_in = im.H - (y0 + g);
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        if (((rows >> k) & 1ull) && k < rows_in && col_in) st_coherent(row, out((T)v[k], flip));
        row += im.ld;
        asm volatile("" : "+v"(row));
      }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int e = lane() + 64 * k;
      const int side = e >= TH, r = side ? e - TH : e;
      if (sw[k]) st_coherent(&((gptr<T>)kp.colJ)[side_at(t, side) + r], out((T)sv[k], flip));
    }
  }

  // ---------------------------------------------------------- scans
  // The passes keep a register chain along the walking direction.  Rows (or
  // columns) are loaded B at a time before they are used, so LDS latency is
  // paid once per batch instead of once per step; every pixel of a pass has a
  // single writer, so loading ahead is safe.  Changed rows are collected as
  // ballot bits in `d` (wave-uniform) and written to rowdirty by the caller.
  // t <- max(t, prev of the lane on the left, prev of the lane on the right).
  // A DPP lane whose source lane is outside the wavefront is not written, so
  // lane 0 (no left lane) and lane 63 (no right lane) keep their t for that
  // side.  The s_nop gives the two wait states a DPP read of a VGPR needs
  // after a VALU write of it, whatever the compiler scheduled before.
  __device__ static int max_sides(int t, int prev) {
    asm("s_nop 1\n\t"
        "v_max_i32_dpp %0, %1, %0 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_max_i32_dpp %0, %1, %0 wave_shl:1 row_mask:0xf bank_mask:0xf"
        : "+v"(t)
        : "v"(prev));
    return t;
  }

  // max(t0, prev, and the prev of the lanes on either side), for one
  // 8-connected step of a pass (t0 holds the pixel's own J and the fill
  // value).  The DPP reads of prev come two wait states after whatever
  // wrote it (the first max and the s_nop), so the block needs no other
  // padding, and the chain through prev is three instructions plus the min
  // that follows.
  __device__ static int max8(int prev, int t0) {
    int b;
    asm("v_max_i32 %0, %1, %2\n\t"
        "s_nop 0\n\t"
        "v_max_i32_dpp %0, %1, %0 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_max_i32_dpp %0, %1, %0 wave_shl:1 row_mask:0xf bank_mask:0xf"
        : "=&v"(b)
        : "v"(prev), "v"(t0));
    return b;
  }

  // Eight consecutive 8-connected steps of one chain in a single asm block.
  // Step k sets r[k] = min(I, max(t[k], the chain value and the chain values
  // of the lanes on either side)) and acc |= chain value ^ its old value,
  // the change made by the step before (bitop3 0xbe is s2 | (s0 ^ s1)).
  // The compiler cannot see into an asm block, so between two blocks it keeps
  // a wait state for the DPP reads that might open the second: one block
  // per step spends an s_nop per step, one block per eight steps one per
  // eight.  In the block every DPP read of a chain value comes two wait
  // states after its write (the max and the change bookkeeping sit
  // between), as the hardware requires.
  // On entry p is the chain value and jp the old value it replaced (equal
  // to p for "no change"); t[k] is the value step k takes with the chain
  // (its own J, for step 0 possibly raised by a halo corner) and o0 the old
  // J of step 0 (the old J of steps 1..7 is t[k]); r[k] receives the results
  // and acc the change bits of steps -1 .. 6 (the caller folds in step 7's).
  __device__ static void step8x8(int p, uint32_t& acc, int jp, int o0, const int (&t)[8],
                                 const int (&ii)[8], int (&r)[8]) {
    int b;
#define IWPP_V8(R, P, T, O, I)                                                  \
  "v_max_i32 %8, " P ", " T "\n\t"                                             \
  "v_bitop3_b32 %9, " P ", " O ", %9 bitop3:0xbe\n\t"                          \
  "v_max_i32_dpp %8, " P ", %8 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"      \
  "v_max_i32_dpp %8, " P ", %8 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"      \
  "v_min_i32 " R ", %8, " I "\n\t"
    asm(IWPP_V8("%0", "%10", "%13", "%11", "%21")
        IWPP_V8("%1", "%0", "%14", "%12", "%22")
        IWPP_V8("%2", "%1", "%15", "%14", "%23")
        IWPP_V8("%3", "%2", "%16", "%15", "%24")
        IWPP_V8("%4", "%3", "%17", "%16", "%25")
        IWPP_V8("%5", "%4", "%18", "%17", "%26")
        IWPP_V8("%6", "%5", "%19", "%18", "%27")
        IWPP_V8("%7", "%6", "%20", "%19", "%28")
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
          "=&v"(r[6]), "=&v"(r[7]), "=&v"(b), "+v"(acc)
        : "v"(p), "v"(jp), "v"(o0), "v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3]), "v"(t[4]),
          "v"(t[5]), "v"(t[6]), "v"(t[7]), "v"(ii[0]), "v"(ii[1]), "v"(ii[2]), "v"(ii[3]),
          "v"(ii[4]), "v"(ii[5]), "v"(ii[6]), "v"(ii[7]));
#undef IWPP_V8
  }

  // Down (D = +1) or up (D = -1) pass, one lane per column: each pixel takes
  // min(I, max(J, the three pixels of the previous row around it)).  The
  // previous row stays in `prev`; its diagonal neighbours come from the lanes
  // beside.  A fixed point needs every neighbour relation to be enforced by
  // one of the four passes, not by all, so the passes share the halo: the
  // vertical passes take the halo rows above and below the tile, the
  // horizontal passes the halo columns beside it.  The four halo corners are
  // reached by neither lane scheme; lanes 0 and 63 take the two corners
  // beside the pass's first previous row at its first step.
  // Changes are collected as bits (`acc`, one bitop per step) and reported
  // per batch of B rows.
  // Rows go in batches of B; the LDS reads of the next batch are issued
  // before the current batch is worked, so their latency overlaps it (the
  // next batch's rows are not written by the current one).
  static constexpr int B = 16;
  static_assert(TH % (2 * B) == 0, "the vertical pass works two batches per iteration");

  // step8x8 without the change bookkeeping, for rounds whose changes nobody
  // reads (see solve): four instructions a step, and an s_nop in place of
  // the bookkeeping keeps every DPP read of a chain value two wait states
  // after its write.
  __device__ static void step8x8n(int p, const int (&t)[8], const int (&ii)[8], int (&r)[8]) {
    int b;
#define IWPP_V8N(R, P, T, I)                                                    \
  "v_max_i32 %8, " P ", " T "\n\t"                                             \
  "s_nop 0\n\t"                                                                \
  "v_max_i32_dpp %8, " P ", %8 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"      \
  "v_max_i32_dpp %8, " P ", %8 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"      \
  "v_min_i32 " R ", %8, " I "\n\t"
    asm(IWPP_V8N("%0", "%9", "%10", "%18")
        IWPP_V8N("%1", "%0", "%11", "%19")
        IWPP_V8N("%2", "%1", "%12", "%20")
        IWPP_V8N("%3", "%2", "%13", "%21")
        IWPP_V8N("%4", "%3", "%14", "%22")
        IWPP_V8N("%5", "%4", "%15", "%23")
        IWPP_V8N("%6", "%5", "%16", "%24")
        IWPP_V8N("%7", "%6", "%17", "%25")
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
          "=&v"(r[6]), "=&v"(r[7]), "=&v"(b)
        : "v"(p), "v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3]), "v"(t[4]), "v"(t[5]), "v"(t[6]),
          "v"(t[7]), "v"(ii[0]), "v"(ii[1]), "v"(ii[2]), "v"(ii[3]), "v"(ii[4]), "v"(ii[5]),
          "v"(ii[6]), "v"(ii[7]));
#undef IWPP_V8N
  }

  // A batch of B steps of one 8-connected chain, eight steps per asm block.
  // jj holds the own J of each step on entry and the results on return;
  // `first` is the value step 0 takes with the chain in place of its own J
  // (the own J raised by a halo corner).  The change bits of every step go
  // to acc.
  __device__ static void steps8(int& prev, uint32_t& acc, int first, int (&jj)[B],
                                const int (&ii)[B]) {
    static_assert(B % 8 == 0, "steps go eight to an asm block");
    int jp = prev;  // the first step sees no change before it
#pragma unroll
    for (int g = 0; g < B; g += 8) {
      int t[8], i8[8], r[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        t[k] = jj[g + k];
        i8[k] = ii[g + k];
      }
      const int o0 = t[0];
      if (g == 0) t[0] = first;
      step8x8(prev, acc, jp, o0, t, i8, r);
      jp = jj[g + 7];
      prev = r[7];
#pragma unroll
      for (int k = 0; k < 8; ++k) jj[g + k] = r[k];
    }
    acc |= (uint32_t)(prev ^ jp);
  }

  // steps8 without change bits (step8x8n).
  __device__ static void steps8n(int& prev, int first, int (&jj)[B], const int (&ii)[B]) {
#pragma unroll
    for (int g = 0; g < B; g += 8) {
      int t[8], i8[8], r[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        t[k] = jj[g + k];
        i8[k] = ii[g + k];
      }
      if (g == 0) t[0] = first;
      step8x8n(prev, t, i8, r);
      prev = r[7];
#pragma unroll
      for (int k = 0; k < 8; ++k) jj[g + k] = r[k];
    }
  }

  // TRACK false: no change bits (d0 and d1 are left alone).
  template <int D, bool TRACK = true>
  __device__ static void pass_vert(L& s, uint64_t& d0, uint64_t& d1) {
    const int x = lane();
    const int ys = D > 0 ? 0 : TH - 1;
    const int fx = x == 0 ? -1 : (x == TW - 1 ? TW : x);
    int prev = jv(s, ys - D, x);
    int corner = CONN == 8 ? jv(s, ys - D, fx) : LO;  // other lanes: their own column
    auto fetch = [&](int kb, int (&jj)[B], int (&ii)[B]) {
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int y = ys + D * (kb + k);
        jj[k] = jv(s, y, x);
        ii[k] = iv(s, y, x);
      }
    };
    auto work = [&](int kb, int (&jj)[B], const int (&ii)[B]) {
      uint32_t acc = 0;
      if constexpr (CONN == 8 && !TRACK) {
        steps8n(prev, imax(jj[0], corner), jj, ii);
      } else if constexpr (CONN == 8) {
        steps8(prev, acc, imax(jj[0], corner), jj, ii);
      } else {
#pragma unroll
        for (int k = 0; k < B; ++k) {
          if (CONN == 8)
            prev = imin(max8(prev, k == 0 ? imax(jj[0], corner) : jj[k]), ii[k]);
          else
            prev = imin(imax(jj[k], prev), ii[k]);
          if (TRACK) acc |= (uint32_t)(prev ^ jj[k]);
          jj[k] = prev;
        }
      }
      corner = LO;
#pragma unroll
      for (int k = 0; k < B; ++k) s.J[G::at(ys + D * (kb + k), x)] = (T)jj[k];
      if (TRACK && __ballot(acc != 0u)) {
        // rows kb .. kb + B - 1 of the pass, i.e. this block of tile rows
        const int y0 = D > 0 ? kb : TH - kb - B;
        const uint64_t blk = ((1ull << B) - 1) << (y0 & 63);
        if (y0 < 64)
          d0 |= blk;
        else
          d1 |= blk;
      }
    };
    int ja[B], ia[B], jb[B], ib[B];
    fetch(0, ja, ia);
    // up to 64 rows the loop is unrolled: no value is carried round it, so
    // the compiler keeps knowing that uint8 values need no masking
#pragma unroll(TH <= 64 ? TH / (2 * B) : 1)
    for (int kb = 0; kb < TH; kb += 2 * B) {
      fetch(kb + B, jb, ib);
      work(kb, ja, ia);
      if (kb + 2 * B < TH) fetch(kb + 2 * B, ja, ia);
      work(kb + B, jb, ib);
    }
  }

  // A 16-column block of a uint8, 8-connected horizontal pass, in one asm
  // block: columns c0 .. c0 + 15 of one row, held packed four to a dword
  // (byte e of the block is byte e % 4 of dword e / 4), worked in
  // increasing (D = +1) or decreasing (D = -1) column order.  Each step is
  // five instructions: b = max(p, J), the packing of the step before's
  // result into `ow`, two DPP maxima with the lanes beside, p = min(b, I).
  // The packing sits between the write of p and its DPP reads, which then
  // come two wait states after it; the first step has an s_nop there
  // instead, and an s_nop after the last packing keeps the next reader of
  // `ow` a wait state away from that partial write.
#define IWPP_HS(JW, S) "v_max_i32_sdwa %1, %0, %" #JW " dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_" #S "\n\t"
#define IWPP_HP(OW, S) "v_mov_b32_sdwa %" #OW ", %0 dst_sel:BYTE_" #S " dst_unused:UNUSED_PRESERVE src0_sel:DWORD\n\t"
#define IWPP_HT(IW, S)                                                 \
  "v_max_i32_dpp %1, %0, %1 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t" \
  "v_max_i32_dpp %1, %0, %1 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t" \
  "v_min_i32_sdwa %0, %1, %" #IW " dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_" #S "\n\t"
#define IWPP_NOP "s_nop 0\n\t"
  template <int D>
  __device__ static void hblock_u8(int& p, const uint32_t (&jw)[4], const uint32_t (&iw)[4],
                                   uint32_t (&ow)[4]) {
    int b;
    if constexpr (D > 0) {
      asm(
          IWPP_HS(6, 0) IWPP_NOP IWPP_HT(10, 0)
          IWPP_HS(6, 1) IWPP_HP(2, 0) IWPP_HT(10, 1)
          IWPP_HS(6, 2) IWPP_HP(2, 1) IWPP_HT(10, 2)
          IWPP_HS(6, 3) IWPP_HP(2, 2) IWPP_HT(10, 3)
          IWPP_HS(7, 0) IWPP_HP(2, 3) IWPP_HT(11, 0)
          IWPP_HS(7, 1) IWPP_HP(3, 0) IWPP_HT(11, 1)
          IWPP_HS(7, 2) IWPP_HP(3, 1) IWPP_HT(11, 2)
          IWPP_HS(7, 3) IWPP_HP(3, 2) IWPP_HT(11, 3)
          IWPP_HS(8, 0) IWPP_HP(3, 3) IWPP_HT(12, 0)
          IWPP_HS(8, 1) IWPP_HP(4, 0) IWPP_HT(12, 1)
          IWPP_HS(8, 2) IWPP_HP(4, 1) IWPP_HT(12, 2)
          IWPP_HS(8, 3) IWPP_HP(4, 2) IWPP_HT(12, 3)
          IWPP_HS(9, 0) IWPP_HP(4, 3) IWPP_HT(13, 0)
          IWPP_HS(9, 1) IWPP_HP(5, 0) IWPP_HT(13, 1)
          IWPP_HS(9, 2) IWPP_HP(5, 1) IWPP_HT(13, 2)
          IWPP_HS(9, 3) IWPP_HP(5, 2) IWPP_HT(13, 3)
          IWPP_HP(5, 3) IWPP_NOP
          : "+v"(p), "=&v"(b), "+v"(ow[0]), "+v"(ow[1]), "+v"(ow[2]), "+v"(ow[3])
          : "v"(jw[0]), "v"(jw[1]), "v"(jw[2]), "v"(jw[3]), "v"(iw[0]), "v"(iw[1]), "v"(iw[2]),
            "v"(iw[3]));
    } else {
      asm(
          IWPP_HS(9, 3) IWPP_NOP IWPP_HT(13, 3)
          IWPP_HS(9, 2) IWPP_HP(5, 3) IWPP_HT(13, 2)
          IWPP_HS(9, 1) IWPP_HP(5, 2) IWPP_HT(13, 1)
          IWPP_HS(9, 0) IWPP_HP(5, 1) IWPP_HT(13, 0)
          IWPP_HS(8, 3) IWPP_HP(5, 0) IWPP_HT(12, 3)
          IWPP_HS(8, 2) IWPP_HP(4, 3) IWPP_HT(12, 2)
          IWPP_HS(8, 1) IWPP_HP(4, 2) IWPP_HT(12, 1)
          IWPP_HS(8, 0) IWPP_HP(4, 1) IWPP_HT(12, 0)
          IWPP_HS(7, 3) IWPP_HP(4, 0) IWPP_HT(11, 3)
          IWPP_HS(7, 2) IWPP_HP(3, 3) IWPP_HT(11, 2)
          IWPP_HS(7, 1) IWPP_HP(3, 2) IWPP_HT(11, 1)
          IWPP_HS(7, 0) IWPP_HP(3, 1) IWPP_HT(11, 0)
          IWPP_HS(6, 3) IWPP_HP(3, 0) IWPP_HT(10, 3)
          IWPP_HS(6, 2) IWPP_HP(2, 3) IWPP_HT(10, 2)
          IWPP_HS(6, 1) IWPP_HP(2, 2) IWPP_HT(10, 1)
          IWPP_HS(6, 0) IWPP_HP(2, 1) IWPP_HT(10, 0)
          IWPP_HP(2, 0) IWPP_NOP
          : "+v"(p), "=&v"(b), "+v"(ow[0]), "+v"(ow[1]), "+v"(ow[2]), "+v"(ow[3])
          : "v"(jw[0]), "v"(jw[1]), "v"(jw[2]), "v"(jw[3]), "v"(iw[0]), "v"(iw[1]), "v"(iw[2]),
            "v"(iw[3]));
    }
  }
#undef IWPP_HS
#undef IWPP_HP
#undef IWPP_HT
#undef IWPP_NOP

  // Right (D = +1) or left (D = -1) pass, one lane per row, in groups of 64
  // rows: each pixel takes min(I, max(J, the three pixels of the previous
  // column around it)).  The halo rows above and below the tile are left to
  // the vertical passes (see above).  In tiles of more than 64 rows, lane 0
  // also takes the row above its group and lane 63 the row below it
  // (`fprev`; other lanes read their own row there, an old value that never
  // exceeds `prev`): the diagonal relations between a halo column and the
  // first or last row of a group are reached by no other pass.  In 32-row
  // tiles lanes 32..63 follow the halo row below the tile: what they compute
  // is min(I, max of valid lower bounds of R), itself a valid lower bound of
  // R, which is all lane 31 needs from its lower neighbour; they write
  // nothing.
  template <int D, bool TRACK = true>
  __device__ static void pass_horz(L& s, uint64_t& d0, uint64_t& d1) {
#pragma unroll 1
    for (int g = 0; g < TH; g += 64) {
      const int nrows = TH - g < 64 ? TH - g : 64;
      const bool live = lane() < nrows;
      const int yc = live ? g + lane() : TH;
      const int xs = D > 0 ? 0 : TW - 1;
      constexpr bool kFill = CONN == 8 && TH > 64;
      const int fy = lane() == 0 ? g - 1 : (lane() == 63 && live ? g + 64 : yc);
      int prev = jv(s, yc, xs - D);
      int fprev = kFill ? jv(s, fy, xs - D) : LO;
      uint32_t acc = 0;
      if constexpr (CONN == 8 && sizeof(T) == 1 && !kFill && B == 16) {
        // packed blocks of 16 columns, one b128 read of J and of I each
#pragma unroll 1
        for (int kb = 0; kb < TW; kb += B) {
          const int c0 = D > 0 ? kb : TW - B - kb;
          uint32_t jw[4], iw[4], ow[4] = {0u, 0u, 0u, 0u};
          __builtin_memcpy(jw, &s.J[G::at(yc, c0)], 16);
          __builtin_memcpy(iw, &s.I[G::at(yc, c0)], 16);
          hblock_u8<D>(prev, jw, iw, ow);
          acc |= (ow[0] ^ jw[0]) | (ow[1] ^ jw[1]) | (ow[2] ^ jw[2]) | (ow[3] ^ jw[3]);
          if (live) __builtin_memcpy(&s.J[G::at(yc, c0)], ow, 16);
        }
      } else {
#pragma unroll 1
      for (int kb = 0; kb < TW; kb += B) {
        int jj[B], ii[B], ff[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
          const int x = xs + D * (kb + k);
          jj[k] = jv(s, yc, x);
          ii[k] = iv(s, yc, x);
          if (kFill) ff[k] = jv(s, fy, x);
        }
        if constexpr (CONN == 8 && !kFill && !TRACK) {
          steps8n(prev, jj[0], jj, ii);
        } else if constexpr (CONN == 8 && !kFill) {
          steps8(prev, acc, jj[0], jj, ii);
        } else {
#pragma unroll
          for (int k = 0; k < B; ++k) {
            if (kFill) {
              prev = imin(max8(prev, imax(jj[k], fprev)), ii[k]);
              fprev = ff[k];
            } else {
              prev = imin(imax(jj[k], prev), ii[k]);
            }
            if (TRACK) acc |= (uint32_t)(prev ^ jj[k]);
            jj[k] = prev;
          }
        }
        if (live) {
#pragma unroll
          for (int k = 0; k < B; ++k) s.J[G::at(yc, xs + D * (kb + k))] = (T)jj[k];
        }
      }
      }
      if (TRACK) {
        const uint64_t b = __ballot(live && acc != 0u);
        if (g == 0)
          d0 |= b;
        else
          d1 |= b;
      }
      wsync();
    }
  }
  // Pass p of a round (0 down, 1 up, 2 right, 3 left); true if it changed a
  // pixel.  The rows it changed are marked in rowdirty.
  __device__ static bool run_pass(L& s, int p) {
    uint64_t d0 = 0, d1 = 0;
    if (p == 0) {
      pass_vert<+1>(s, d0, d1);
      wsync();
    } else if (p == 1) {
      pass_vert<-1>(s, d0, d1);
      wsync();
    } else if (p == 2) {
      pass_horz<+1>(s, d0, d1);
    } else {
      pass_horz<-1>(s, d0, d1);
    }
    for (int y = lane(); y < TH; y += 64)
      if ((y < 64 ? (d0 >> y) : (d1 >> (y - 64))) & 1ull) s.rowdirty[y] = 1;
    return (d0 | d1) != 0;
  }

  // One round of the four passes without change bits: every row counts as
  // changed (the caller writes them all back) and the round as one that
  // left work, so a scan of receivers follows.
  __device__ static void untracked_round(L& s) {
    uint64_t d0 = 0, d1 = 0;
    pass_vert<+1, false>(s, d0, d1);
    wsync();
    pass_vert<-1, false>(s, d0, d1);
    wsync();
    pass_horz<+1, false>(s, d0, d1);
    pass_horz<-1, false>(s, d0, d1);
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 1;
  }

  // Up to `budget` rounds of passes.  A pass that changes nothing leaves the
  // tile as it was, so four passes in a row that change nothing (one per
  // direction, in any cyclic order) all saw the same tile: it is then at a
  // fixed point for its halo, and this returns true without running the
  // rest of the round and a whole confirming round.
  // uint8 tiles, whose rounds are long, also keep the seams moving while
  // they work (both make a visit's chain of tile hops shorter):
  // - after a round that left work, `early`: if the tile's border now
  //   raises a neighbour, stop here (kEarly) so that the caller publishes
  //   the border and resumes;
  // - after a round that left work, a neighbour's request on the tile's
  //   state word (`watch`; null for none) is taken now: the halo is re-read
  //   and the rounds go on, instead of a re-run after this visit.
  static constexpr bool kStreaming = sizeof(T) == 1;
  // int32 8-connected tiles of 32 rows: first visits run their round without
  // change bits (see solve)
  static constexpr bool kUntrackedFirst = sizeof(T) == 4 && CONN == 8 && TH == 32;
  enum { kRoundsLeft = 0, kFixed = 1, kEarly = 2 };
  __device__ static int sweep_rounds(L& s, int budget, int first_pass, VisitStats& vs,
                                     uint32_t* watch, const DevImage& im, int64_t y0, int64_t x0,
                                     const KParams& kp, int64_t t, int64_t tx, int sides,
                                     bool early) {
    int quiet = 0, k = 0;
    int res = kRoundsLeft;
    // Each pass is idempotent: right after it, running it again changes
    // nothing.  Bit p of `stale` is set while the tile or its halo may have
    // changed since pass p last ran; a pass whose bit is clear is a no-op
    // and counts as quiet without running (the pass that would confirm the
    // fixed point at the end of a solve, most often).
    uint32_t stale = 0xFu;
    for (; k < 4 * budget && quiet < 4; ++k) {
      const int p = (first_pass + k) & 3;
      if ((stale >> p & 1u) && run_pass(s, p)) {
        quiet = 0;
        stale = 0xFu;
      } else {
        ++quiet;
      }
      stale &= ~(1u << p);
      if (kStreaming && watch && (k & 3) == 3 && quiet < 4) {
        int amax;
        if (early && activation_mask(s, y0, x0, false, amax) != 0u) {
          res = kEarly;
          ++k;
          break;
        }
        if (take_request(watch, peek_request(watch))) {
          refresh_halo(s, im, y0, x0, kp, t, tx, sides);
          quiet = 0;
          stale = 0xFu;
        }
      }
    }
    vs.rounds += (uint32_t)((k + 3) / 4);
    // with no pass stale, every pass has seen the tile as it is now: it is
    // at its fixed point even if the budget ran out before four quiet passes
    return (quiet >= 4 || stale == 0u) ? kFixed : res;
  }

  // ---------------------------------------------------------- seeds
  __device__ static int nbr_max(const L& s, int y, int x) {
    const int a = G::at(y, x);
    constexpr int P = G::P;
    int m = imax(imax((int)s.J[a - P], (int)s.J[a + P]), imax((int)s.J[a - 1], (int)s.J[a + 1]));
    if (CONN == 8)
      m = imax(m, imax(imax((int)s.J[a - P - 1], (int)s.J[a - P + 1]),
                       imax((int)s.J[a + P - 1], (int)s.J[a + P + 1])));
    return m;
  }

  // Every pixel a neighbour can still raise goes to queue 0; returns its
  // length.  One lane per column walks down the rows with rows y - 1, y and
  // y + 1 of J in registers (and, for lanes 0 and 63, the halo column beside
  // them, as in the passes); the columns beside come from the lanes beside.
  // A pixel's own value is part of the maximum, which changes nothing: the
  // test is whether the maximum exceeds it.  Each lane collects its
  // receivers as a bitmask over 32 rows; only the rows where some lane has
  // one are then compacted (ballot + mbcnt, in row order), since after a
  // round of passes most rows hold none.
  __device__ static int scan_receivers(L& s) {
    int n = 0;
    const int x = lane();
    const int fx = x == 0 ? -1 : (x == TW - 1 ? TW : x);
    int ja = jv(s, -1, x), jb = jv(s, 0, x);
    int fa = jv(s, -1, fx), fb = jv(s, 0, fx);
    constexpr int R = 8;
    static_assert(TH % 32 == 0, "receiver rows are gathered 32 at a time");
    uint32_t bits = 0;  // bit y % 32: pixel (y, x) is a receiver (see below)
#pragma unroll 1
    for (int yb = 0; yb < TH; yb += R) {
      int jn[R], fn[R], ii[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        jn[k] = jv(s, yb + k + 1, x);
        fn[k] = jv(s, yb + k + 1, fx);
        ii[k] = iv(s, yb + k, x);
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        int m;
        if (CONN == 8) {
          const int c = imax(imax(ja, jb), jn[k]);
          m = max_sides(imax(c, imax(imax(fa, fb), fn[k])), c);
        } else {
          m = max_sides(imax(imax(ja, jn[k]), fb), jb);
        }
        // a receiver iff min(m, I) > J; the bit goes in at the bottom and
        // the earlier rows move up (bits = 2 bits + carry, two instructions)
        const int mi = imin(m, ii[k]);
        asm("v_cmp_gt_i32 vcc, %1, %2\n\t"
            "v_addc_co_u32 %0, vcc, %0, %0, vcc"
            : "+v"(bits)
            : "v"(mi), "v"(jb)
            : "vcc");
        ja = jb;
        jb = jn[k];
        fa = fb;
        fb = fn[k];
      }
      // after each 32 rows: compact the rows that hold a receiver, in row
      // order (most rows hold none); bit 31 - y holds row y until reversed
      if (((yb + R) & 31) == 0) {
        bits = __builtin_bitreverse32(bits);
        const int g = (yb + R - 32) * TW + x;
        for (uint32_t rows = wave_or(bits); rows; rows &= rows - 1) {
          const int y = __builtin_ctz(rows);
          push(s, 0, n, (bits >> y) & 1u, g + y * TW);
        }
        bits = 0;
      }
    }
    wsync();
    return n;
  }

  // Border pixels that a neighbour in the halo can raise go to queue 0.
  // `first_pass` receives the pass that carries such a change inwards first
  // (0 down for a top row, 1 up for a bottom row, 2 right for a left column,
  // 3 left for a right column; the first of these that occurs).  The top and
  // bottom rows go one lane per column, corners included (lanes 0 and 63
  // also look at the halo column beside them); then the left and right
  // columns without their corners, one lane per pixel.
  __device__ static int halo_receivers(L& s, int& first_pass) {
    int n = 0;
    uint32_t sides = 0;
    {
      const int x = lane();
      const int fx = x == 0 ? -1 : (x == TW - 1 ? TW : x);
      // every read first, then the tests (one wait for all of them); lanes
      // 0 and 63 also take the halo column beside them
      int j[2], i[2], h[2], f[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int y = b == 0 ? 0 : TH - 1, hy = b == 0 ? -1 : TH, iy = b == 0 ? 1 : TH - 2;
        j[b] = jv(s, y, x);
        i[b] = iv(s, y, x);
        h[b] = jv(s, hy, x);
        if (CONN == 8) h[b] = imax(h[b], imax(jv(s, hy, x - 1), jv(s, hy, x + 1)));
        f[b] = jv(s, y, fx);
        if (CONN == 8) f[b] = imax(f[b], jv(s, iy, fx));
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int y = b == 0 ? 0 : TH - 1;
        const int hh = fx != x ? imax(h[b], f[b]) : h[b];
        const bool r = j[b] < i[b] && hh > j[b];
        if (r) sides |= (1u << b) | (x == 0 ? 4u : 0u) | (x == TW - 1 ? 8u : 0u);
        push(s, 0, n, r, y * TW + x);
      }
    }
    constexpr int NS = TH - 2;
    for (int base = 0; base < 2 * NS; base += 64) {
      const int e = base + lane();
      const bool right = e >= NS;
      const int y = 1 + (right ? e - NS : e);
      const int x = right ? TW - 1 : 0, hx = right ? TW : -1;
      // lanes past the last entry read row 1 and take nothing
      const int yr = e < 2 * NS ? y : 1;
      const int j = jv(s, yr, x), i = iv(s, yr, x);
      int h = jv(s, yr, hx);
      if (CONN == 8) h = imax(h, imax(jv(s, yr - 1, hx), jv(s, yr + 1, hx)));
      const bool r = e < 2 * NS && j < i && h > j;
      if (r) sides |= right ? 8u : 4u;
      push(s, 0, n, r, y * TW + x);
    }
    const uint32_t all = wave_or(sides);
    first_pass = all ? __builtin_ctz(all) : 0;
    wsync();
    return n;
  }

  // ---------------------------------------------------------- queue phase
  // Two-phase queue loop starting from n receivers in queue 0.  Returns
  // false when the queue ran dry (the tile is at a fixed point), true on
  // overflow or after `waves` waves with receivers left (then sweep rounds
  // and a scan must follow: a front that winds through the tile is carried
  // further by one round of passes than by many queue waves).
  // With `seam` (a seam visit), each wave first stages the rows its entries
  // and their neighbours lie on.
  __device__ static bool queue_loop(L& s, int n, VisitStats& vs, uint32_t waves,
                                    uint32_t iter_limit, bool& hit_limit, bool seam,
                                    const DevImage& im, int64_t y0, int64_t x0,
                                    const KParams& kp) {
    for (int w = lane(); w < G::NWORDS; w += 64) s.claim[w] = 0;
    wsync();
    for (uint32_t iter = 0;; ++iter) {
      if (n > G::QCAP) {
        vs.ovf++;
        return true;
      }
      if (n == 0) return false;
      if (iter >= waves) return true;
      if (iter >= iter_limit) {
        hit_limit = true;
        return false;
      }
      if constexpr (kSeamVisits) {
        if (seam) {  // false unless the caller compiled seam visits
          // rows y - 1 .. y + 1 of every entry
          uint32_t need = 0;
          for (int e = lane(); e < n; e += 64) {
            const int y = (s.q[0][e] & ~kRose) / TW;
            need |= (uint32_t)((7ull << y) >> 1);
          }
          if (need) atomicOr(&s.need, need);
          wsync();
          need = __builtin_amdgcn_readfirstlane(s.need);
          ensure_rows(s, im, y0, x0, kp, need & kAllRows);
        }
      }
      vs.iters++;
      vs.pushes += n;
      // propagation: each receiver updates only itself
      for (int e = lane(); e < n; e += 64) {
        const int idx = s.q[0][e];
        const int y = idx / TW, x = idx % TW;
        const int a = G::at(y, x);
        const int j = (int)s.J[a];
        const int v = imin(nbr_max(s, y, x), (int)s.I[a]);
        if (v > j) {
          s.J[a] = (T)v;
          s.rowdirty[y] = 1;
          s.q[0][e] = (uint16_t)(idx | kRose);
        }
      }
      wsync();
      // identification: neighbours of risen pixels that can now be raised,
      // each claimed once through the bitmap (all reads, then all claims,
      // then the compaction, so the LDS round trips overlap)
      int nn = 0;
#pragma unroll 1
      for (int base = 0; base < n; base += 64) {
        const int e = base + lane();
        int idx = 0, jp = LO;
        bool live = false;
        if (e < n) {
          const int q = s.q[0][e];
          live = (q & kRose) != 0;
          idx = q & ~kRose;
        }
        const int y = idx / TW, x = idx % TW;
        if (live) jp = (int)s.J[G::at(y, x)];
        constexpr int ND = CONN;
        int qi[ND], jq[ND], iq[ND];
        bool cand[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) {
          const int d = CONN == 8 ? (k < 4 ? k : k + 1) : (k == 0 ? 1 : k == 1 ? 3 : k == 2 ? 5 : 7);
          const int yy = y + d / 3 - 1, xx = x + d % 3 - 1;
          cand[k] = live && yy >= 0 && yy < TH && xx >= 0 && xx < TW;
          qi[k] = cand[k] ? yy * TW + xx : 0;
          const int a = G::at(qi[k] / TW, qi[k] % TW);
          jq[k] = (int)s.J[a];
          iq[k] = (int)s.I[a];
        }
        uint32_t old[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) {
          cand[k] = cand[k] && jq[k] < jp && jq[k] < iq[k];
          old[k] = atomicOr(&s.claim[qi[k] >> 5], cand[k] ? 1u << (qi[k] & 31) : 0u);
        }
#pragma unroll
        for (int k = 0; k < ND; ++k) {
          const bool win = cand[k] && !(old[k] & (1u << (qi[k] & 31)));
          push(s, 1, nn, win, qi[k]);
        }
      }
      wsync();
      n = nn;
      for (int w = lane(); w < G::NWORDS; w += 64) s.claim[w] = 0;
      if (n <= G::QCAP)
        for (int e = lane(); e < n; e += 64) s.q[0][e] = s.q[1][e];
      wsync();
    }
  }

  // ---------------------------------------------------------- visit
  // Bring the tile to a fixed point given its halo.  `seeded`: the tile was
  // at a fixed point for an older halo, so only border pixels next to a
  // changed halo pixel can rise at first.  `resume`: go on with rounds
  // after an early return.  `early`: the solve may return true before the
  // fixed point, once its border raises a neighbour (sweep_rounds).
  // Inlined into each caller: the counters and the limit flag then stay in
  // registers instead of scratch memory.
  template <bool SEAM = false>
  __device__ __forceinline__ static bool solve(L& s, int64_t y0, int64_t x0, int sweeps, bool seeded,
                               int seed_queue_max, uint32_t waves, uint32_t iter_limit,
                               VisitStats& vs, bool& hit_limit, uint32_t* watch,
                               const DevImage& im, const KParams& kp, int64_t t, int64_t tx,
                               int sides, bool resume, bool early) {
    int budget = sweeps;
    int first_pass = 0;
    // a seam visit (load_seam; only workers that make them compile SEAM) has
    // staged only part of the tile
    bool seam = false;
    if constexpr (SEAM && kSeamVisits)
      seam = __builtin_amdgcn_readfirstlane(s.loaded) != kAllRows;
    if (resume) {
      if (budget < 1) budget = 1;
    } else if (seeded) {
      const int n = halo_receivers(s, first_pass);
      if (n == 0) return false;
      if (n <= seed_queue_max) {
        if (!queue_loop(s, n, vs, waves, iter_limit, hit_limit, seam, im, y0, x0, kp))
          return false;
      }
      if (budget < 1) budget = 1;
    }
    // rounds of passes and scans read the whole tile
    if (seam) ensure_all_rows(s, im, y0, x0, kp);
    // A first visit of an int32 tile (the initial solve: neither seeded nor
    // resumed) with a budget of one round changes nearly every row, so its
    // round skips the per-step change bits, writes every row back, and goes
    // on to the scan as a round that left work would.
    bool untracked = kUntrackedFirst && !seeded && !resume && !early && budget == 1;
    for (uint32_t guard = 0;; ++guard) {
      if (untracked) {
        untracked_round(s);
        vs.rounds += 1;
        untracked = false;
      } else {
        const int r = sweep_rounds(s, budget, first_pass, vs, watch, im, y0, x0, kp, t, tx,
                                   sides, early);
        if (r == kFixed) return false;
        if (r == kEarly) return true;
      }
      const int n = scan_receivers(s);
      if (n == 0) return false;
      if (!queue_loop(s, n, vs, waves, iter_limit, hit_limit, false, im, y0, x0, kp))
        return false;
      if (budget < 1) budget = 1;
      if (guard >= iter_limit) {
        hit_limit = true;
        return false;
      }
    }
  }

  __device__ __forceinline__ static void clear_dirty(L& s) {
    for (int y = lane(); y < TH; y += 64) s.rowdirty[y] = 0;
    wsync();
  }

  // Neighbour tiles (3x3 grid index) that a changed border pixel can
  // propagate into.  Halo values are the ones seen at load time; they never
  // exceed the current ones, so no needed activation is missed.
  // With `want_max`, `amax` receives the largest value among the border
  // pixels that activate a neighbour (the class of the visit's fronts for
  // gray-level bands); the wavefront reduction is skipped otherwise.
  // Each side is checked against the halo pixels beyond it (the top and
  // bottom rows one lane per column, the left and right columns one lane
  // per row), so every pair of a border pixel and a halo neighbour is seen;
  // corner pixels are seen from both of their sides.
  __device__ __forceinline__ static uint32_t activation_mask(const L& s, int64_t, int64_t, bool want_max,
                                             int& amax) {
    uint32_t m = 0;
    int vmax = LO;
    constexpr int ND = CONN == 8 ? 3 : 1;  // halo pixels beside a border pixel
    // border pixel (value j, `changed` since the load) against halo pixel
    // (hy, hx) of value jh and mask value ih
    auto check = [&](bool changed, int j, int jh, int ih, int hy, int hx) {
      if (changed && j > jh && jh < ih) {
        const int cy = hy < 0 ? 0 : (hy >= TH ? 2 : 1);
        const int cx = hx < 0 ? 0 : (hx >= TW ? 2 : 1);
        m |= 1u << (cy * 3 + cx);
        vmax = imax(vmax, j);
      }
    };
    // every LDS read of a side is issued before the first test, so that they
    // share one wait
    {
      const int x = lane();
      const int jt = jv(s, 0, x), jb = jv(s, TH - 1, x);
      const int bt = (int)s.b_top[x], bb = (int)s.b_bot[x];
      int ht[ND], it[ND], hb[ND], ib[ND];
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        const int d = ND == 3 ? k - 1 : 0;
        ht[k] = jv(s, -1, x + d);
        it[k] = iv(s, -1, x + d);
        hb[k] = jv(s, TH, x + d);
        ib[k] = iv(s, TH, x + d);
      }
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        const int d = ND == 3 ? k - 1 : 0;
        check(jt != bt, jt, ht[k], it[k], -1, x + d);
        check(jb != bb, jb, hb[k], ib[k], TH, x + d);
      }
    }
    for (int y = lane(); y < TH; y += 64) {
      const int jl = jv(s, y, 0), jr = jv(s, y, TW - 1);
      const int bl = (int)s.b_left[y], br = (int)s.b_right[y];
      int hl[ND], il[ND], hr[ND], ir[ND];
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        const int d = ND == 3 ? k - 1 : 0;
        hl[k] = jv(s, y + d, -1);
        il[k] = iv(s, y + d, -1);
        hr[k] = jv(s, y + d, TW);
        ir[k] = iv(s, y + d, TW);
      }
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        const int d = ND == 3 ? k - 1 : 0;
        check(jl != bl, jl, hl[k], il[k], y + d, -1);
        check(jr != br, jr, hr[k], ir[k], y + d, TW);
      }
    }
    amax = LO;
    if (want_max) {
      for (int off = 32; off > 0; off >>= 1) vmax = imax(vmax, __shfl_xor(vmax, off));
      amax = __builtin_amdgcn_readfirstlane(vmax);
    }
    return wave_or(m);
  }

};

template <typename T, int CONN, int TH>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_persistent(
    DevImage one, const DevImage* __restrict__ imgs,
                                                   KParams kp, DevCtl* ctl, int* queue,
                                                   uint32_t* state, uint8_t* visited) {
  persistent_worker<Tile<T, CONN, TH>>(one, imgs, kp, ctl, queue, state, visited);
}

// The same worker with the next tile's loads in flight during the current
// tile's write-back (32-row int32 tiles; plain launches only, see
// prefetch_worker).
template <typename T, int CONN, int TH>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_persistent_pf(
    DevImage one, const DevImage* __restrict__ imgs, KParams kp, DevCtl* ctl, int* queue,
    uint32_t* state, uint8_t* visited) {
  if constexpr (Tile<T, CONN, TH>::kPrefetch)
    prefetch_worker<Tile<T, CONN, TH>>(one, imgs, kp, ctl, queue, state, visited);
}

// ------------------------------------------------------------ host-driven rounds

// One round: every active tile is visited once; tiles it activates are
// flagged for the next round.  Workgroups are mapped so that each XCD (the
// dispatcher deals workgroups to the 8 XCDs in turn) gets a contiguous run
// of tiles, keeping neighbouring tiles under one L2.
template <typename T, int CONN, int TH>
__global__ __launch_bounds__(64) void k_round(DevImage one, const DevImage* __restrict__ imgs,
                                              KParams kp, DevCtl* ctl, uint8_t* act_cur,
                                              uint8_t* act_next, uint8_t* visited) {
  using TP = Tile<T, CONN, TH>;
  __shared__ typename TP::L s;
  const int64_t per = (kp.ntiles + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= kp.ntiles || !act_cur[t]) return;
  const int k = imgs ? image_of(kp, imgs, t) : 0;
  const DevImage im = imgs ? imgs[k] : one;
  const int64_t tl = t - im.tile_base;
  const int64_t ty = tl / im.tiles_x, tx = tl % im.tiles_x;
  const int64_t y0 = ty * TH, x0 = tx * TW;
  const bool first = visited[t] == 0;
  VisitStats vs;
  bool hit = false;
  const bool viol = TP::load(s, im, y0, x0, first, kp, t, tx, 0);
  TP::solve(s, y0, x0, kp.sweeps, !first, kp.seed_queue_max, kp.queue_waves, kp.spin_limit,
            vs, hit, nullptr, im, kp, t, tx, 0, false, false);
  TP::store(s, im, y0, x0, kp, t, first);
  int amax = 0;
  const uint32_t act = TP::activation_mask(s, y0, x0, false, amax);
  if (threadIdx.x == 0) {
    WorkerStats ws;
    ws.add(vs);
    ws.visits = 1;
    if (viol) atomicOr((int*)&ctl->status.v, ST_MARKER_GT_MASK);
    if (hit) atomicOr((int*)&ctl->status.v, ST_INTERNAL);
    ws.flush(ctl);
    bool any = false;
    for (int d = 0; d < 9; ++d) {
      if (!((act >> d) & 1u)) continue;
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

// Reset the control block, per-tile state and the queue rings.
__global__ void k_init(KParams kp, DevCtl* ctl, int* queue, uint32_t* state, uint8_t* visited,
                       uint8_t* active) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = gid; i < kp.ntiles; i += stride) {
    // a list launch (gray-level bands after the first) keeps the tile states
    // (all idle after the previous launch) and the first-visit flags; its
    // listed tiles are marked pending by k_list_mark
    if (!kp.list_mode) {
      if (state) state[i] = TS_PENDING;
      visited[i] = 0;
      if (kp.band >= 0) {
        kp.dclass[i] = -1;
        kp.listed[i] = 0;
      }
    }
    if (active) active[i] = 1;
  }
  if (queue) {
    const int64_t n = (int64_t)kp.nq * kp.qcap;
    for (int64_t i = gid; i < n; i += stride) queue[i] = kSlotEmpty;
  }
  // the control block: one 32-bit word per thread of the first workgroup
  uint32_t* w = (uint32_t*)ctl;
  const int nw = (int)(sizeof(DevCtl) / 4);
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0;
    __syncthreads();
    // first-pass chunks are counted from 0; ring tickets and ring positions
    // both start after the first pass
    if (threadIdx.x < kMaxQueues && queue && threadIdx.x < kp.nq) {
      ctl->fphead[threadIdx.x].v = 0u;
      ctl->head[threadIdx.x].v = (uint32_t)first_pass_len(kp, threadIdx.x);
      ctl->tail[threadIdx.x].v = (uint32_t)first_pass_len(kp, threadIdx.x);
    }
    if (threadIdx.x == 0) {
      ctl->pending.v = state ? (uint32_t)(kp.list_mode ? kp.list_len : kp.ntiles) : 0u;
      ctl->max_deferred.v = 0xFFFFFFFFu;  // -1: nothing deferred
    }
  }
}

// Gray-level bands: the tiles of this launch's list start pending, and may
// enter the next launch's list again.
__global__ void k_list_mark(KParams kp, uint32_t* state) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kp.list_len; i += stride) {
    const int t = kp.list_in[i];
    state[t] = TS_PENDING;
    kp.listed[t] = 0;
  }
}

// Smallest and largest marker value in the tile order (after the complement
// of an erosion), for the class boundaries of gray-level bands.
template <typename T>
__global__ __launch_bounds__(256) void k_minmax(const T* __restrict__ J, int64_t H, int64_t W,
                                                int64_t ld, uint32_t flip, int* out) {
  int lo = INT_MAX, hi = INT_MIN;
  for (int64_t y = blockIdx.y; y < H; y += gridDim.y)
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < W;
         x += (int64_t)gridDim.x * 256) {
      const int v = (int)(T)(J[y * ld + x] ^ (T)flip);
      lo = imin(lo, v);
      hi = imax(hi, v);
    }
  for (int off = 32; off > 0; off >>= 1) {
    lo = imin(lo, __shfl_xor(lo, off));
    hi = imax(hi, __shfl_xor(hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&out[0], lo);
    atomicMax(&out[1], hi);
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
  X(int32_t, 4, 32)      \
  X(int32_t, 8, 32)      \
  X(int32_t, 4, 64)      \
  X(int32_t, 8, 64)

static int dtype_of(uint8_t*) { return 0; }
static int dtype_of(int32_t*) { return 1; }

bool variant_supported(const Variant& v) {
  if (v.dtype == kDtypeEdt) return edt_variant_supported(v.conn, v.tile_h);
#define X(T, C, H) \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) return true;
  IWPP_VARIANTS(X)
#undef X
  return false;
}

hipError_t launch_persistent(const Variant& v, const DevImage& one, const DevImage* imgs,
                             const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                             uint8_t* visited, int grid, hipStream_t st) {
  if (v.dtype == kDtypeEdt)
    return launch_persistent_edt(v.conn, v.tile_h, one, kp, ctl, queue, state, visited, grid,
                                 st);
  // plain launches of the tiles that prefetch take the prefetching worker
  const bool pf = kp.band < 0 && kp.max_visits == 0;
#define X(T, C, H)                                                                          \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) {                   \
    if (pf && Tile<T, C, H>::kPrefetch)                                                     \
      hipLaunchKernelGGL((k_persistent_pf<T, C, H>), dim3(grid), dim3(kThreads), 0, st,     \
                         one, imgs, kp, ctl, queue, state, visited);                        \
    else                                                                                    \
      hipLaunchKernelGGL((k_persistent<T, C, H>), dim3(grid), dim3(kThreads), 0, st, one,   \
                         imgs, kp, ctl, queue, state, visited);                             \
    return hipGetLastError();                                                               \
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
#define X(T, C, H)                                                                            \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) {                     \
    hipLaunchKernelGGL((k_round<T, C, H>), dim3(grid), dim3(kThreads), 0, st, one, imgs, kp, \
                       ctl, act_cur, act_next, visited);                                      \
    return hipGetLastError();                                                                 \
  }
  IWPP_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int persistent_blocks_per_cu(const Variant& v) {
  if (v.dtype == kDtypeEdt) return persistent_edt_blocks_per_cu(v.conn, v.tile_h);
  int nb = 0;
#define X(T, C, H)                                                                            \
  if (v.dtype == dtype_of((T*)nullptr) && v.conn == C && v.tile_h == H) {                     \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<T, C, H>, kThreads, 0) \
        != hipSuccess)                                                                        \
      return 0;                                                                               \
    return nb;                                                                                \
  }
  IWPP_VARIANTS(X)
#undef X
  return 0;
}

// Image index of every tile of a batch.
__global__ void k_tile_images(const DevImage* imgs, int nimg, int64_t ntiles, int32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += stride)
    out[t] = find_image(imgs, nimg, t);
}

hipError_t launch_tile_images(const DevImage* imgs, int nimg, int64_t ntiles, int32_t* out,
                              hipStream_t st) {
  int64_t blocks = (ntiles + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_tile_images, dim3((unsigned)blocks), dim3(256), 0, st, imgs, nimg, ntiles,
                     out);
  return hipGetLastError();
}

hipError_t launch_init(const KParams& kp, DevCtl* ctl, int* queue, uint32_t* state,
                       uint8_t* visited, uint8_t* active, hipStream_t st) {
  const int64_t ring = queue ? (int64_t)kp.nq * kp.qcap : 0;
  int64_t work = kp.ntiles > ring ? kp.ntiles : ring;
  int64_t blocks = (work + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, st, kp, ctl, queue, state,
                     visited, active);
  return hipGetLastError();
}

hipError_t launch_list_mark(const KParams& kp, uint32_t* state, hipStream_t st) {
  int64_t blocks = (kp.list_len + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_list_mark, dim3((unsigned)blocks), dim3(256), 0, st, kp, state);
  return hipGetLastError();
}

hipError_t launch_minmax(int dtype, const void* J, int64_t H, int64_t W, int64_t ld,
                         uint32_t flip, int* out, hipStream_t st) {
  int64_t gx = (W + 255) / 256, gy = H;
  if (gx > 16) gx = 16;
  if (gy > 1024) gy = 1024;
  const dim3 grid((unsigned)gx, (unsigned)gy);
  if (dtype == 0)
    hipLaunchKernelGGL(k_minmax<uint8_t>, grid, dim3(256), 0, st, (const uint8_t*)J, H, W, ld,
                       flip, out);
  else
    hipLaunchKernelGGL(k_minmax<int32_t>, grid, dim3(256), 0, st, (const int32_t*)J, H, W, ld,
                       flip, out);
  return hipGetLastError();
}

hipError_t launch_clear_round(DevCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_round, dim3(1), dim3(1), 0, st, ctl);
  return hipGetLastError();
}

// Fill-holes marker (the "Fill Holes" subsection of the IWPP chapter): the
// image itself on its 1-pixel frame and the highest value everywhere else;
// reconstruction by erosion of the image from it lowers every region that
// the frame reaches to what the frame lets through and leaves the holes (the
// regions it cannot reach) filled to the level of their surroundings.
template <typename T>
__global__ __launch_bounds__(256) void k_frame_marker(T* __restrict__ out,
                                                      const T* __restrict__ img, int64_t H,
                                                      int64_t W, int64_t ld) {
  for (int64_t y = blockIdx.y; y < H; y += gridDim.y) {
    const bool edge_row = y == 0 || y == H - 1;
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < W;
         x += (int64_t)gridDim.x * 256) {
      const bool frame = edge_row || x == 0 || x == W - 1;
      out[y * ld + x] = frame ? img[y * ld + x] : Highest<T>::v;
    }
  }
}

hipError_t launch_frame_marker(int dtype, void* out, const void* img, int64_t H, int64_t W,
                               int64_t ld, hipStream_t st) {
  int64_t gx = (W + 255) / 256, gy = H;
  if (gx > 64) gx = 64;
  if (gy > 65535) gy = 65535;
  const dim3 grid((unsigned)gx, (unsigned)gy);
  if (dtype == 0)
    hipLaunchKernelGGL(k_frame_marker<uint8_t>, grid, dim3(256), 0, st, (uint8_t*)out,
                       (const uint8_t*)img, H, W, ld);
  else
    hipLaunchKernelGGL(k_frame_marker<int32_t>, grid, dim3(256), 0, st, (int32_t*)out,
                       (const int32_t*)img, H, W, ld);
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
