/*
 * oracle.h -- sequential CPU reference for grayscale morphological
 * reconstruction by dilation (Gomes & Teodoro, "Efficient Execution of
 * Irregular Wavefront Propagation Pattern on Many Integrated Core
 * Architecture").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can check and time the GPU
 * library against a plain, obviously correct implementation.  It shares no
 * code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Images are row-major, H rows by W columns, contiguous (row pitch = W).
 * Pixel values are either uint8 (0..255) or int32 (full signed range).
 * Only max, min and comparisons are used, so nothing rounds or overflows.
 *
 * Status codes (returned by every entry point):
 */
#ifndef IWPP_ORACLE_H
#define IWPP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_MARKER_GT_MASK (-2)
#define ORACLE_E_NOMEM (-3)
#define ORACLE_E_INCOMPLETE (-5)

/* flags */
#define ORACLE_FLAG_CLAMP_MARKER 1u /* replace J by min(J, I) first instead of failing */

/* queue disciplines for the irregular propagation phase */
#define ORACLE_ORDER_FIFO 0   /* the paper's FIFO queue */
#define ORACLE_ORDER_LIFO 1   /* stack: a different legal order */
#define ORACLE_ORDER_RANDOM 2 /* uniformly random pop, seeded */

typedef struct oracle_stats {
  int64_t seeds;  /* pixels queued by the initialisation phase            */
  int64_t pushes; /* pixels queued by the propagation phase               */
  int64_t pops;   /* elements processed in the propagation phase          */
  int64_t iters;  /* whole-image iterations (brute force only)            */
} oracle_stats;

/*
 * Reconstruction, hybrid raster-scan + FIFO form (the paper's IWPP
 * reconstruction algorithm, Section "Reconstrucao Morfologica" of the IWPP
 * chapter).  J (marker) is reconstructed in place under mask I.
 *   conn      4 or 8
 *   flags     ORACLE_FLAG_*
 *   nsweeps   >= 1: that many raster/anti-raster pairs; the last anti-raster
 *             pass queues the paper's seeds.  0: no scans; the initial active
 *             set is every pixel that can still raise a neighbour (generic
 *             IWPP initialisation).
 *   order     ORACLE_ORDER_*; seed feeds ORACLE_ORDER_RANDOM
 *   max_pops  < 0: run to the fixed point.  >= 0: stop after that many pops
 *             and return ORACLE_E_INCOMPLETE (J is then a valid partial
 *             result: J0 <= J <= R).
 *   st        may be NULL
 * Returns ORACLE_E_MARKER_GT_MASK (J untouched) when J > I somewhere and the
 * clamp flag is not set.
 */
int oracle_reconstruct_u8(uint8_t *J, const uint8_t *I, int64_t H, int64_t W,
                          int conn, unsigned flags, int nsweeps, int order,
                          uint64_t seed, int64_t max_pops, oracle_stats *st);
int oracle_reconstruct_i32(int32_t *J, const int32_t *I, int64_t H, int64_t W,
                           int conn, unsigned flags, int nsweeps, int order,
                           uint64_t seed, int64_t max_pops, oracle_stats *st);

/*
 * Reconstruction by the definition: J <- dilate(J) ^ I over a copy of J,
 * repeated until no pixel changes (the paper's iterative reconstruction
 * algorithm and its Equation for the elementary step).  Assumes J <= I.
 */
int oracle_brute_u8(uint8_t *J, const uint8_t *I, int64_t H, int64_t W,
                    int conn, oracle_stats *st);
int oracle_brute_i32(int32_t *J, const int32_t *I, int64_t H, int64_t W,
                     int conn, oracle_stats *st);

/*
 * Reconstruction as a widest-path problem solved with a max-heap (the
 * priority-queue ordering the paper evaluates in "Uso de Diferentes
 * Estruturas de Dados"): every pixel is finalised the first time it leaves
 * the heap.  Assumes J <= I.
 */
int oracle_widest_u8(uint8_t *J, const uint8_t *I, int64_t H, int64_t W,
                     int conn, oracle_stats *st);
int oracle_widest_i32(int32_t *J, const int32_t *I, int64_t H, int64_t W,
                      int conn, oracle_stats *st);

/*
 * R at n single pixels (rows[k], cols[k]) without reconstructing the whole
 * image: a best-first search from each pixel over decreasing path
 * bottleneck, stopped once no unexplored path can beat the best marker value
 * found.  out[k] receives R.  max_visit > 0 bounds the pixels one query may
 * explore; a query that hits it gets out[k] = INT32_MIN (u8: -1) and the call
 * returns ORACLE_E_INCOMPLETE after finishing the other queries.
 */
int oracle_pixels_u8(const uint8_t *J, const uint8_t *I, int64_t H, int64_t W,
                     int conn, const int64_t *rows, const int64_t *cols,
                     int64_t n, int64_t max_visit, int32_t *out);
int oracle_pixels_i32(const int32_t *J, const int32_t *I, int64_t H,
                      int64_t W, int conn, const int64_t *rows,
                      const int64_t *cols, int64_t n, int64_t max_visit,
                      int32_t *out);

/*
 * Euclidean distance transform in IWPP form (the distance-transform
 * algorithm of the IWPP chapter, "Transformada de Distancia Euclidiana"):
 * pixels of `img` equal to 0 are background and are their own site VR;
 * object pixels start with no site.  The initialisation queues every
 * background pixel with an object neighbour; then a FIFO queue pops p and,
 * for each neighbour q whose distance to VR(p) is strictly below its
 * distance to VR(q), sets VR(q) = VR(p) and queues q.  Outputs:
 *   sites[p]  VR(p) packed (y << 16) | x, or -1 for no site;
 *   dist2[p]  squared Euclidean distance to VR(p), or -1 (may be NULL).
 * H and W are at most 32768.  st (may be NULL) counts queued and popped
 * pixels.
 */
int oracle_edt(const uint8_t *img, int64_t H, int64_t W, int conn, int32_t *sites,
               int64_t *dist2, oracle_stats *st);

#ifdef __cplusplus
}
#endif
#endif
