/*
 * Driver for a sanitizer build of the CPU oracle (test infrastructure).
 * Runs every oracle entry point on small seeded inputs -- degenerate shapes,
 * both connectivities, both element types, every queue order, partial runs,
 * the error and clamp paths, single-pixel queries and the distance transform
 * -- and checks the three reconstruction forms against each other, so that a
 * memory or undefined-behaviour error shows up either in the sanitizer or as
 * a mismatch.  Exit status 0 when everything agrees.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) { /* splitmix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");              \
      failures++;                         \
    }                                     \
  } while (0)

static void case_u8(int64_t H, int64_t W, int conn, int lo_mask) {
  const int64_t n = H * W;
  uint8_t *I = malloc((size_t)n), *J = malloc((size_t)n), *R = malloc((size_t)n);
  uint8_t *B = malloc((size_t)n), *P = malloc((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    I[k] = (uint8_t)(lo_mask + next_u64() % (uint64_t)(256 - lo_mask));
    J[k] = (uint8_t)(next_u64() % ((uint64_t)I[k] + 1));
  }
  memcpy(B, J, (size_t)n);
  CHECK(oracle_brute_u8(B, I, H, W, conn, NULL) == ORACLE_OK, "brute u8");
  for (int order = 0; order < 3; ++order)
    for (int sweeps = 0; sweeps < 3; ++sweeps) {
      memcpy(R, J, (size_t)n);
      oracle_stats st;
      CHECK(oracle_reconstruct_u8(R, I, H, W, conn, 0, sweeps, order, 7, -1, &st) == ORACLE_OK,
            "reconstruct u8");
      CHECK(memcmp(R, B, (size_t)n) == 0, "u8 %lldx%lld conn %d order %d sweeps %d",
            (long long)H, (long long)W, conn, order, sweeps);
    }
  memcpy(P, J, (size_t)n);
  CHECK(oracle_widest_u8(P, I, H, W, conn, NULL) == ORACLE_OK, "widest u8");
  CHECK(memcmp(P, B, (size_t)n) == 0, "widest u8 differs");
  /* a partial run, then the rest */
  memcpy(R, J, (size_t)n);
  const int rc = oracle_reconstruct_u8(R, I, H, W, conn, 0, 1, 0, 0, n / 3, NULL);
  CHECK(rc == ORACLE_OK || rc == ORACLE_E_INCOMPLETE, "partial u8");
  CHECK(oracle_reconstruct_u8(R, I, H, W, conn, 0, 1, 0, 0, -1, NULL) == ORACLE_OK, "resume");
  CHECK(memcmp(R, B, (size_t)n) == 0, "restart u8 differs");
  /* single-pixel queries, including the corners */
  int64_t rows[4] = {0, H - 1, 0, H - 1}, cols[4] = {0, 0, W - 1, W - 1};
  int32_t out[4];
  CHECK(oracle_pixels_u8(J, I, H, W, conn, rows, cols, 4, 0, out) == ORACLE_OK, "pixels u8");
  for (int q = 0; q < 4; ++q) CHECK(out[q] == B[rows[q] * W + cols[q]], "pixel query u8");
  /* marker above the mask: error without clamp, min(J, I) with it */
  if (n > 0) {
    memcpy(R, J, (size_t)n);
    const int64_t k = (int64_t)(next_u64() % (uint64_t)n);
    if (I[k] < 255) {
      R[k] = (uint8_t)(I[k] + 1);
      CHECK(oracle_reconstruct_u8(R, I, H, W, conn, 0, 1, 0, 0, -1, NULL) ==
                ORACLE_E_MARKER_GT_MASK, "marker above mask u8");
      CHECK(oracle_reconstruct_u8(R, I, H, W, conn, ORACLE_FLAG_CLAMP_MARKER, 1, 0, 0, -1,
                                  NULL) == ORACLE_OK, "clamp u8");
    }
  }
  free(I); free(J); free(R); free(B); free(P);
}

static void case_i32(int64_t H, int64_t W, int conn) {
  const int64_t n = H * W;
  int32_t *I = malloc((size_t)n * 4), *J = malloc((size_t)n * 4), *R = malloc((size_t)n * 4);
  int32_t *B = malloc((size_t)n * 4), *P = malloc((size_t)n * 4);
  for (int64_t k = 0; k < n; ++k) {
    /* the full signed range, extremes included */
    const uint64_t r = next_u64();
    I[k] = (r % 7 == 0) ? INT32_MAX : (int32_t)(uint32_t)(r >> 32);
    const int64_t span = (int64_t)I[k] - (int64_t)INT32_MIN + 1;
    J[k] = (r % 11 == 0) ? INT32_MIN : (int32_t)((int64_t)INT32_MIN + (int64_t)(next_u64() % (uint64_t)span));
  }
  memcpy(B, J, (size_t)n * 4);
  CHECK(oracle_brute_i32(B, I, H, W, conn, NULL) == ORACLE_OK, "brute i32");
  for (int order = 0; order < 3; ++order) {
    memcpy(R, J, (size_t)n * 4);
    CHECK(oracle_reconstruct_i32(R, I, H, W, conn, 0, order == 1 ? 0 : 1, order, 3, -1, NULL) ==
              ORACLE_OK, "reconstruct i32");
    CHECK(memcmp(R, B, (size_t)n * 4) == 0, "i32 %lldx%lld conn %d order %d", (long long)H,
          (long long)W, conn, order);
  }
  memcpy(P, J, (size_t)n * 4);
  CHECK(oracle_widest_i32(P, I, H, W, conn, NULL) == ORACLE_OK, "widest i32");
  CHECK(memcmp(P, B, (size_t)n * 4) == 0, "widest i32 differs");
  int64_t rows[2] = {H / 2, H - 1}, cols[2] = {W / 2, 0};
  int32_t out[2];
  CHECK(oracle_pixels_i32(J, I, H, W, conn, rows, cols, 2, 0, out) == ORACLE_OK, "pixels i32");
  for (int q = 0; q < 2; ++q) CHECK(out[q] == B[rows[q] * W + cols[q]], "pixel query i32");
  free(I); free(J); free(R); free(B); free(P);
}

static void case_edt(int64_t H, int64_t W, int conn, unsigned object_pct) {
  const int64_t n = H * W;
  uint8_t *img = malloc((size_t)n);
  int32_t *sites = malloc((size_t)n * 4);
  int64_t *d2 = malloc((size_t)n * 8);
  for (int64_t k = 0; k < n; ++k) img[k] = (next_u64() % 100) < object_pct ? 1 : 0;
  CHECK(oracle_edt(img, H, W, conn, sites, d2, NULL) == ORACLE_OK, "edt");
  for (int64_t k = 0; k < n; ++k) {
    if (img[k] == 0) CHECK(d2[k] == 0, "background pixel not its own site");
    if (sites[k] >= 0) {
      const int64_t sy = sites[k] >> 16, sx = sites[k] & 0xFFFF;
      const int64_t dy = k / W - sy, dx = k % W - sx;
      CHECK(sy < H && sx < W && img[sy * W + sx] == 0, "site not background");
      CHECK(d2[k] == dy * dy + dx * dx, "distance does not match site");
    }
  }
  CHECK(oracle_edt(img, H, W, conn, sites, NULL, NULL) == ORACLE_OK, "edt without dist2");
  free(img); free(sites); free(d2);
}

int main(void) {
  const int64_t shapes[][2] = {{1, 1}, {1, 2}, {2, 1}, {1, 37}, {29, 1}, {2, 2},
                               {3, 5}, {7, 3}, {16, 16}, {33, 47}, {64, 65}};
  for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
    for (int conn = 4; conn <= 8; conn += 4) {
      case_u8(shapes[s][0], shapes[s][1], conn, 0);
      case_u8(shapes[s][0], shapes[s][1], conn, 200);
      case_i32(shapes[s][0], shapes[s][1], conn);
      case_edt(shapes[s][0], shapes[s][1], conn, 90);
      case_edt(shapes[s][0], shapes[s][1], conn, 100);
    }
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("oracle sanitizer driver: all cases agree\n");
  return 0;
}
