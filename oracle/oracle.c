/*
 * oracle.c -- sequential CPU reference for grayscale reconstruction by
 * dilation.  TEST INFRASTRUCTURE ONLY (see oracle.h): used by tests, the
 * smoke check and the benchmark's CPU-baseline leg; never by the library.
 *
 * Neighbourhoods (square grid G, Section "Notacoes em Algoritmos
 * Morfologicos"): 4-connected = the edge-adjacent pixels, 8-connected = edge
 * or corner adjacent.  N+(p) is the half visited before p in raster order
 * (upper-left half), N-(p) the half visited after it (lower-right half).
 * Neighbours outside the image do not exist.
 */
#include "oracle.h"

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int dy, dx;
} nbr_t;

static const nbr_t NPLUS8[4] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}};
static const nbr_t NMINUS8[4] = {{0, 1}, {1, -1}, {1, 0}, {1, 1}};
static const nbr_t NPLUS4[2] = {{-1, 0}, {0, -1}};
static const nbr_t NMINUS4[2] = {{0, 1}, {1, 0}};
static const nbr_t NALL8[8] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1},
                               {0, 1},   {1, -1}, {1, 0},  {1, 1}};
static const nbr_t NALL4[4] = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};

/* ---- growable ring buffer of pixel indices (FIFO / LIFO / random pop) ---- */
typedef struct {
  int64_t *buf;
  int64_t cap; /* power of two */
  int64_t head;
  int64_t n;
} queue_t;

static int queue_init(queue_t *q) {
  q->cap = 1024;
  q->head = 0;
  q->n = 0;
  q->buf = (int64_t *)malloc((size_t)q->cap * sizeof(int64_t));
  return q->buf ? 0 : -1;
}

static void queue_free(queue_t *q) {
  free(q->buf);
  q->buf = NULL;
}

static int queue_push(queue_t *q, int64_t v) {
  if (q->n == q->cap) {
    const int64_t ncap = q->cap * 2;
    int64_t *nb = (int64_t *)malloc((size_t)ncap * sizeof(int64_t));
    if (!nb) return -1;
    for (int64_t i = 0; i < q->n; ++i) nb[i] = q->buf[(q->head + i) & (q->cap - 1)];
    free(q->buf);
    q->buf = nb;
    q->cap = ncap;
    q->head = 0;
  }
  q->buf[(q->head + q->n) & (q->cap - 1)] = v;
  q->n++;
  return 0;
}

static int64_t queue_pop_front(queue_t *q) {
  const int64_t v = q->buf[q->head];
  q->head = (q->head + 1) & (q->cap - 1);
  q->n--;
  return v;
}

static int64_t queue_pop_back(queue_t *q) {
  q->n--;
  return q->buf[(q->head + q->n) & (q->cap - 1)];
}

/* splitmix64 (Steele, Lea & Flood, 2014) */
static uint64_t splitmix64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int64_t queue_pop_random(queue_t *q, uint64_t *rng) {
  const int64_t k = (int64_t)(splitmix64(rng) % (uint64_t)q->n);
  const int64_t at = (q->head + k) & (q->cap - 1);
  const int64_t v = q->buf[at];
  q->buf[at] = q->buf[q->head];
  q->head = (q->head + 1) & (q->cap - 1);
  q->n--;
  return v;
}

/* ---- binary max-heap of (key, pixel) ---- */
typedef struct {
  int64_t key;
  int64_t idx;
} heap_ent;

typedef struct {
  heap_ent *a;
  int64_t n, cap;
} heap_t;

static int heap_init(heap_t *h, int64_t cap) {
  if (cap < 16) cap = 16;
  h->a = (heap_ent *)malloc((size_t)cap * sizeof(heap_ent));
  h->n = 0;
  h->cap = cap;
  return h->a ? 0 : -1;
}

static void heap_free(heap_t *h) {
  free(h->a);
  h->a = NULL;
}

static void heap_down(heap_t *h, int64_t i) {
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && h->a[l].key > h->a[m].key) m = l;
    if (r < h->n && h->a[r].key > h->a[m].key) m = r;
    if (m == i) return;
    const heap_ent t = h->a[i];
    h->a[i] = h->a[m];
    h->a[m] = t;
    i = m;
  }
}

static void heap_make(heap_t *h) {
  for (int64_t i = h->n / 2 - 1; i >= 0; --i) heap_down(h, i);
}

static int heap_push(heap_t *h, int64_t key, int64_t idx) {
  if (h->n == h->cap) {
    const int64_t ncap = h->cap * 2;
    heap_ent *na = (heap_ent *)realloc(h->a, (size_t)ncap * sizeof(heap_ent));
    if (!na) return -1;
    h->a = na;
    h->cap = ncap;
  }
  int64_t i = h->n++;
  while (i > 0) {
    const int64_t par = (i - 1) / 2;
    if (h->a[par].key >= key) break;
    h->a[i] = h->a[par];
    i = par;
  }
  h->a[i].key = key;
  h->a[i].idx = idx;
  return 0;
}

static heap_ent heap_pop(heap_t *h) {
  const heap_ent top = h->a[0];
  h->a[0] = h->a[--h->n];
  heap_down(h, 0);
  return top;
}

#define OT uint8_t
#define OSUF u8
#include "oracle_body.inc"
#undef OT
#undef OSUF

#define OT int32_t
#define OSUF i32
#include "oracle_body.inc"
#undef OT
#undef OSUF

/* ------------------------------------------------------------------ EDT */

/* squared distance from pixel index p to site index v (W columns) */
static int64_t sq_dist(int64_t p, int64_t v, int64_t W) {
  const int64_t dy = p / W - v / W, dx = p % W - v % W;
  return dy * dy + dx * dx;
}

int oracle_edt(const uint8_t *img, int64_t H, int64_t W, int conn, int32_t *sites,
               int64_t *dist2, oracle_stats *st) {
  if (!img || !sites || H < 1 || W < 1 || H > 32768 || W > 32768) return ORACLE_E_ARG;
  if (conn != 4 && conn != 8) return ORACLE_E_ARG;
  const nbr_t *nb = conn == 8 ? NALL8 : NALL4;
  const int nn = conn;
  const int64_t N = H * W;
  /* VR as a pixel index, -1 for "no site" (infinitely far) */
  int64_t *vr = (int64_t *)malloc((size_t)N * sizeof(int64_t));
  if (!vr) return ORACLE_E_NOMEM;
  queue_t q;
  if (queue_init(&q)) {
    free(vr);
    return ORACLE_E_NOMEM;
  }
  int64_t seeds = 0, pushes = 0, pops = 0;
  /* initialisation phase */
  for (int64_t p = 0; p < N; ++p) vr[p] = img[p] == 0 ? p : -1;
  for (int64_t p = 0; p < N; ++p) {
    if (img[p] != 0) continue;
    const int64_t y = p / W, x = p % W;
    int has_object = 0;
    for (int k = 0; k < nn; ++k) {
      const int64_t yy = y + nb[k].dy, xx = x + nb[k].dx;
      if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      if (img[yy * W + xx] != 0) has_object = 1;
    }
    if (has_object) {
      if (queue_push(&q, p)) goto nomem;
      seeds++;
    }
  }
  /* irregular propagation phase */
  while (q.n > 0) {
    const int64_t p = queue_pop_front(&q);
    pops++;
    const int64_t y = p / W, x = p % W;
    for (int k = 0; k < nn; ++k) {
      const int64_t yy = y + nb[k].dy, xx = x + nb[k].dx;
      if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      const int64_t qi = yy * W + xx;
      /* DIST(q, VR(p)) < DIST(q, VR(q)); "no site" is infinitely far */
      if (vr[qi] < 0 || sq_dist(qi, vr[p], W) < sq_dist(qi, vr[qi], W)) {
        vr[qi] = vr[p];
        if (queue_push(&q, qi)) goto nomem;
        pushes++;
      }
    }
  }
  /* distance map from the Voronoi sites */
  for (int64_t p = 0; p < N; ++p) {
    if (vr[p] < 0) {
      sites[p] = -1;
      if (dist2) dist2[p] = -1;
    } else {
      sites[p] = (int32_t)(((vr[p] / W) << 16) | (vr[p] % W));
      if (dist2) dist2[p] = sq_dist(p, vr[p], W);
    }
  }
  if (st) {
    st->seeds = seeds;
    st->pushes = pushes;
    st->pops = pops;
    st->iters = 0;
  }
  queue_free(&q);
  free(vr);
  return ORACLE_OK;
nomem:
  queue_free(&q);
  free(vr);
  return ORACLE_E_NOMEM;
}
