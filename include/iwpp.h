/*
 * iwpp.h -- C ABI of an MI355X (gfx950) library for grayscale morphological
 * reconstruction by dilation, computed as an irregular wavefront propagation
 * (IWPP): tile scans, wavefront-seed detection, queue-driven propagation to
 * a fixed point (Gomes & Teodoro, "Efficient Execution of Irregular
 * Wavefront Propagation Pattern on Many Integrated Core Architecture").
 *
 * The operation (background chapter, "Reconstrucao Morfologica", and its
 * reconstruction Equation): given a mask I and a marker J with J <= I
 * pixelwise, the reconstruction R_I(J) is the limit of J <- dilate_G(J) ^ I,
 * where dilate_G takes the maximum over a pixel and its neighbours on the
 * square grid G (4- or 8-connected, Section "Notacoes em Algoritmos
 * Morfologicos") and ^ is the pixelwise minimum.  The result is unique.
 *
 * Conventions shared by every entry point:
 *  - Images are 2-D, row-major, H rows by W columns, row pitch `ld` elements
 *    (ld >= W; 0 means W).  Pixel (y, x) is at element y*ld + x.
 *  - dtype IWPP_U8 (uint8, 0..255) or IWPP_I32 (int32, full range).  Paper
 *    runs use 32-bit integers; the arithmetic is max/min/compare only, so
 *    results are exact for both types.
 *  - `marker` and `mask` are DEVICE pointers owned by the caller; `marker`
 *    is overwritten with R in place (the output J of the IWPP reconstruction
 *    algorithm).  Marker and mask must not overlap.
 *  - Pixels outside the image do not exist (no padding value propagates).
 *  - Every function returns an IWPP_* status code; nothing throws.  Argument
 *    errors are detected on the host before any GPU work is queued.
 *  - Streams are hipStream_t values passed as void*; NULL is the null stream.
 *  - If J > I at some pixel the call reports IWPP_E_MARKER_GT_MASK; the
 *    marker then holds R_I(min(J, I)).  With IWPP_FLAG_CLAMP_MARKER the same
 *    result is produced and the call succeeds.
 *  - With IWPP_FLAG_EROSION the call computes the reconstruction by erosion
 *    instead (the "max/min" choice of the IWPP algorithm): J >= I, and J
 *    becomes the limit of J <- erode_G(J) v I (v the pixelwise maximum).  It
 *    runs the same kernels through duality: tiles hold the bitwise
 *    complement (255 - x for uint8, -1 - x for int32, both order-reversing),
 *    applied as values are staged and written back, so it moves no extra
 *    bytes.  Its precondition error is J < I somewhere (reported as
 *    IWPP_E_MARKER_GT_MASK of the complemented images); with
 *    IWPP_FLAG_CLAMP_MARKER the marker is max(J, I).
 *  - The library keeps a workspace per (device, stream), grown on demand and
 *    freed by iwpp_release_workspace().  Calls on one stream run in stream
 *    order; calls on different streams may run concurrently.  Its largest
 *    parts are per tile: a state word, a visited byte, an image index for
 *    batches, and the tile's first and last column of I and J (so that a
 *    neighbour reads them as one run): about 3% of the two images' bytes,
 *    plus the tile queues.
 */
#ifndef IWPP_H
#define IWPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define IWPP_OK 0
#define IWPP_E_ARG (-1)             /* invalid argument (host check)        */
#define IWPP_E_MARKER_GT_MASK (-2)  /* J > I somewhere (precondition)       */
#define IWPP_E_NOMEM (-3)           /* device or host allocation failed     */
#define IWPP_E_HIP (-4)             /* a HIP runtime call failed            */
#define IWPP_E_INCOMPLETE (-5)      /* stopped at max_tile_visits; marker is
                                       a valid partial result J <= J' <= R,
                                       and calling again completes it      */
#define IWPP_E_BUDGET (-6)          /* request exceeds the server budget    */
#define IWPP_E_INTERNAL (-7)        /* a bounded device wait ran out        */
#define IWPP_E_TIMEOUT (-8)         /* server wait timed out                */
#define IWPP_E_UNSUPPORTED (-9)     /* parameter combination not compiled   */
#define IWPP_E_SCRATCH (-10)        /* iwpp_reconstruct_noalloc: the image
                                       needs more workspace than its static
                                       array holds                         */

/* ---- element types ---- */
#define IWPP_U8 0
#define IWPP_I32 1

/* ---- flags ---- */
#define IWPP_FLAG_CLAMP_MARKER 1u /* use min(J, I) as the marker, no error */
#define IWPP_FLAG_EROSION 2u      /* reconstruction by erosion (see above)    */

typedef void *iwpp_stream_t;

typedef struct iwpp_image {
  void *marker;     /* device, in/out */
  const void *mask; /* device, in */
  int64_t H, W;     /* rows, columns (>= 1) */
  int64_t ld;       /* row pitch in elements; 0 means W */
} iwpp_image;

/* Work counters of the last call on a stream (or of a batch plan). */
typedef struct iwpp_stats {
  int32_t status;          /* IWPP_OK, _MARKER_GT_MASK, _INCOMPLETE or _INTERNAL  */
  int32_t images;          /* images in the call                                  */
  int64_t tiles;           /* tiles in the call                                   */
  int64_t tile_visits;     /* tile visits (first, re-activated and re-run)        */
  int64_t sweep_rounds;    /* rounds of the four directional passes              */
  int64_t pixels_queued;   /* queue entries processed: the paper's "elements
                              processed in the propagation phase"                 */
  int64_t queue_overflows; /* tile-queue overflows (each falls back to a scan)    */
  int64_t reprocessed;     /* tiles re-run in place after a neighbour changed     */
  int64_t requeued;        /* tiles put back on a work queue after their first visit */
  int64_t launches;        /* kernel launches                                     */
  double kernel_ms;        /* device time of the reconstruction kernels when
                              iwpp_params.timing was set, else 0                  */
  int64_t queue_iterations; /* identify/propagate pairs over all tile queues      */
  /* wavefront-milliseconds summed over the persistent workers: waiting for a
     tile, loading tiles, solving them, storing them, publishing them (release
     fence and tile-state updates) */
  double idle_ms, load_ms, solve_ms, store_ms, sync_ms;
} iwpp_stats;

/*
 * Execution parameters.  Zero fields take the library default (or the value
 * the autotuner stored for this problem class).
 *   tile_h        tile height in rows: 64 or 128 (u8), 32 or 64 (i32); tiles
 *                 are 64 columns wide, one wavefront per tile.
 *   sweeps        rounds of directional passes before switching a tile to its
 *                 queue (>= 0; -1 selects 0 explicitly).
 *   mode          0 persistent kernel with a global tile queue (default);
 *                 1 host-driven rounds (one launch per round, for comparison);
 *                 2 gray-level bands: the priority ordering of the paper's
 *                 "Uso de Diferentes Estruturas de Dados" at the granularity
 *                 of tiles and bands of values.  The marker's value range is
 *                 split into `bands` classes; a sequence of persistent
 *                 launches handles the classes from the highest down, each
 *                 queueing only the tile activations whose value lies in or
 *                 above its class and deferring the others to a later
 *                 launch.  Single images only (batched calls return
 *                 IWPP_E_UNSUPPORTED); one extra pass reads the marker for
 *                 its range, and the host waits once per launch.
 *   grid          persistent workgroups (0 = fill the device).
 *   max_tile_visits  stop after this many tile visits (0 = no limit); used to
 *                 test restart: the call then returns IWPP_E_INCOMPLETE.
 *   order_seed    0: the first visits go in four groups of tiles of
 *                 alternate rows and columns (no two tiles of a group
 *                 touch), in the order `first_pass` picks; otherwise a
 *                 seeded permutation of the tiles (results must not depend
 *                 on it).
 *   timing        non-zero: bracket the reconstruction kernels with HIP
 *                 events on the call's stream; iwpp_stats.kernel_ms then
 *                 reports their device time.
 *   seed_queue    a re-visited tile whose new halo can raise at most this
 *                 many border pixels goes straight to its queue; more start
 *                 with a scan round (0 = default: always scan for uint8, 8
 *                 for int32; -1 = always scan).
 *   queue_waves   a tile queue that still holds receivers after this many
 *                 waves hands the tile to rounds of directional passes and a
 *                 new scan (0 = default 4, -1 = no limit).
 *   bands         mode 2: number of gray-level classes (0 = default 16).
 *   first_pass    order of the four groups of first visits (order_seed 0):
 *                 1 by rows of the group grid -- (even row, even column),
 *                 (even, odd), (odd, even), (odd, odd) -- so that the second
 *                 group already starts beside finished tiles, which suits
 *                 fronts that travel from tile to tile (fill-holes); 2 the
 *                 two diagonal groups first -- (even, even), (odd, odd),
 *                 then (even, odd) and (odd, even) -- so that half the tiles
 *                 start with all four edge neighbours finished and few need
 *                 a re-visit, which suits fronts that stay local (h-domes).
 *                 0 = default: 1 for uint8, 2 for int32 and the distance
 *                 transform.  Results do not depend on it.
 */
typedef struct iwpp_params {
  int32_t tile_h;
  int32_t sweeps;
  int32_t mode;
  int32_t grid;
  int64_t max_tile_visits;
  uint32_t order_seed;
  uint32_t spin_limit; /* bound on device-side waits (0 = default) */
  int32_t timing;
  int32_t seed_queue;
  int32_t queue_waves;
  int32_t bands;
  int32_t first_pass;
} iwpp_params;

/* Library version, e.g. 10000 for 1.0.0. */
int iwpp_version(void);

/* Static description of a status code. */
const char *iwpp_strerror(int code);

/* Text of the last HIP error seen by this thread ("" if none). */
const char *iwpp_last_error(void);

/*
 * Synchronous reconstruction on the null stream (IWPP reconstruction
 * algorithm; operation defined above).  Returns the device status.
 */
int iwpp_reconstruct(void *marker, const void *mask, int64_t H, int64_t W, int dtype,
                     int conn);

/*
 * Asynchronous reconstruction of one image on `stream`.  Returns IWPP_OK once
 * the work is queued (or a host-side argument error).  The device status and
 * counters of the last call on that stream are read with
 * iwpp_stream_status().  `params` may be NULL.  In mode 1 (host-driven
 * rounds) the call synchronises the stream once per round.
 */
int iwpp_reconstruct_async(const iwpp_image *img, int dtype, int conn, uint32_t flags,
                           const iwpp_params *params, iwpp_stream_t stream);

/*
 * Waits for `stream`, then returns the status of the last reconstruction
 * queued on it and fills `stats` (may be NULL).
 */
int iwpp_stream_status(iwpp_stream_t stream, iwpp_stats *stats);

/*
 * Several independent images in one persistent launch (a task queue of image
 * tiles, as in the paper's cooperative execution, "Execucao Cooperativa em
 * Processadores Heterogeneos"): tiles of all images share one work queue and
 * fronts never cross from one image to another.  Asynchronous like
 * iwpp_reconstruct_async; the descriptor array is copied before returning.
 */
int iwpp_reconstruct_batched(const iwpp_image *imgs, int32_t n, int dtype, int conn,
                             uint32_t flags, const iwpp_params *params,
                             iwpp_stream_t stream);

/*
 * Reusable batch plan: descriptors, tile queue and per-tile state are
 * allocated once; iwpp_batch_launch() re-runs the batch (with use_graph != 0
 * the launch sequence is captured once into a HIP graph and replayed).  The
 * images' buffers must stay valid while the plan exists.  Parameters are
 * fixed at creation (NULL = defaults / autotuned values).
 */
typedef struct iwpp_batch iwpp_batch;
int iwpp_batch_create(const iwpp_image *imgs, int32_t n, int dtype, int conn, uint32_t flags,
                      const iwpp_params *params, iwpp_batch **out);
int iwpp_batch_launch(iwpp_batch *b, iwpp_stream_t stream, int use_graph);
/* Waits for the plan's last launch, returns its status and fills stats. */
int iwpp_batch_status(iwpp_batch *b, iwpp_stats *stats);
int iwpp_batch_destroy(iwpp_batch *b);

/*
 * Times candidate parameter sets on one image and returns the fastest in
 * *best (bit-exactness of every candidate is the caller's to test).  The
 * search is coordinate descent: tile height x sweeps, then seed_queue, then
 * queue_waves, each stage from the best set so far (about 19 candidates,
 * four runs each).  The
 * marker is left unchanged: candidates run on a scratch copy.  Results are
 * remembered per (dtype, conn, size class) and used when params are NULL;
 * if IWPP_TUNE_CACHE names a file, they are also stored there as JSON.
 */
int iwpp_autotune(const iwpp_image *img, int dtype, int conn, iwpp_stream_t stream,
                  iwpp_params *best);

/*
 * Continuous-batching server for reconstructions whose buffers already live
 * on the device (a serving loop built around the same kernels; it has no
 * counterpart in the paper).  A dispatcher thread admits pending requests in
 * arrival order while the device bytes they hold (marker, mask and their
 * tiles' share of the library workspace) fit in `budget_bytes` and fewer
 * than `max_inflight` requests are unfinished.  The requests admitted
 * together form one batched persistent launch on a free slot of `streams`
 * HIP streams; launches on different slots overlap on the device, so
 * requests that arrive while others run start as soon as a slot and memory
 * free up.  create allocates each slot's workspace for the most tiles the
 * budget admits at once (whole 64-column tiles: about 3% of the budget per
 * slot for uint8), so the dispatch path allocates and frees nothing.
 *   submit: non-blocking.  The buffers are the caller's and must stay valid
 *           until the request is waited for.  `stream` is the stream on
 *           which the caller produced them (NULL: the null stream): the
 *           request's work starts only after the work queued on it before
 *           submit (an event recorded there).  If `marker_init` is not NULL
 *           it is a device image with the marker's shape and row pitch that
 *           is copied into the marker (on the launch stream) before the
 *           reconstruction.  Returns IWPP_E_BUDGET if the request alone
 *           exceeds the budget.
 *   wait:   blocks until the request finishes (timeout_us < 0: forever;
 *           IWPP_E_TIMEOUT otherwise) and returns its status (the status of
 *           the launch it ran in); latency_us receives completion - submit
 *           time in microseconds.  A ticket can be waited for once.
 *   destroy: finishes every admitted and pending request, then frees.
 */
typedef struct iwpp_server iwpp_server;
int iwpp_server_create(size_t budget_bytes, int dtype, int conn, int streams,
                       int max_inflight, iwpp_server **out);
int iwpp_server_submit(iwpp_server *s, const iwpp_image *img, const void *marker_init,
                       iwpp_stream_t stream, uint64_t *ticket);
int iwpp_server_wait(iwpp_server *s, uint64_t ticket, int64_t timeout_us, double *latency_us);
int iwpp_server_destroy(iwpp_server *s);

/* Frees the cached per-stream workspaces (after synchronising the device). */
int iwpp_release_workspace(void);

/*
 * Fill holes ("Fill Holes" subsection of the IWPP chapter): `out` receives
 * the image with every hole filled, where a hole is a region the image's
 * 1-pixel frame cannot reach without climbing; a grayscale hole is raised to
 * the lowest level through which it can be left.  Computed as the
 * reconstruction by erosion of `image` from a marker equal to the image on
 * its frame and the highest value inside (equivalently, by duality, the
 * complement of the reconstruction by dilation of the complemented image
 * from its frame).  `image` (in) and `out` (out) are device arrays of H x W
 * pixels with row pitch `ld` (0 = W) that must not overlap.  Asynchronous
 * on `stream` like iwpp_reconstruct_async: one marker-initialisation kernel,
 * then the reconstruction; iwpp_stream_status() reports the result.
 */
int iwpp_fill_holes_async(const void *image, void *out, int64_t H, int64_t W, int64_t ld,
                          int dtype, int conn, const iwpp_params *params,
                          iwpp_stream_t stream);

/*
 * Euclidean distance transform as an irregular wavefront propagation ("Transformada de
 * Distancia Euclidiana" subsection of the IWPP chapter and its distance-transform
 * algorithm).  `image` is a uint8 device array (row pitch `ld_image`, 0 = W) whose 0
 * pixels are background and others object.  Every background pixel is its own site;
 * a pixel takes a neighbour's site (4- or 8-connected) whenever that site is strictly
 * closer in Euclidean distance, until nothing changes.  Outputs (int32 device arrays,
 * row pitch `ld_out`, 0 = W):
 *   sites  the site each pixel ended with, packed (y << 16) | x, or -1 if the image
 *          has no background pixel;
 *   dist2  (may be NULL) the squared Euclidean distance to that site, or -1.
 * Like the paper's algorithm this is the vector-propagation approximation of the exact
 * transform: each site is a background pixel and dist2 is exact for it, but a few pixels
 * may hold a site slightly farther than the nearest background pixel, and ties between
 * equally close sites may resolve differently from run to run.  H and W are at most
 * 32768.  Arrays must not overlap; the int32 arrays must be 4-byte aligned.  Only the
 * tile height 32 and the persistent mode exist (other values of tile_h or mode return
 * IWPP_E_UNSUPPORTED); `max_tile_visits`, `grid`, `order_seed`, `spin_limit` and
 * `timing` apply.  Asynchronous on `stream`; iwpp_stream_status() reports the result.
 */
int iwpp_edt_async(const void *image, int64_t ld_image, void *sites, void *dist2,
                   int64_t ld_out, int64_t H, int64_t W, int conn, const iwpp_params *params,
                   iwpp_stream_t stream);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the single-image
 * reconstruction of iwpp_reconstruct_async (same kernels, same result),
 * asynchronous on `stream`, allocating nothing.  Its library workspace
 * (control block, per-tile state and first-visit flags, tile-queue rings,
 * packed side columns) is carved from one static device array of
 * IWPP_NOALLOC_SCRATCH_BYTES (128 MiB) that every device the library runs on
 * holds until the process ends; its address is looked up once per device, on
 * the first call with that device current.  An image whose workspace would
 * not fit returns IWPP_E_SCRATCH before any GPU work (about 265 bytes per
 * 64 x 64 uint8 tile and 521 bytes per 64 x 32 int32 tile, plus the queue
 * rings of up to 8192 workgroups: up to about 2 Gpx uint8 or 0.5 Gpx int32).
 *   img, dtype, conn, flags, params: as for iwpp_reconstruct_async; the
 *     autotuner's stored values are not consulted, and only mode 0 (the
 *     persistent kernel) is accepted (others return IWPP_E_UNSUPPORTED);
 *     params->timing is ignored.
 *   status: device pointer to one int32 owned by the caller (may be NULL);
 *     when the reconstruction has finished on `stream`, it holds the IWPP_*
 *     status the existing entry point reports (IWPP_OK, _MARKER_GT_MASK,
 *     _INCOMPLETE or _INTERNAL).
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: the call clears what must start at zero itself (with a
 * kernel, no memset), and calls that overlap on one device (other streams,
 * other threads) race and must not be issued.  Returns IWPP_OK once queued,
 * or a host-side argument error.
 */
#define IWPP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int iwpp_reconstruct_noalloc(const iwpp_image *img, int dtype, int conn, uint32_t flags,
                             const iwpp_params *params, int32_t *status, iwpp_stream_t stream);

/*
 * Plain device-to-device streaming copy of `bytes` (a multiple of 16) with
 * the library's own kernel: the reference for bandwidth and for scaling
 * hardware byte counters.
 */
int iwpp_device_copy(void *dst, const void *src, size_t bytes, iwpp_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* IWPP_H */
