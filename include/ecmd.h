/*
 * ecmd.h - C ABI of the MI355X exact event-based divergence estimator.
 *
 * Method: "Globally Optimal Event-Based Divergence Estimation for Ventral
 * Landing" (arXiv 2209.13168).  Given the events of a window of length tau,
 * the library finds the divergence d = -nu (Z0 = 1, Sec. 4.1) that maximises
 * the contrast of the motion-compensated event image (Sec. 4.2, eqs.
 * (12)-(14)) with the branch and bound of Algorithm 1 and the upper bound of
 * Sec. 4.3 (eqs. (15)-(20)), on the GPU.
 *
 * Fixed readings of the method (a separate CPU implementation in the tests
 * states the same readings independently and checks the results against):
 *   - fp32 warp in this order: per event ax = (x - cx)(tau - t'),
 *     ay = (y - cy)(tau - t'); per hypothesis r = d / (1 - d tau);
 *     xw = fmaf(ax, r, x), yw = fmaf(ay, r, y) (eq. (12));
 *   - pixel k covers [k, k+1); an event counts iff 0 <= xw < W, 0 <= yw < H;
 *   - contrast key K = M*S - N^2 = M^2 C (eq. (14)), S = sum H^2,
 *     N = sum H, M = W*H; bound key K_bar = M*S_bar - N_low^2 (eq. (15)),
 *     S_bar from the upper-bound image of eq. (17) and N_low from eq. (20);
 *   - candidates: the dyadic grid d_j = float(d_lo + (d_hi - d_lo) j 2^-L),
 *     j = 1 .. 2^L - 1, with L the smallest depth whose spacing is <= eps;
 *   - the result is the largest K, ties to the smallest j (gamma = 0), or
 *     Algorithm 1's gamma-optimal stop (gamma > 0).
 *
 * Conventions for every entry point:
 *   - return 0 (ECMD_OK) or a negative ECMD_E* code; ecmd_last_error(ctx)
 *     then holds a message.  On error, outputs are left untouched except
 *     the status fields of result structs;
 *   - array arguments are host pointers unless `flags & ECMD_DEVICE_PTR`,
 *     in which case every array argument of that call (inputs and array
 *     outputs, not the result structs) is a device pointer on the context's
 *     device.  The caller owns all arrays; they are only borrowed for the
 *     duration of the call.  Result structs are always host memory;
 *   - calls are synchronous with respect to the host and are ordered on the
 *     context's HIP stream;
 *   - a context is not thread-safe: use one per host thread.
 */
#ifndef ECMD_H
#define ECMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ECMD_OK 0
#define ECMD_EINVAL (-1)    /* invalid argument (message says which) */
#define ECMD_ENOMEM (-2)    /* device or host allocation failed */
#define ECMD_EDEVICE (-3)   /* HIP runtime error (message has the HIP text) */
#define ECMD_EBUDGET (-4)   /* node budget reached: incumbent + certified gap */
#define ECMD_EFRONTIER (-5) /* frontier capacity exceeded (per window) */

#define ECMD_DEVICE_PTR 1u

typedef struct ecmd_ctx ecmd_ctx;

/* Sensor geometry.  The focus of expansion (foe_x, foe_y) is the principal
 * point (the FOE of Sec. 3.2), in pixel coordinates where pixel k covers
 * [k, k+1).  An integer FOE strictly inside the sensor lets the library cut
 * the image into quadrants that no event ever leaves. */
typedef struct {
    int32_t width, height;
    float foe_x, foe_y;
} ecmd_sensor;

/* Events of a stream, structure of arrays.  t is absolute time in seconds
 * (sorted is not required).  p (nullable, one byte per event, same memory
 * kind as x) selects the polarity-aware contrast: NULL gives the event image
 * of eq. (13), which ignores polarity; otherwise the events with p > 0 and
 * those with p <= 0 form two images and the contrast of eq. (14) is the
 * variance over all 2*W*H cells of both (the paper notes after eq. (14)
 * that polarity can be accommodated); keys and contrasts then use
 * M = 2*W*H.  Both +1/-1 and 1/0 encodings work. */
typedef struct {
    const float *x;
    const float *y;
    const double *t;
    int64_t n;
    const int8_t *p;
} ecmd_events;

/* Window [t0, t1] (closed): the batch of Sec. 3.3, tau = float(t1 - t0). */
typedef struct {
    double t0, t1;
} ecmd_window;

/* A window holds fewer than 2^28 events (ECMD_EINVAL otherwise), and
 * n^2 * 2 * (width + height + 3) < 9e18 so that the exact sums fit 64 bits.
 *
 * Search: d in [d_lo, d_hi] with grid spacing <= eps (0 <= d_lo < d_hi,
 * float(d_hi * tau) < 1: the cheirality limit of eq. (11)).  gamma > 0 stops
 * Algorithm 1 once the best bound is within gamma of the incumbent in
 * contrast units.  max_nodes > 0 caps node expansions (ECMD_EBUDGET).
 * frontier_batch is the expansion policy: the number of queued nodes
 * expanded together per step.  1 = Algorithm 1's order: the queued node with
 * the largest bound, ties to the smaller grid index, one per step.  k > 1 =
 * up to k nodes evaluated in one launch, chosen by bound gap K_bar - K_inc
 * in power-of-two classes: every node of the larger classes, then nodes of
 * the class where the count reaches k in queue order (each within a factor
 * two of the largest gap).  0 = the context's tuning, 96 by default.  The
 * canonical result does not depend on it.  frontier_capacity caps queued
 * nodes per window (0 = 16384; a window that needs more stops with
 * ECMD_EFRONTIER, its incumbent and gap = infinity).
 *
 * flags: ECMD_SEARCH_EXACT_BOUNDS computes the bound of eqs. (15)-(20) for
 * every child interval.  Without it (the default), a child whose decision
 * cannot depend on its bound's value (no node budget, and every node the
 * queue can hold after this step is expanded next) is first given
 * a cheaper certificate from its endpoints alone: with U the sum over the
 * owned events with both endpoints in the image of |dkx| + |dky| + 1 (the
 * walk visits that many distinct image pixels), Cauchy-Schwarz over the M
 * cells gives M * S_bar >= U^2, so K_bar >= U^2 - N_low^2.  When that
 * exceeds the incumbent the node is kept, the decision the exact bound
 * gives; otherwise the exact bound is computed in the same step.  With
 * gamma = 0 the nodes expanded, the incumbent and the result are those of
 * the exact search.  With gamma > 0 the stop test bounds a certified node's
 * points by the exact bound of its nearest exactly bounded ancestor (an
 * interval containing them), which is looser: the search stops at the same
 * step as the exact search or later, with the same guarantee.  bound_evals
 * and pixel_updates count exact bounds only. */
#define ECMD_SEARCH_EXACT_BOUNDS 1u

typedef struct {
    float d_lo, d_hi, eps;
    uint32_t flags;
    double gamma;
    int64_t max_nodes;
    int32_t frontier_batch;
    int32_t frontier_capacity;
} ecmd_search;

/* Per-window result.  K = K_hi * 2^64 + K_lo is the exact contrast key of
 * the returned grid point; contrast = K / M^2; d_end = d_hat/(1 - d_hat tau)
 * is the divergence at the window end (Sec. 4.1's point estimate with
 * nu = -d_hat).  gap is 0 when the result is certified optimal; otherwise
 * an upper bound on (best contrast - returned contrast).  Counters:
 * event_hyp_evals = sum over evaluated hypotheses of the window's event
 * count (exact bounds and points); pixel_updates = upper-bound image
 * increments; bound_certs = child intervals kept on the endpoint certificate
 * (see ecmd_search.flags), whose walks were not made.  A search cut short
 * while such a node is queued takes that node's gap from its nearest
 * exactly bounded ancestor (infinity when it has none). */
typedef struct {
    int32_t status;
    uint32_t j_star;
    uint32_t L;
    float d_hat;
    double contrast;
    double d_end;
    double gap;
    uint64_t K_lo;
    int64_t K_hi;
    int64_t n_events;
    int64_t nodes_expanded;
    int64_t nodes_pruned;
    int64_t point_evals;
    int64_t bound_evals;
    int64_t event_hyp_evals;
    int64_t pixel_updates;
    int32_t steps;
    int32_t seeded;
    int64_t bound_certs;
} ecmd_result;

/* ------------------------------------------------------------ context */

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = a blocking stream of default priority that the
 * context creates and owns).  The context owns all device scratch;
 * ecmd_ctx_destroy frees it, together with the device memory of every
 * network still alive on it (those handles then accept only
 * ecmd_cnn_destroy; every other call on them returns ECMD_EINVAL). */
int ecmd_ctx_create(ecmd_ctx **out, int device, void *hip_stream);
void ecmd_ctx_destroy(ecmd_ctx *ctx);
/* Last error message of this context ("" if none). */
const char *ecmd_last_error(const ecmd_ctx *ctx);
/* Library version string. */
const char *ecmd_version(void);

/* Per-phase device timers of a context (off by default).  The evaluation
 * and frontier kernels are timed by start/stop events attached to their own
 * dispatch (kernel time only); window prep by events recorded on the
 * context's stream around it.  Times are summed over all calls since the
 * last reset. */
typedef struct {
    int64_t calls;
    int64_t eval_launches;     /* hypothesis evaluation kernel (eqs. (13)-(20)) */
    double eval_ms;
    int64_t frontier_launches; /* frontier step kernel (Algorithm 1) */
    double frontier_ms;
    double prep_ms;            /* window prep (event binning) */
} ecmd_profile;

int ecmd_ctx_set_profiling(ecmd_ctx *ctx, int enable);
/* Copy the accumulated timers; reset them when `reset` is non-zero. */
int ecmd_ctx_get_profile(ecmd_ctx *ctx, ecmd_profile *out, int reset);

/* Launch tuning of a context, used by every search call whose
 * ecmd_search.frontier_batch is 0.  frontier_batch: nodes expanded together
 * per window and step (0 = 96).  tile_px: most LDS counters per image
 * tile, (w + 2)(h + 2) for a w x h tile with its one-pixel border (0 = what
 * the LDS holds; smaller values split the FOE quadrants further, trading
 * guest copies for occupancy).  tile_px and eval_threads both 0: the
 * default rule of ecmd_plan picks both.  graph: replay the step
 * loop as a captured hipGraph (0 = plain launches).  group: hypotheses of
 * one window and tile evaluated per work item (0 = chosen at every step:
 * 1 while the step has fewer than ~48 items per CU, else 2). */
typedef struct {
    int32_t frontier_batch;
    int32_t tile_px;
    int32_t graph;
    int32_t group;
    int32_t eval_threads;  /* threads per evaluation workgroup: 256, 512, 1024 (0 = 1024) */
} ecmd_tuning;

int ecmd_ctx_set_tuning(ecmd_ctx *ctx, const ecmd_tuning *tuning);
int ecmd_ctx_get_tuning(const ecmd_ctx *ctx, ecmd_tuning *out);

/* Search plan, computed on the host without a device: the grid depth L of
 * the dyadic grid (smallest L >= 1 with (d_hi - d_lo) 2^-L <= eps), and
 * the image tiling the evaluation kernel uses — cuts at the FOE lines when
 * the FOE is an integer point strictly inside the sensor (the warp of
 * eq. (12) never moves an event across them), bands split evenly until each
 * tile's counters fit the budget.  lds_bytes = LDS per CU (0 = 160 KiB,
 * gfx950); tile_px caps the counters per tile as ecmd_tuning.tile_px does
 * (0: the default rule, which takes the first of: tiles whose counters let
 * three 512-thread workgroups share a CU, then two — each only when it
 * cuts the image into at most 24 tiles — then one 1024-thread workgroup
 * with the whole LDS);
 * polarity != 0 plans the two images of the polarity-aware contrast. */
typedef struct {
    int32_t L;
    int32_t segments;        /* event segments per window: tiles x images */
    int32_t ntx, nty;        /* tile grid */
    int32_t max_tile_px;     /* largest tile (pixels) */
    int32_t tile_budget_px;  /* the limit the plan met on (w + 2)(h + 2) of the largest tile */
    int32_t colcut[65];      /* column band edges, ntx + 1 used */
    int32_t rowcut[65];      /* row band edges, nty + 1 used */
    int32_t eval_threads;    /* threads per evaluation workgroup */
} ecmd_plan_info;

int ecmd_plan(const ecmd_sensor *sensor, const ecmd_search *search, int32_t polarity,
              int64_t lds_bytes, int32_t tile_px, ecmd_plan_info *out);

/* Grid point d_j = float(d_lo + (d_hi - d_lo) j 2^-L), computed in fp64
 * (the candidates of the search are j = 1 .. 2^L - 1); NaN when L is
 * outside 1..30 or j > 2^L.  Host only. */
float ecmd_grid_point(float d_lo, float d_hi, uint32_t L, uint32_t j);

/* Measured roofline denominators of this device (run on the context's
 * stream, timed with HIP events, best of three): the rate of conflict-free
 * LDS atomic adds that return nothing (lane operations per second, the
 * operation the event-image histograms use; 2 workgroups of 1024 lanes per CU, each lane
 * on its own counter) and the HBM read bandwidth of a streaming sum over
 * hbm_bytes (0 = 4 GiB, allocated for the call and freed). */
int ecmd_measure_peaks(ecmd_ctx *ctx, int64_t hbm_bytes, double *lds_atomics_per_s,
                       double *hbm_read_bytes_per_s);

/* Autotuner: times candidate tunings (frontier batch, tile size, graph
 * replay, hypotheses per item) on the given batch (arguments as ecmd_estimate_divergence_batched,
 * with search->frontier_batch ignored), keeps the fastest in the context and
 * writes it to `best`; ms_best (nullable) receives its time per call. */
int ecmd_autotune(ecmd_ctx *ctx, const ecmd_sensor *sensor, const float *x, const float *y,
                  const float *t_rel, const int64_t *offsets, const float *tau, int32_t B,
                  const ecmd_search *search, uint32_t flags, ecmd_tuning *best, double *ms_best);

/* ---------------------------------------------------------- estimation */

/* One window (Algorithm 1 on the events with t in [t0, t1]).  d_seed
 * (nullable, host) is a starting incumbent proposal: its nearest grid point
 * is evaluated first.  It can only speed pruning; the result is unchanged. */
int ecmd_estimate_divergence(ecmd_ctx *ctx, const ecmd_sensor *sensor,
                             const ecmd_events *events, ecmd_window window,
                             const ecmd_search *search, uint32_t flags,
                             const float *d_seed, ecmd_result *out);

/* B windows in one launch sequence.  Window b holds the events
 * [offsets[b], offsets[b+1]) of x, y, t_rel, with t_rel the offset from the
 * window start (0 <= t_rel <= tau[b]).  offsets (B+1, non-decreasing, int64)
 * and tau (B) follow `flags` like the event arrays.  d_seeds (nullable, B
 * values, NaN = none) follow `flags` too.  out[b].status reports per-window
 * budget/frontier outcomes; the call returns the first such status, or a
 * negative code for a call-level error (nothing computed). */
int ecmd_estimate_divergence_batched(ecmd_ctx *ctx, const ecmd_sensor *sensor,
                                     const float *x, const float *y,
                                     const float *t_rel, const int64_t *offsets,
                                     const float *tau, int32_t B,
                                     const ecmd_search *search, uint32_t flags,
                                     const float *d_seeds, ecmd_result *out);

/* The batched call on the polarity-aware contrast (see ecmd_events):
 * polarity (non-NULL, one byte per event, indexed like x) splits every
 * window's events into two event images; K and contrast use M = 2*W*H.
 * The sensor may have at most 32 tiles (64 segments), a limit reached only
 * by sensors far above 1280x720. */
int ecmd_estimate_divergence_batched_polarity(ecmd_ctx *ctx, const ecmd_sensor *sensor,
                                              const float *x, const float *y,
                                              const float *t_rel, const int8_t *polarity,
                                              const int64_t *offsets, const float *tau,
                                              int32_t B, const ecmd_search *search,
                                              uint32_t flags, const float *d_seeds,
                                              ecmd_result *out);

/* Stream estimation (Sec. 4.4): the events of [t_start, t_start + K tau)
 * are cut into K consecutive windows [t_start + k tau, t_start + (k+1) tau)
 * (half-open, fp64), each estimated as in the batched call (one launch
 * sequence for all K windows); out[k] is window k's result.  events->t must
 * be non-decreasing. */
int ecmd_estimate_stream(ecmd_ctx *ctx, const ecmd_sensor *sensor, const ecmd_events *events,
                         double t_start, double tau, int32_t K, const ecmd_search *search,
                         uint32_t flags, ecmd_result *out);

/* --------------------------------------------------- asynchronous batches */

/* A plan holds every device buffer of batched searches up to fixed limits,
 * so that ecmd_plan_launch only enqueues kernels on the context's stream:
 * it allocates nothing, copies nothing between host and device and never
 * waits, and a caller may capture it into a hipGraph and replay it.  The
 * checks that the synchronous batched call makes on the host are made on
 * the device, per window; a fixed number of frontier steps (Algorithm 1's
 * loop, four per block) replaces the host's polling of the search.
 *   max_windows: B of a launch, 1 .. 65535;
 *   max_steps:   frontier steps per launch, rounded up to a multiple of 4
 *                (0 = 2L + 8 for the grid depth L, e.g. 44 for L = 18; a
 *                search of F nodes per step usually needs about L steps);
 *                each costs four kernel launches (two evaluations and
 *                the two frontier phases), which return at once for
 *                finished windows;
 *   max_events:  events of a launch over all windows, 1 .. 2^40;
 *   max_records: binned event records, guest copies included (0 = the worst
 *                case: max_events times the tiles of one FOE quadrant);
 *   polarity:    non-zero: launches take polarities (the contrast over
 *                2*W*H cells, as ecmd_estimate_divergence_batched_polarity). */
typedef struct {
    int32_t max_windows;
    int32_t max_steps;
    int64_t max_events;
    int64_t max_records;
    int32_t polarity;
    int32_t reserved;
} ecmd_plan_limits;

typedef struct ecmd_batch_plan ecmd_batch_plan;

/* Allocate a plan on the context for `sensor` and `search` (both copied;
 * the context's tuning at this call applies).  `limits` is read, and its
 * zero fields are replaced by the values used.  The plan's device memory is
 * freed by ecmd_plan_destroy, or with the context: the handle then accepts
 * only ecmd_plan_destroy. */
int ecmd_plan_create(ecmd_ctx *ctx, const ecmd_sensor *sensor, const ecmd_search *search,
                     ecmd_plan_limits *limits, ecmd_batch_plan **out);

/* Enqueue the batched search of B windows: arguments as
 * ecmd_estimate_divergence_batched, every array a device pointer, polarity
 * non-NULL exactly when the plan has limits.polarity.  The results reach
 * out[0..B) (device memory, or pinned host memory the device can write)
 * when the stream gets there; they equal the synchronous call's, except:
 * out[w].status = ECMD_EINVAL (other fields zero) for a window that fails
 * the synchronous call's checks (offsets, event count, tau, d_hi * tau,
 * an event with a non-finite coordinate or t_rel outside [0, tau[w]]),
 * and for every window when the valid ones hold more than max_events
 * events; ECMD_ENOMEM for every window when the binned records exceed
 * max_records; ECMD_EBUDGET, with the incumbent and its certified gap, for a
 * window still searching after max_steps steps.  Returns a call-level error
 * only: NULL arrays, B outside 1 .. max_windows, a launch failure.  Launches
 * of one plan share its buffers: they must not overlap (one stream orders
 * them). */
int ecmd_plan_launch(ecmd_batch_plan *plan, const float *x, const float *y, const float *t_rel,
                     const int8_t *polarity, const int64_t *offsets, const float *tau, int32_t B,
                     const float *d_seeds, ecmd_result *out);

/* Free the plan (waits for the context's stream first). */
void ecmd_plan_destroy(ecmd_batch_plan *plan);

/* ------------------------------------------------ allocation-free search */

/* Bytes of device memory the library holds on each device it runs on, for
 * ecmd_estimate_divergence_batched_noalloc (until the process ends). */
#define ECMD_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory: code under stream or
 * graph capture, serving loops and harnesses that forbid hipMalloc.  The
 * batched search of ecmd_plan_launch without a plan: every device buffer
 * it needs comes from one static array of ECMD_NOALLOC_SCRATCH_BYTES on the
 * context's device, so the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and only enqueues kernels on the context's
 * stream; ecmd_ctx_create looks the array's address up on its device.
 * Arguments and results are those of ecmd_plan_launch for a plan with
 * limits {max_windows = B, max_steps = 0, max_events, max_records = 0,
 * polarity = 0}: every array a device pointer on the context's device, out
 * in device memory or pinned host memory, written when the stream gets
 * there, with the plan's per-window statuses.  Returns ECMD_ENOMEM, with a
 * message and nothing launched, when the buffers for B windows of up to
 * max_events events exceed the array (the event store takes 16 bytes per
 * event and image tile of its FOE quadrant, the frontier 32 bytes per node
 * of frontier_capacity per window); ECMD_EINVAL for the plan's argument
 * errors.  The array keeps the last call's contents (each call clears what
 * it reads before writing it); calls that overlap on one device (other
 * streams, threads or contexts) race. */
int ecmd_estimate_divergence_batched_noalloc(ecmd_ctx *ctx, const ecmd_sensor *sensor,
                                             const ecmd_search *search, const float *x,
                                             const float *y, const float *t_rel,
                                             const int64_t *offsets, const float *tau, int32_t B,
                                             int64_t max_events, const float *d_seeds,
                                             ecmd_result *out);

/* -------------------------------------------------------------- probes */

/* Pixel index ky*W + kx of every event at divergence d (-1 = outside),
 * eqs. (12)-(13). */
int ecmd_probe_pixels(ecmd_ctx *ctx, const ecmd_sensor *sensor, const float *x,
                      const float *y, const float *t_rel, int64_t n, float tau,
                      float d, uint32_t flags, int32_t *pix_out);

/* Point values (S_k, N_k) of m divergences d[k] (eqs. (13)-(14)); when
 * img_out is non-null it receives the m event images H (m*W*H uint32).
 * polarity (nullable) as in ecmd_estimate_divergence_batched_polarity: S
 * and N then cover both images and img_out holds 2*W*H cells per
 * hypothesis (the p <= 0 image first). */
int ecmd_probe_point(ecmd_ctx *ctx, const ecmd_sensor *sensor, const float *x,
                     const float *y, const float *t_rel, const int8_t *polarity,
                     int64_t n, float tau,
                     const float *d, int32_t m, uint32_t flags, uint64_t *S,
                     int64_t *N, uint32_t *img_out);

/* Interval values (S_bar_k, N_low_k) of m intervals [d_a[k], d_b[k]]
 * (eqs. (17)-(20)); img_out (nullable) receives the m upper-bound images.
 * The search range [d_lo, d_hi] bounds every interval (it sets the event
 * binning); pass the range the intervals come from.  polarity (nullable) as
 * in ecmd_probe_point. */
int ecmd_probe_bound(ecmd_ctx *ctx, const ecmd_sensor *sensor, const float *x,
                     const float *y, const float *t_rel, const int8_t *polarity,
                     int64_t n, float tau,
                     float d_lo, float d_hi, const float *d_a, const float *d_b,
                     int32_t m, uint32_t flags, uint64_t *S_bar, int64_t *N_low,
                     uint32_t *img_out);

/* --------------------------------------------------------- preprocessing */

/* Both calls copy the kept events of every window, in order, to x_out,
 * y_out, t_out (capacity offsets[B] - offsets[0] each) and write the new
 * window offsets to offsets_out (B + 1 values, starting at 0).  Windows and
 * pointers as in ecmd_estimate_divergence_batched. */

/* Hot-pixel removal (Sec. 6, "Preprocessing"): drop every event of a pixel
 * (floor(x), floor(y)) that holds more than max_count events of its window. */
int ecmd_hot_pixel_filter(ecmd_ctx *ctx, const ecmd_sensor *sensor, const float *x,
                          const float *y, const float *t_rel, const int64_t *offsets,
                          int32_t B, int32_t max_count, uint32_t flags, float *x_out,
                          float *y_out, float *t_out, int64_t *offsets_out);

/* "Resized and resampled" data (Sec. 6): coordinates scaled to the output
 * sensor, x' = x * float(W_out / W_in), y' = y * float(H_out / H_in) (fp32),
 * and event k of window w (k from the window start) kept iff
 * (SplitMix64(seed + (w * 2^32 + k + 1) * 0x9E3779B97F4A7C15) >> 40) <
 * floor(keep_frac * 2^24), i.e. with probability keep_frac (the paper keeps
 * 25%).  The output sensor's FOE is the caller's (normally the scaled one). */
int ecmd_resample(ecmd_ctx *ctx, const ecmd_sensor *in_sensor, const ecmd_sensor *out_sensor,
                  const float *x, const float *y, const float *t_rel, const int64_t *offsets,
                  int32_t B, float keep_frac, uint64_t seed, uint32_t flags, float *x_out,
                  float *y_out, float *t_out, int64_t *offsets_out);

/* ------------------------------------------------ learned incumbent */

typedef struct ecmd_cnn ecmd_cnn;

/* Input of the proposal network: the unwarped (d = 0) event counts of each
 * window on a 64x64 grid (cell floor(float(x*64)/W), clamped to 63), scaled
 * by 4096/N and rounded to bfloat16 (round to nearest even); out holds
 * B*64*64 uint16 bfloat16 bit patterns.  Windows as in the batched call. */
int ecmd_downsample(ecmd_ctx *ctx, const ecmd_sensor *sensor, const float *x,
                    const float *y, const int64_t *offsets, int32_t B,
                    uint32_t flags, uint16_t *out);

/* Network: conv3x3/s2 1->16, ReLU, conv3x3/s2 16->32, ReLU, conv3x3/s2
 * 32->64, ReLU, global average pool, linear 64->1 (23,361 parameters).
 * Activations and weights are rounded to bfloat16 at each layer input;
 * products accumulate in fp32.  Parameters are fp32 masters (Adam). */
#define ECMD_CNN_NPARAM 23361
int ecmd_cnn_create(ecmd_ctx *ctx, uint64_t seed, ecmd_cnn **out);
/* Free a network (before or after its context is destroyed). */
void ecmd_cnn_destroy(ecmd_cnn *cnn);
/* Copy the fp32 parameter vector (ECMD_CNN_NPARAM values, host). */
int ecmd_cnn_get_params(ecmd_cnn *cnn, float *host_params);
int ecmd_cnn_set_params(ecmd_cnn *cnn, const float *host_params);
/* Checkpoint of a network: its parameters and Adam state (first and second
 * moments, step count), so that training resumes exactly where it stopped.
 * File layout (little-endian): the 8 bytes "ECMDCNN1", uint32 parameter
 * count, int32 Adam step, then the parameters, the first moments and the
 * second moments, ECMD_CNN_NPARAM fp32 values each.  ecmd_cnn_load rejects a
 * file with another magic, count or length, or a non-finite value
 * (ECMD_EINVAL; the network is unchanged); I/O failures are ECMD_EINVAL with
 * the path in the message. */
int ecmd_cnn_save(ecmd_cnn *cnn, const char *path);
int ecmd_cnn_load(ecmd_cnn *cnn, const char *path);
/* Forward pass on B images (bf16 bits, B*64*64): d_out[b] (fp32). */
int ecmd_cnn_forward(ecmd_cnn *cnn, const uint16_t *imgs, int32_t B, uint32_t flags,
                     float *d_out);
/* Mean squared error against labels and its gradient w.r.t. the
 * parameters (host, ECMD_CNN_NPARAM values). */
int ecmd_cnn_grads(ecmd_cnn *cnn, const uint16_t *imgs, const float *labels, int32_t B,
                   uint32_t flags, float *grad_out, float *loss_out);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the MSE loss. */
int ecmd_cnn_train_step(ecmd_cnn *cnn, const uint16_t *imgs, const float *labels,
                        int32_t B, float lr, uint32_t flags, float *loss_out);

/* Batched estimation seeded by the network: downsample -> forward -> the
 * predicted d seeds each window's incumbent -> certified branch and bound.
 * Same arguments and results as ecmd_estimate_divergence_batched. */
int ecmd_estimate_divergence_learned(ecmd_ctx *ctx, ecmd_cnn *cnn,
                                     const ecmd_sensor *sensor, const float *x,
                                     const float *y, const float *t_rel,
                                     const int64_t *offsets, const float *tau,
                                     int32_t B, const ecmd_search *search,
                                     uint32_t flags, ecmd_result *out);

#ifdef __cplusplus
}
#endif
#endif /* ECMD_H */
