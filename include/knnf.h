/*
 * knnf.h -- C-ABI of the MI355X (gfx950) KNN filtering library.
 *
 * The library implements the spatial stage of the spatial-spectral classifier
 * of Lazcano et al. (Sec. II.C.3 and Fig. 2): given the one-band image I (the
 * first principal component, "PCA band") and the per-pixel class-probability
 * maps P of the pixel-wise classifier, it finds each pixel's K nearest
 * neighbours inside a search window and averages their probabilities.
 *
 *   Feature of pixel (r, c):   (I[r][c], lambda*r, lambda*c)      Sec. II.C.3
 *   Distance (Eq. 1):          squared Euclidean distance of the features,
 *                              evaluated in IEEE binary32 as
 *                                fr(x) = fl32(lambda * (float)x)
 *                                a = fl32(fr(r) - fr(i)), b = fl32(fr(c) - fr(j))
 *                                e = fl32(I[r][c] - I[i][j])
 *                                d = fmaf(e, e, fmaf(b, b, fl32(a * a)))
 *                              (the equation's column term is (c - j)^2; the
 *                              printed (r - j)^2 contradicts the definitions
 *                              under it)
 *   Window (Sec. III.A.3):     rows max(0, r-R) .. min(H-1, r+R), all columns,
 *                              clipped at the frame edges, the pixel included
 *   Neighbours:                the K smallest candidates in the strict order
 *                              (d, then linear index i*W + j), ascending
 *   Filtered maps (Eq. 2):     S_c = sum of the neighbours' P[.][c] in that
 *                              order from +0 in binary32; O_c = fl32(S_c / K)
 *   Class map (Sec. III.A.3.b): the class with the largest S_c; ties go to the
 *                              lowest class index
 *
 * Memory layout (all device memory, owned by the caller, row-major):
 *   pc1       float [H][W]
 *   prob      float [H][W][C]   (class index fastest)
 *   out_prob  float [H][W][C]
 *   out_class int32 [H][W]
 *   out_nbr   int32 [H][W][K]   optional (NULL to skip); linear indices i*W+j
 *   out_dist  float [H][W][K]   optional (NULL to skip)
 * Output buffers must not overlap the inputs or each other.
 *
 * Streams: every filtering call is asynchronous on the given HIP stream
 * (hipStream_t passed as void*, NULL = the null stream).  Inputs must stay valid
 * and outputs untouched until the stream has reached the call.  Parameter
 * validation is synchronous and happens before anything is enqueued.
 *
 * Errors: functions return a knnf_status.  Validation is synchronous and
 * happens before anything is enqueued; KNNF_EINVAL leaves the context usable.
 * It covers sizes, parameters, pointers and, unless the plan's
 * KNNF_PLAN_NO_INPUT_CHECK flag is set, the input values: a non-finite pc1 or
 * prob value (NaN or +-inf) is rejected with KNNF_EINVAL.  That check is one
 * device pass over the inputs on the caller's stream, after which the call
 * waits for the stream (so the check makes the call synchronous); nothing else
 * is enqueued when it fails.  With the check skipped the caller vouches for
 * finite inputs: non-finite values then do not make the library read or write
 * out of bounds, but the selected neighbours are unspecified.
 * A failed HIP call returns KNNF_EDEVICE and marks the context as failed: every
 * later call on it (and on servers created on it) returns KNNF_EDEVICE
 * ("sticky"), since device state after a failure cannot be trusted; destroy the
 * context.  knnf_last_error() gives a text description of the last failure on
 * the calling thread.
 */
#ifndef KNNF_H
#define KNNF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KNNF_OK = 0,
    KNNF_EINVAL = -1,  /* bad parameter or pointer; nothing was enqueued     */
    KNNF_ENOMEM = -2,  /* a device or host allocation failed                 */
    KNNF_EDEVICE = -3, /* a HIP call failed                                  */
    KNNF_EAGAIN = -4,  /* serving queue full; retry later                    */
    KNNF_ESTATE = -5   /* call not valid in the object's current state       */
} knnf_status;

/* Parameter limits checked by every filtering call. */
#define KNNF_MAX_K 64
#define KNNF_MAX_C 16
#define KNNF_MAX_SIDE 16777216 /* 2^24: larger row/column numbers are not exact in binary32 */

/*
 * One frame: sizes, filter parameters and device pointers.
 *   H, W    1..KNNF_MAX_SIDE, H*W <= 2^31 - 1
 *   C       number of classes, 1..KNNF_MAX_C          (Sec. II.C.1, Eq. 2)
 *   K       neighbours, 1..KNNF_MAX_K and no larger than the smallest window,
 *           min(H, R+1) * W (the paper leaves K > window size undefined)
 *   R       window half-height in rows, >= 0         (Sec. III.A.3)
 *   lambda  spatial weight, finite, >= 0, lambda * max(H, W) <= 1e18
 *           (Sec. II.C.3: 0 ignores the coordinates)
 */
typedef struct {
    int32_t H, W, C, K, R;
    float lambda;
    const float* pc1;
    const float* prob;
    float* out_prob;
    int32_t* out_class;
    int32_t* out_nbr;
    float* out_dist;
} knnf_frame;

/* Opaque library context: device, workspace for batch tables, tuned plans. */
typedef struct knnf_ctx knnf_ctx;

/*
 * Search strategy.
 *   KNNF_SEARCH_EXHAUSTIVE  evaluates Eq. 1 for every candidate of every window.
 *   KNNF_SEARCH_PRUNED      skips candidate rows and column chunks whose
 *                           spatial part of Eq. 1 alone already exceeds the
 *                           current K-th distance.  Since every term of Eq. 1
 *                           is non-negative and binary32 rounding is monotone,
 *                           the skipped candidates could never be selected:
 *                           the outputs are bit-identical to the exhaustive
 *                           search.  With lambda = 0 (the spectral distance
 *                           alone) a single-frame call (knnf_filter) under
 *                           this search runs a 1-D selection instead when the
 *                           band of 2R + 2 rows (clipped to H) holds at most
 *                           16,384 pixels: the band of two query rows'
 *                           windows is sorted by PC1 value and each query
 *                           walks outward from its own value over its own
 *                           window's pixels; same outputs again.  Its launches
 *                           leave the work counters (knnf_stats_*) unchanged.
 */
typedef enum { KNNF_SEARCH_EXHAUSTIVE = 0, KNNF_SEARCH_PRUNED = 1 } knnf_search;

/*
 * Launch plan: how a frame is cut into work.
 *   search        one of knnf_search
 *   tile_rows     query pixels per wavefront task = tile_rows x tile_cols;
 *   tile_cols     supported tiles (rows x cols): 1x8, 1x16, 2x4, 2x8, 4x4
 *   waves         wavefronts per workgroup; 1, 2 or 4
 *   launch        knnf_launch (batched launches only)
 *   chunk_rows    window chunk of the pruned search: the candidates a
 *                 wavefront evaluates per step form a patch of chunk_rows rows
 *                 x (64 / chunk_rows) columns; 8, 16 or 32 (the exhaustive
 *                 search always sweeps 4 rows x 64 columns)
 *   flags         KNNF_PLAN_* bits
 * A zero tile, wave, launch or chunk field means "the context's default"
 * (initially a pruned search with 1 x 8 tiles, one wavefront per workgroup,
 * grid launches and 16-row chunks); search and flags are always taken from
 * the plan (0 = exhaustive, input check on).  Every plan gives bitwise
 * identical outputs.
 */
#define KNNF_PLAN_NO_INPUT_CHECK 1 /* skip the non-finite input check */

typedef struct {
    int32_t search;
    int32_t tile_rows;
    int32_t tile_cols;
    int32_t waves;
    int32_t launch;     /* batched launches: knnf_launch                          */
    int32_t chunk_rows; /* pruned search: window chunk rows (8, 16, 32)           */
    int32_t flags;      /* KNNF_PLAN_* bits                                       */
} knnf_plan;

/*
 * How a batched launch distributes tile tasks.
 *   KNNF_LAUNCH_PERSISTENT  a grid sized to the device; wavefronts claim
 *                           consecutive tasks from a counter until none is left
 *   KNNF_LAUNCH_GRID        one wavefront per task; the hardware dispatcher
 *                           balances the load
 * 0 means the context's default (grid: faster than persistent on uneven
 * and small-frame batches on MI355X).
 */
typedef enum { KNNF_LAUNCH_DEFAULT = 0, KNNF_LAUNCH_PERSISTENT = 1, KNNF_LAUNCH_GRID = 2 } knnf_launch;

/*
 * Create a context on HIP device `device` (ordinal).  *out is NULL on error
 * (KNNF_EDEVICE when no HIP device is usable).  If the environment variable
 * KNNF_TUNE_CACHE names a readable file written by knnf_tune, its plans are
 * loaded (see knnf_tune).
 */
knnf_status knnf_create(knnf_ctx** out, int device);

/* Free the context and its device workspace.  NULL is accepted. */
knnf_status knnf_destroy(knnf_ctx* ctx);

/*
 * KNNF_OK, or KNNF_EDEVICE once a HIP call on the context has failed (the
 * context stays failed).  KNNF_EINVAL for NULL.
 */
knnf_status knnf_ctx_status(const knnf_ctx* ctx);

/*
 * Marks the context as failed exactly as a failed HIP call would (every later
 * call returns KNNF_EDEVICE).  For testing how callers handle device failures;
 * launches nothing.
 */
knnf_status knnf_inject_fault(knnf_ctx* ctx);

/* Default plan used when a call passes no plan (NULL).  Validated. */
knnf_status knnf_set_default_plan(knnf_ctx* ctx, const knnf_plan* plan);
knnf_status knnf_get_default_plan(const knnf_ctx* ctx, knnf_plan* plan);

/*
 * Check a frame's sizes, parameters and pointers without launching anything.
 * Returns KNNF_OK or KNNF_EINVAL.
 */
knnf_status knnf_validate(const knnf_frame* frame);

/*
 * Filter one frame (Sec. II.C.3, Eq. 1 and 2) with one kernel launch on
 * `stream` (two with the input check).  plan may be NULL: then the plan
 * knnf_tune cached for the frame's (H, W, K, R, C), else the context's
 * default.
 */
knnf_status knnf_filter(knnf_ctx* ctx, const knnf_frame* frame,
                        const knnf_plan* plan, void* stream);

/*
 * Filter n frames of possibly different sizes and parameters with one launch
 * on `stream` over a table of per-wavefront tile tasks, largest frames first
 * (plan->launch: one wavefront per task, or a persistent grid whose
 * wavefronts claim tasks from a shared counter).  Every frame's outputs are bitwise
 * equal to knnf_filter() of that frame alone.  The frame table is copied to
 * the context's device workspace with an asynchronous copy on `stream`; the
 * caller's array may be reused when the call returns.  plan may be NULL: then
 * the plan knnf_tune cached for this frame list, else the context's default.
 * Calls on one context must not run concurrently from several host threads.
 */
knnf_status knnf_filter_batch(knnf_ctx* ctx, const knnf_frame* frames, int n,
                              const knnf_plan* plan, void* stream);

/*
 * Autotuner: times every plan -- search, tile shape, waves, window chunk
 * (pruned search) and, for n > 1, launch mode -- on the given frames (device
 * buffers of the caller; their outputs are overwritten), `reps` timed
 * repetitions each (>= 1) after one warm-up, with HIP events on `stream`
 * (synchronised).  The fastest plan is written to *best (if not NULL) and
 * cached in the context under the frames' key: for n = 1 the frame's
 * (H, W, K, R, C); for n > 1 the list of those tuples in order.  Calls that
 * pass no plan use the cached plan of their key.  If KNNF_TUNE_CACHE was set
 * when the context was created, the cache is also written to that file as
 * JSON after every tuning (and read back by later contexts); KNNF_EINVAL if
 * it cannot be written (the plan is still cached in the context and in *best).
 */
knnf_status knnf_tune(knnf_ctx* ctx, const knnf_frame* frames, int n, int reps,
                      void* stream, knnf_plan* best);

/*
 * The plan a call without a plan would use for these frames: the cached plan
 * of their key (returns KNNF_OK) or the context's default (returns
 * KNNF_ESTATE: nothing cached).  Frames are validated (sizes only).
 */
knnf_status knnf_tune_lookup(const knnf_ctx* ctx, const knnf_frame* frames, int n,
                             knnf_plan* plan);

/*
 * Work counters of the filtering kernels, for roofline accounting.  While
 * enabled, every launch adds the number of candidate distances it evaluated
 * for on-frame query pixels (pass-A block slots included) and the number of
 * tiles it processed.  Off by default; enabling allocates 16 bytes of device
 * memory once.  knnf_stats_read synchronises the device; reset != 0 zeroes
 * the counters after reading.
 */
knnf_status knnf_stats_enable(knnf_ctx* ctx, int on);
knnf_status knnf_stats_read(knnf_ctx* ctx, uint64_t* pairs, uint64_t* tiles, int reset);

/*
 * Bytes of device memory a frame occupies (inputs + outputs, each buffer
 * rounded up to 256 bytes), used to admit frames into a fixed pool.
 */
size_t knnf_frame_bytes(int H, int W, int C, int K, int with_nbr);

/* ---------------------------------------------------------------------------
 * Serving.  The paper's real-time requirement is per frame: a frame must be
 * classified before the sensor delivers the next one (Sec. I; Sec. II.B for
 * the neurosurgical and dermatological use cases).  A server accepts frames
 * of different sizes from the host at any time, admits them by device memory
 * into a caller-owned pool, keeps inputs and outputs resident, and processes
 * all admitted frames together (continuous batching): every GPU step is one
 * batched launch over tile ranges of all admitted frames, bounded by a tile
 * budget, so a large frame is processed in slices and frames that arrive
 * meanwhile join the next step.  Up to `max_inflight` steps are queued on
 * separate streams, so the next step is ready when the current one ends.
 *
 * KNNF_SERVE_PLAIN is the comparison baseline: one whole frame per launch,
 * one launch at a time, in arrival order.
 *
 * Outputs are bitwise identical to knnf_filter() of the same frame alone.
 * The server and ticket functions may be called from any host thread.
 * ------------------------------------------------------------------------- */
typedef struct knnf_server knnf_server;

typedef enum { KNNF_SERVE_BATCHED = 0, KNNF_SERVE_PLAIN = 1 } knnf_serve_mode;

typedef struct {
    int32_t mode;          /* knnf_serve_mode                                   */
    int32_t max_queue;     /* frames submitted but not admitted; 0: 4096         */
    int32_t max_inflight;  /* GPU steps queued at once (batched mode), 0: 2; <=4 */
    int32_t step_tiles;    /* tile budget of one batched step; 0: 32768 (a lone  */
                           /* frame with nothing waiting runs whole)             */
    knnf_plan plan;        /* kernel plan; zero fields: the context's default,    */
                           /* except launch, which defaults to KNNF_LAUNCH_GRID;  */
                           /* without KNNF_PLAN_NO_INPUT_CHECK, submit checks     */
                           /* the host inputs for non-finite values               */
} knnf_server_opts;

typedef struct {
    int32_t H, W, C, K, R;  /* as in knnf_frame                                  */
    float lambda;
    const float* pc1;       /* host memory, H*W; must stay valid until the frame */
    const float* prob;      /* is done (pinned memory allows asynchronous copies) */
    int32_t with_nbr;       /* keep out_nbr and out_dist as well                 */
    double t_arrival;       /* arrival time on knnf_server_clock(); < 0: now     */
} knnf_host_frame;

typedef struct {
    int32_t done;           /* 1 once the outputs are final in device memory     */
    int32_t released;
    double t_arrival;       /* knnf_server_clock() seconds                       */
    double t_admit;         /* pool memory granted, copy to the device enqueued  */
    double t_launch;        /* first GPU step containing the frame enqueued      */
    double t_done;          /* completion observed by the server                 */
} knnf_ticket_info;

/* Monotonic clock of the server, in seconds. */
double knnf_server_clock(void);

/*
 * Create a server on `ctx` that sub-allocates frames from the device buffer
 * `pool` (pool_bytes >= 4096 bytes, 256-byte aligned as hipMalloc returns it,
 * caller-owned, must outlive the server; its contents are overwritten).
 * Starts one scheduler thread after one small warm-up operation on each of
 * its streams.  opts may be NULL (batched mode, defaults).  KNNF_EINVAL for
 * bad arguments, KNNF_EDEVICE if a stream cannot be set up.
 */
knnf_status knnf_server_create(knnf_server** out, knnf_ctx* ctx, void* pool,
                               size_t pool_bytes, const knnf_server_opts* opts);

/*
 * Submit a frame.  Returns a ticket.  KNNF_EINVAL for a bad frame (including
 * non-finite input values, checked on the host unless the server's plan has
 * KNNF_PLAN_NO_INPUT_CHECK), KNNF_ENOMEM if the frame can never fit the pool,
 * KNNF_EAGAIN if the admission queue is full (retry later), KNNF_EDEVICE once
 * the server or its context has failed.
 */
knnf_status knnf_server_submit(knnf_server* srv, const knnf_host_frame* frame,
                               uint64_t* ticket);

/* State and timestamps of a ticket.  KNNF_EINVAL for an unknown ticket. */
knnf_status knnf_server_poll(knnf_server* srv, uint64_t ticket, knnf_ticket_info* info);

/*
 * Device view of a finished frame: pointers into the pool (inputs and
 * outputs), valid until knnf_server_release().  KNNF_ESTATE if not done.
 */
knnf_status knnf_server_result(knnf_server* srv, uint64_t ticket, knnf_frame* view);

/* Return a finished frame's pool memory.  KNNF_ESTATE if not done. */
knnf_status knnf_server_release(knnf_server* srv, uint64_t ticket);

/* Wait until every submitted frame is done (timeout in seconds; <= 0: none). */
knnf_status knnf_server_drain(knnf_server* srv, double timeout_s);

/* Stop the scheduler after the GPU work in flight ends, and free the server. */
knnf_status knnf_server_destroy(knnf_server* srv);

/* ---- PC1 projection: the one-band image the filter reads ---------------
 *
 * The PCA of Sec. II.C.2 centres every band by its average (step (i)) and
 * projects the centred image onto the first eigenvector of the covariance
 * matrix, keeping that one component (step (iv)); the GPU versions do both
 * in double precision (Sec. III.A.2.a/d, Sec. III.B.2.a/d).  The covariance
 * and eigenvector steps (ii)-(iii) are not part of this library: the band
 * averages and the eigenvector are inputs.  The filter reads a normalised I
 * (Sec. II.C.3); normalisation here is min-max to [0, 1] over the frame.
 *
 *   I[p]  = sum_b (cube[p][b] - mean[b]) * vec[b]        binary64
 *   I'[p] = (I[p] - min I) / (max I - min I)             binary64, 0 if I is constant
 *   out[p] = I'[p] (normalize != 0) or I[p], rounded once to binary32
 *
 * cube  device, npix x bands float32, pixel-major (a pixel's bands contiguous)
 * mean  device, bands float64 (band averages)
 * vec   device, bands float64 (first eigenvector)
 * out   device, npix float32; may be the pc1 buffer of a knnf_frame
 * Asynchronous on `stream`.  Uses a context workspace (8 B per pixel when
 * normalize != 0, plus 16 KB) that grows on first use of a larger frame (that
 * call synchronizes the device and allocates).  Calls that overlap on one
 * context race on the workspace: issue them on one stream.
 * Errors: KNNF_EINVAL for a NULL argument, npix outside [1, 2^40], bands
 * outside [1, KNNF_PC1_MAX_BANDS]; KNNF_ENOMEM if the workspace cannot grow;
 * KNNF_EDEVICE for a failed launch.
 */
#define KNNF_PC1_MAX_BANDS 4096
#define KNNF_PC1_MAX_PIXELS (1LL << 40)
knnf_status knnf_pc1(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                     const double* mean, const double* vec, float* out, int32_t normalize,
                     void* stream);

/*
 * knnf_pc1 without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as knnf_pc1, but its
 * workspace is a static scratch array that each device holds for the life of
 * the process (8 MiB + 16 KiB), so the call never allocates or synchronises.
 * Limit: with normalize != 0, npix <= KNNF_PC1_NOALLOC_MAX_PIXELS (larger:
 * KNNF_EINVAL, nothing enqueued); the raw projection uses no scratch.  Every
 * call on one device shares that device's scratch (nothing in it needs to
 * start at zero): calls that overlap on one GPU -- on different streams, or
 * from several contexts or threads -- race and must be serialised by the
 * caller, e.g. issued on one stream.
 */
#define KNNF_PC1_NOALLOC_MAX_PIXELS (1 << 20)
knnf_status knnf_pc1_noalloc(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                             const double* mean, const double* vec, float* out,
                             int32_t normalize, void* stream);

/* ---- SVM probabilities: the maps the filter averages ---------------------
 *
 * The classification stage of the one-vs-one SVM of Sec. II.C.1 (GPU
 * versions Sec. III.A.1, III.B.1), per pixel x: decision values against every
 * binary hyperplane, their binary probabilities through a sigmoid, and the
 * multiclass probabilities by pairwise coupling (the second method of the
 * paper's reference [30], Wu, Lin and Weng).  Training is offline and not
 * part of the library: the model is an input.
 *
 *   f[m] = sum_b w[m][b] x[b] + bias[m]                       binary64
 *   r[m] = 1 / (1 + exp(A[m] f[m] + B[m])), clamped to [1e-7, 1 - 1e-7]
 *          (class i of the pair; 1 - r[m] for class j)
 *   Q[t][t] = sum_{s != t} r_st^2,  Q[t][j] = -r_jt r_tj
 *   p = uniform; sweep t = 0..C-1: p[t] <- (p'Qp - sum_{j != t} Q[t][j] p[j]) / Q[t][t],
 *          then p /= sum(p); until max_t |(Qp)[t] - p'Qp| < 0.005 / C, at most 100 sweeps
 *   out[p][c] = p[c] rounded once to binary32
 *
 * Hyperplane m covers the class pair (i, j), i < j, in lexicographic order
 * (0,1), (0,2), ..., (0,C-1), (1,2), ...; M = C (C - 1) / 2.
 * cube     device, npix x bands float32, pixel-major (a pixel's bands contiguous)
 * w        device, M x bands float64 (hyperplanes, row m = pair m)
 * bias, A, B  device, M float64 each (offsets and sigmoid parameters)
 * out      device, npix x classes float32, class fastest; may be the prob
 *          buffer of a knnf_frame
 * A non-finite cube or model value gives unspecified probabilities for the
 * pixels it reaches (the kernel still ends normally).
 * Asynchronous on `stream`; no workspace, no allocation.
 * Errors: KNNF_EINVAL for a NULL argument, npix outside [1, 2^31], bands
 * outside [1, KNNF_SVM_MAX_BANDS], classes outside [2, KNNF_SVM_MAX_CLASSES];
 * KNNF_EDEVICE for a failed launch.
 */
#define KNNF_SVM_MAX_CLASSES 8
#define KNNF_SVM_MAX_BANDS 4096
#define KNNF_SVM_MAX_PIXELS (1LL << 31)
knnf_status knnf_svm(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                     int32_t classes, const double* w, const double* bias, const double* A,
                     const double* B, float* out, void* stream);

/* ---- Both steps before the filter from one read of the cube ------------
 *
 * knnf_svm and knnf_pc1 of the same cube in one pass over it: the kernel that
 * computes the SVM probability maps also accumulates each pixel's PC1
 * projection from the same staged bands (the pipeline's classification and
 * dimensionality-reduction steps, Sec. II.C.1-2, read the image once instead
 * of twice).  out_prob is knnf_svm's output (bitwise the same); out_band is
 * knnf_pc1's (normalize as there; the projection is summed band by band in
 * ascending order, so it can differ from knnf_pc1's, whose summation order is
 * different, by the last binary32 bit).  Arguments, layouts and limits as in
 * those two calls; `cube` must hold both steps' input.  With normalize != 0
 * it uses the context workspace of knnf_pc1 (8 B per pixel plus 16 B per 256
 * pixels; growing it synchronizes the device and allocates).  Asynchronous on
 * `stream`.  Errors: as knnf_svm, plus KNNF_EINVAL for NULL mean, vec or
 * out_band, KNNF_ENOMEM if the workspace cannot grow.
 */
knnf_status knnf_svm_pc1(knnf_ctx* ctx, const float* cube, int64_t npix, int32_t bands,
                         int32_t classes, const double* w, const double* bias, const double* A,
                         const double* B, const double* mean, const double* vec, float* out_prob,
                         float* out_band, int32_t normalize, void* stream);

/* Text of the last error on the calling thread ("" if none). */
const char* knnf_last_error(void);

/* Library version, e.g. "knnf 0.1.0 gfx950". */
const char* knnf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KNNF_H */
