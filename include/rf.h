/*
 * rf.h -- C ABI of librf, the MI355X (gfx950) realfast search hot path.
 *
 * The search (Law et al. 2018, section 3.1 and Figure 2) loops over trial
 * dispersion measures and trial sampling times.  For each (DM, width) it
 * dedisperses the visibilities, boxcar-resamples them in time, forms a Stokes
 * I image of every resampled integration by gridding and a 2-D FFT, and keeps
 * images whose peak exceeds a threshold in units of the image noise.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers named h_* are host memory, d_* are device memory on the current
 * HIP device.  All d_* buffers are owned by the caller; the library never
 * allocates device memory.  A plan's device tables live in a caller-provided
 * buffer (rf_plan_create).  Workspaces are caller-provided too; their sizes
 * come from rf_workspace_bytes.
 *
 * `stream` is a hipStream_t passed as void* (NULL is the null stream).  Every
 * call except rf_plan_create, rf_get_* and rf_search_segment (which each
 * synchronise `stream` once, as documented there) enqueues its kernels on
 * `stream` and returns at once.  The returned status covers the host-side checks only; on
 * any error nothing has been enqueued.  Faults found on the device are
 * reported as data (candidate overflow via the true count in *d_ncand).
 *
 * Visibility layout: [nint][nbl][nchan][npol] row-major, each element a
 * complex number stored as interleaved (re, im):
 *   RF_CF32  two float32 (8 bytes),  RF_CF16  two IEEE binary16 (4 bytes).
 * Arithmetic is float32 in every kernel whatever the storage type; float64
 * is used only for the dispersion-delay and uv-cell arguments.
 *
 * Plans are immutable once created; concurrent calls on distinct streams
 * with distinct output buffers are safe.  No C++ exception crosses the ABI.
 */
#ifndef RF_H
#define RF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rf_status;
#define RF_OK             0
#define RF_EINVAL        -1  /* null pointer or malformed argument            */
#define RF_ESHAPE        -2  /* buffer or count does not match the plan        */
#define RF_ERANGE        -3  /* value out of the supported range               */
#define RF_EWORKSPACE    -4  /* workspace or table buffer too small            */
#define RF_EHIP          -5  /* the HIP runtime reported an error              */
#define RF_EUNSUPPORTED  -6  /* valid request this build does not implement    */

enum { RF_CF32 = 0, RF_CF16 = 1 };

/* Workspace queries (rf_workspace_bytes `op`). */
enum { RF_OP_IMAGE = 1, RF_OP_SEARCH = 2, RF_OP_SEGMENT = 3, RF_OP_SEGMENT_STEPS = 4 };

/*
 * Plan description: the pipeline state of section 3.2 (observation metadata
 * plus search preferences).  All arrays are host memory and are copied.
 *
 *  nint, nbl, nchan, npol  segment shape; npol in {1, 2}; nbl = number of
 *                          antenna pairs (section 2.2).
 *  vis_dtype               RF_CF32 or RF_CF16 storage of the segment.
 *  tint_s                  integration time, seconds (> 0).
 *  freq_ghz[nchan]         channel centre frequencies, GHz (> 0).
 *  uvw_m[nbl][3]           baseline coordinates, metres, constant over the
 *                          segment; w is ignored (zenith phase centre).
 *  dm[ndm]                 trial dispersion measures, pc cm^-3 (>= 0).
 *  width[nwidth]           trial boxcar widths, integrations (1..nint).
 *  npix                    image side N, a power of two in [64, 2048].
 *  du, dv                  uv cell size, wavelengths (> 0).
 *  kdm                     dispersion constant, s GHz^2 per pc cm^-3; the
 *                          section 2.1 footnote prints 4.15e-3.
 *  threshold               S/N threshold (section 3.1: typically 6).
 *  t_begin, t_end          candidates are kept only if their start
 *                          integration t = k * width is in [t_begin, t_end).
 */
typedef struct rf_plan_desc {
  int32_t nint, nbl, nchan, npol;
  int32_t vis_dtype;
  double tint_s;
  const double *freq_ghz;
  const double *uvw_m;
  const double *dm;
  int32_t ndm;
  const int32_t *width;
  int32_t nwidth;
  int32_t npix;
  double du, dv;
  double kdm;
  float threshold;
  int32_t t_begin, t_end;
} rf_plan_desc;

typedef struct rf_plan rf_plan;

typedef struct rf_plan_info {
  int64_t n_images;     /* ndm * sum_w floor(nint / w)                         */
  int32_t n_valid;      /* W: (baseline, channel) pairs inside the grid        */
  int32_t n_dropped;    /* nbl * nchan - W                                     */
  int32_t n_cells;      /* distinct occupied uv cells                          */
  int32_t n_rows;       /* grid rows v or -v of which holds an occupied cell   */
  int32_t max_delay;    /* largest delay in the table, integrations            */
  int32_t npix;
  size_t table_bytes;   /* bytes of the device table buffer actually used      */
  int32_t lanes;        /* tuning: lane streams of the fused search            */
  int32_t m_budget_mb;  /* tuning: all lanes' row-transformed batches, MB      */
} rf_plan_info;

/* One image's identity: DM trial index, width index, start integration. */
typedef struct rf_image_tag { int32_t dm_idx, width_idx, t_int; } rf_image_tag;

/* Per-image statistics (section 3.1 thresholding): signed peak at pixel
 * (x, y), sigma = 1.4826 * lower median of |image|, snr = peak / sigma (0
 * when sigma is 0). */
typedef struct rf_image_stats { float peak, sigma, snr; int32_t x, y; } rf_image_stats;

/* A candidate (section 3.3 candidate database record), 32 bytes. */
typedef struct rf_candidate {
  int32_t dm_idx, width_idx, t_int, x, y;
  float snr, peak, sigma;
} rf_candidate;

/* Human-readable name of a status code (static storage). */
const char *rf_status_string(rf_status s);

/*
 * rf_plan_table_bytes: size of the device buffer rf_plan_create needs for
 * `desc` (an upper bound that depends on the shapes only).  Validates desc.
 */
rf_status rf_plan_table_bytes(const rf_plan_desc *desc, size_t *bytes);

/*
 * rf_plan_create: validate `desc`, compute the plan tables and return a plan.
 * The integer delay table (section 2.1 footnote, delay relative to the top
 * channel, rounded half-even to whole integrations) and the nearest uv cell
 * of every (baseline, channel) are computed on the device in float64 with no
 * fused multiply-add.  The cell-sorted gather order and the occupied-row list
 * are derived on the host and uploaded.  d_tables must hold at least
 * rf_plan_table_bytes bytes and must outlive the plan.  Synchronises
 * `stream`.  On error *out is NULL and nothing is left allocated.
 */
rf_status rf_plan_create(const rf_plan_desc *desc, void *d_tables, size_t bytes,
                         void *stream, rf_plan **out);

/* rf_plan_destroy: free the host-side plan object (NULL is allowed). */
rf_status rf_plan_destroy(rf_plan *plan);

rf_status rf_plan_query(const rf_plan *plan, rf_plan_info *info);

/* Copy the delay table, int32 [ndm][nchan], to host memory (synchronous). */
rf_status rf_get_delays(const rf_plan *plan, int32_t *h_out);

/* Copy the cell table, int32 [nbl][nchan][2] = (iu, iv), to host memory. */
rf_status rf_get_cells(const rf_plan *plan, int32_t *h_out);

/* Workspace bytes for `op` on `nimg` images (RF_OP_IMAGE, RF_OP_SEARCH) or
 * for a whole segment (RF_OP_SEGMENT for rf_search_segment,
 * RF_OP_SEGMENT_STEPS for rf_search_segment_steps; nimg ignored). */
rf_status rf_workspace_bytes(const rf_plan *plan, int32_t op, int64_t nimg, size_t *bytes);

/*
 * rf_dedisperse (section 2.2: dedispersion in the visibility domain):
 *   d_out[t][b][c][p] = d_vis[t + d[dm_idx][c]][b][c][p]  if t + d < nint,
 *                       0                                  otherwise.
 * Both buffers are [nint][nbl][nchan][npol] of the plan's vis_dtype and must
 * not overlap.  A pure copy: bit-exact in either storage type.
 */
rf_status rf_dedisperse(const rf_plan *plan, int32_t dm_idx, const void *d_vis,
                        void *d_out, void *stream);

/*
 * rf_resample (Figure 2 loop over sampling time): decimating boxcar mean
 *   d_out[k] = (sum_{j<width} d_in[k*width + j]) / width,  k < nin / width,
 * accumulated in float32 in increasing j and scaled by the float reciprocal
 * of width (the quotient itself for powers of two; within one rounding of it
 * otherwise), as the fused search does.  d_in is [nin][nbl][nchan][npol]
 * of the plan's vis_dtype; d_out is RF_CF32 [nin / width][nbl][nchan][npol].
 */
rf_status rf_resample(const rf_plan *plan, int32_t width, const void *d_in, int32_t nin,
                      void *d_out, void *stream);

/*
 * rf_grid: Stokes I (mean of the two polarisations, section 3.1) gridded to
 * the nearest uv cell with unit weights:
 *   G[n][iv mod N][iu mod N] = sum over valid (b, c) in that cell of V_I,
 * summed in float32 in increasing b*nchan + c.  d_vis is RF_CF32
 * [nimg][nbl][nchan][npol]; d_grid is RF_CF32 [nimg][N][N] (fully written).
 */
rf_status rf_grid(const rf_plan *plan, const void *d_vis, int32_t nimg, void *d_grid,
                  void *stream);

/*
 * rf_image (section 3.2: 2-D FFT imaging):
 *   img[n][Y][X] = (1/W) Re sum_{iu,iv} G[n][iv][iu]
 *                  exp(+2 pi i (iu (X - N/2) + iv (Y - N/2)) / N),
 * float32 [nimg][N][N], phase centre at pixel (N/2, N/2).  Images are
 * transformed two at a time as the real and imaginary parts of one complex
 * FFT of their Hermitian-symmetrised grids.  d_ws: rf_workspace_bytes(
 * RF_OP_IMAGE, nimg) bytes.
 */
rf_status rf_image(const rf_plan *plan, const void *d_grid, int32_t nimg, float *d_img,
                   void *d_ws, size_t ws_bytes, void *stream);

/*
 * rf_image_static: rf_image for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same kernels and results as rf_image, bit for bit, but
 * the scratch between the row and column passes is a fixed array of the
 * library on each GPU (rf_image_static_max_bytes: 64 MiB, held until the
 * process ends) instead of a workspace argument; nothing is allocated.  The
 * call needs image_ws = ceil(nimg / 2) * rows * N * 8 bytes of it (rows: the
 * plan's n_rows): up to 16 images of 1024^2, 4 of 2048^2; larger nimg is
 * rejected with RF_EWORKSPACE.  Calls on one GPU share the array: calls
 * that overlap in time on that GPU (other streams, other threads) race.
 * RF_EINVAL on NULL, RF_ERANGE if nimg < 0; asynchronous on `stream`.
 */
rf_status rf_image_static(const rf_plan *plan, const void *d_grid, int32_t nimg, float *d_img,
                          void *stream);
rf_status rf_image_static_max_bytes(size_t *bytes);

/*
 * rf_search (section 3.1: threshold each image on S/N):
 * per image, peak = signed max (ties: lowest y*N + x), sigma = 1.4826 *
 * lower median of |img| (exact order statistic of rank floor((N*N-1)/2)),
 * snr = peak / sigma.  If snr > threshold and t_begin <= tag.t_int < t_end a
 * candidate is appended: slot = atomic increment of *d_ncand, written if
 * slot < cap.  *d_ncand ends as the true count; the caller zeroes it before
 * the first call and compares it with cap.  Candidate order is unspecified.
 * d_tags[nimg] (device) names each image; d_stats[nimg] may be NULL.
 */
rf_status rf_search(const rf_plan *plan, const float *d_img, int32_t nimg,
                    const rf_image_tag *d_tags, rf_image_stats *d_stats,
                    rf_candidate *d_cand, int32_t cap, int32_t *d_ncand,
                    void *d_ws, size_t ws_bytes, void *stream);

/*
 * rf_search_segment: the whole search of one segment (every DM trial, every
 * width, every integration; the loops of Figure 2), with the same results as
 * the chain rf_dedisperse -> rf_resample -> rf_grid -> rf_image -> rf_search.
 * Fused path: one pass over the segment per DM trial forms the resampled
 * Stokes I samples of every width, the uv grid is never materialised (rows
 * are gathered from cells) and no image is written to memory: the column
 * transform reduces each image to its peak and to the pixels that can hold
 * its lower median, bracketed around 0.6745 x its rms (known beforehand from
 * Parseval's theorem).  An image whose median falls outside the bracket is
 * recomputed exactly by the step chain, so sigma is always the exact lower
 * median.  d_vis: [nint][nbl][nchan][npol] of the plan's vis_dtype.  *d_ncand
 * is set to 0 on the device first.  d_stats (nullable) receives [n_images]
 * stats in (dm_idx, width_idx, k) order.  d_ws: rf_workspace_bytes(
 * RF_OP_SEGMENT).  Synchronises `stream` once before returning (to learn
 * whether any image needs the exact recomputation); that recomputation is
 * enqueued on `stream` after it, so the results are complete in `stream`
 * order, not necessarily when the call returns.
 */
rf_status rf_search_segment(const rf_plan *plan, const void *d_vis, rf_candidate *d_cand,
                            int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                            void *d_ws, size_t ws_bytes, void *stream);

/*
 * rf_search_segment in two calls, for callers that must not block while the
 * search runs.  rf_search_segment_begin checks the arguments as
 * rf_search_segment does, enqueues the fused search on `stream` (and lane
 * streams of its own, joined back to `stream`) and returns at once with a job;
 * nothing is enqueued on error (*job is then NULL).  rf_search_segment_end
 * waits for the search (one synchronisation of `stream`), enqueues the exact
 * recomputation of the images whose median left the bracket on `stream` and
 * frees the job; its status is the search's.  The results are complete in
 * `stream` order after rf_search_segment_end (as after rf_search_segment).
 * Between the two calls every buffer stays in use by the search; every
 * begin must be ended once.  Results are those of rf_search_segment, bit
 * for bit.
 */
typedef struct rf_segment_job rf_segment_job;
rf_status rf_search_segment_begin(const rf_plan *plan, const void *d_vis, rf_candidate *d_cand,
                                  int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                                  void *d_ws, size_t ws_bytes, void *stream,
                                  rf_segment_job **job);
rf_status rf_search_segment_end(rf_segment_job *job);

/* Device time of the fused path's kernels, per kernel kind, measured with
 * HIP events on the stream each kernel is launched on
 * (rf_search_segment_profile). */
enum { RF_K_DRS = 0, RF_K_ROWS = 1, RF_K_COLS = 2, RF_K_SELECT = 3, RF_K_FALLBACK = 4,
       RF_K_GRID = 5, RF_NK = 8 };
typedef struct rf_kernel_times {
  int32_t concurrent;      /* in: 0 = every launch in order on `stream`, so that
                              durations do not overlap; 1 = the streams and order
                              of rf_search_segment (concurrent batches: one
                              kernel's duration includes the time it shares the
                              device with the other streams' kernels)          */
  int32_t sample;          /* in: time every sample-th launch of each kind (the
                              first included); 0 or 1 = every launch.  Events
                              around every launch delay the next launch on the
                              stream and change how the streams overlap; a
                              sparse sample keeps the schedule of
                              rf_search_segment                                */
  double ms[RF_NK];        /* out: summed event-timed duration, milliseconds   */
  int64_t launches[RF_NK]; /* out: number of launches timed                    */
} rf_kernel_times;

/*
 * rf_search_segment_profile: rf_search_segment with an event pair recorded
 * around the sampled kernel launches; ms and launches of *times receive the
 * summed durations per kernel kind (concurrent and sample are read, then
 * kept).  Results are identical to rf_search_segment; with every launch timed
 * the extra events (and a synchronisation every 16384 launches timed) make it
 * slower, so time throughput with rf_search_segment or a sparse sample.
 * RF_EINVAL if concurrent is not 0 or 1, RF_ERANGE if sample < 0.
 */
rf_status rf_search_segment_profile(const rf_plan *plan, const void *d_vis, rf_candidate *d_cand,
                                    int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                                    void *d_ws, size_t ws_bytes, void *stream,
                                    rf_kernel_times *times);

/*
 * rf_search_segment_steps: the same search driven as the plain chain of the
 * step entry points above (dense grids and images in the workspace), kept as
 * the reference path that the fused one is measured against.  Asynchronous.
 * d_ws: rf_workspace_bytes(RF_OP_SEGMENT_STEPS).
 */
rf_status rf_search_segment_steps(const rf_plan *plan, const void *d_vis, rf_candidate *d_cand,
                                  int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                                  void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop over streamed segments (Law et al. 2018, section
 * 3.2: the correlator output is cut into independent, overlapping segments
 * that the search cluster processes as they arrive).  A segment is released
 * (submitted) when its last integration has arrived; it is admitted when one
 * of the server's slots is free and its device block fits in the caller's
 * arena (first fit; among waiting segments the earliest that fits goes
 * first), copied host to device on the slot's stream, searched with
 * rf_search_segment, and its candidates are copied back.  Slots run
 * concurrently, so segments of different plans (shapes) overlap on the device.
 * ------------------------------------------------------------------------ */
typedef struct rf_server rf_server;

typedef struct rf_serve_times {
  double released_s;  /* submission, seconds since the server was created */
  double started_s;   /* admission                                        */
  double done_s;      /* candidates on the host                           */
  double latency_s;   /* done - released                                  */
} rf_serve_times;

/* Device bytes one request of `plan` with candidate capacity `cap` takes from
 * the arena: segment copy + rf_workspace_bytes(RF_OP_SEGMENT) + cap rows +
 * the count, each 256-byte aligned.  RF_EINVAL on NULL, RF_ERANGE if cap < 0. */
rf_status rf_server_request_bytes(const rf_plan *plan, int32_t cap, size_t *bytes);

/* Starts nslots (1..16) slot threads on the current device, each with its own
 * stream (default priority).  d_arena: caller-owned device memory of
 * arena_bytes (256-byte aligned), used until rf_server_destroy returns; the
 * server allocates no device memory.  RF_EINVAL on NULL, zero size or a
 * misaligned arena; RF_ERANGE for nslots outside 1..16; RF_EHIP if the
 * current device cannot be read. */
rf_status rf_server_create(void *d_arena, size_t arena_bytes, int32_t nslots, rf_server **out);

/* Releases one segment: h_vis is host memory in the plan's segment layout
 * (pinned memory makes the copy asynchronous); it and the plan must stay
 * valid until rf_server_wait returns for the ticket.  Returns at once.
 * flags: 0 or a combination of
 *   RF_SERVE_SUBTRACT_MEAN    run rf_subtract_mean on the device copy before
 *                             the search;
 *   RF_SERVE_FAIL_AFTER_COPY  fault injection for tests of the error path:
 *                             the slot enqueues the copy (and the mean
 *                             subtraction) and then fails the request with
 *                             RF_EHIP without searching.
 * A request that fails has its slot stream drained before its arena block is
 * reused, so no later request is admitted into memory still being written.
 * RF_EWORKSPACE if the request could never fit in the arena, RF_EINVAL on
 * NULL arguments, unknown flags or after rf_server_destroy began, RF_ERANGE
 * if cap < 0. */
enum { RF_SERVE_SUBTRACT_MEAN = 1, RF_SERVE_FAIL_AFTER_COPY = 2 };
rf_status rf_server_submit(rf_server *server, const rf_plan *plan, const void *h_vis, int32_t cap,
                           int32_t flags, int64_t *ticket);

/* Blocks until the ticket's segment is done, then copies min(count, cap)
 * candidate rows (device order) to h_cand, the true count to *ncand and the
 * timestamps to *times (nullable); the ticket is then forgotten (a second
 * wait on it returns RF_EINVAL).  Returns the search's status. */
rf_status rf_server_wait(rf_server *server, int64_t ticket, rf_candidate *h_cand, int32_t cap,
                         int32_t *ncand, rf_serve_times *times);

/* Runs every released segment to completion, stops the slots and frees the
 * server (results not collected are dropped).  Must not overlap other calls
 * on the same server. */
rf_status rf_server_destroy(rf_server *server);

/*
 * rf_subtract_mean (section 3.1: the mean visibility in time is subtracted on
 * timescales below the fringe rate, removing constant sources; section 3.2:
 * a segment is about that long): in place on d_vis (the plan's segment
 * layout and storage type), every (baseline, channel, polarisation) value
 * loses its mean over the segment's nint integrations (summed in float64,
 * subtracted in float32; CF16 storage rounded back to nearest even).
 * Asynchronous on `stream`.  RF_EINVAL on NULL.
 */
rf_status rf_subtract_mean(const rf_plan *plan, void *d_vis, void *stream);

/* ------------------------------------------------------------------------
 * Synthetic data: mock transients and counter-based noise.
 * ------------------------------------------------------------------------ */

/* A mock transient (section 3.3: mock sources are inserted into calibrated
 * data to measure the search's efficiency and sensitivity): a dispersed
 * boxcar point source.  48 bytes. */
typedef struct rf_mock {
  double dm;     /* pc cm^-3; sweep follows the plan's kdm (section 2.1 footnote) */
  double t0;     /* arrival at the highest channel, integrations from the
                    buffer's first integration (fractional allowed)            */
  double width;  /* duration in integrations, > 0 (fractional allowed)        */
  double l, m;   /* direction cosines from the phase centre                   */
  double amp;    /* flux in visibility units, the same in every polarisation  */
} rf_mock;

/* Adds mocks[0..nmock) (host array, read before the call returns) to d_vis in
 * place: the plan's segment layout and storage type, nint integrations that
 * are integrations t_first .. t_first + nint - 1 of the segment the mocks'
 * t0 refer to.  In channel c a mock occupies [s, s + width) integrations with
 * s = t0 + ((kdm * dm) * (1/(nu_c*nu_c) - 1/(nu_top*nu_top))) / t_int;
 * integration t receives amp * |[t, t+1) overlap| * exp(-2 pi i (u l + v m)),
 * u and v the baseline in wavelengths at nu_c, in every polarisation.  Lag,
 * overlap and phase are float64 operations in that order (no contraction),
 * in absolute integrations, so a segment filled window by window gets the
 * same values as one filled at once.  Each mock's sum with the stored value is
 * rounded once to the storage type (nearest even), mocks in array order.
 * Parts of a sweep outside the window are dropped.  With CF16 storage a
 * per-sample signal of a few float16 spacings of the stored values is
 * quantised against them without dither (a unit-noise segment loses about
 * 0.4% of a 4e-3 signal): to model data whose signal was present before
 * storage, inject into CF32 and round once.  Asynchronous on `stream`.
 * RF_EINVAL on NULL or nmock < 0, RF_ERANGE for a non-finite field,
 * width <= 0, |t0| > 1e15, |dm| > 1e9 or t_first outside [0, 2^50]. */
rf_status rf_inject(const rf_plan *plan, const rf_mock *h_mocks, int32_t nmock, int64_t t_first,
                    void *d_vis, void *stream);

/* Fills d_vis (the plan's segment layout and storage, nint integrations) with
 * complex Gaussian noise, Re and Im each N(0, 1), of integrations t_first ..
 * t_first + nint - 1 of a stream: complex element e = ((t * nbl + b) * nchan
 * + c) * npol + p (t absolute) takes Philox4x32-10 (Salmon et al. 2011)
 * block e/2, counter (e/2 mod 2^32, e/2 div 2^32, stream, 0), key (seed mod
 * 2^32, seed div 2^32); words (x0, x1) for even e, (x2, x3) for odd e give
 * u = (x + 1/2) 2^-32 and the Box-Muller pair (Box and Muller 1958)
 * sqrt(-2 ln u_a) (cos, sin)(2 pi u_b) in float64, rounded to float32 (CF16:
 * those float32 values rounded to nearest even).  Every element depends only
 * on (seed, stream, e), so overlapping windows hold the same values.  Not
 * part of the search; a source of large synthetic segments on the device.
 * Asynchronous on `stream`.  RF_EINVAL on NULL, RF_ERANGE if t_first < 0 or
 * the last element index would pass 2^61. */
rf_status rf_noise(const rf_plan *plan, uint64_t seed, uint32_t stream_id, int64_t t_first,
                   void *d_vis, void *stream);

/* ------------------------------------------------------------------------
 * Periodicity search (section 3.1 footnote: a time segment is Fourier
 * transformed to frequencies and each frequency imaged; Figure 2 caption: a
 * modification of the innermost loop).
 * ------------------------------------------------------------------------ */

/* Workspace of rf_search_periodic: the fluctuation spectrum of one DM trial
 * (nint/2 x nbl x nchan complex64), one batch of frequency grids, images and
 * amplitude images, the imaging scratch.  RF_ERANGE unless nint is a power
 * of two in [2, 8192]. */
rf_status rf_periodic_workspace_bytes(const rf_plan *plan, size_t *bytes);

/* For every DM trial i of the plan: the segment is dedispersed (zero past its
 * end), Stokes I formed, and the fluctuation spectrum taken along time per
 * (baseline, channel): F[f] = (1/T) sum_t V_I[t] exp(-2 pi i f t / T), T =
 * nint.  Each frequency f = 1 .. T/2 is gridded like an integration and
 * imaged without taking the real part: I_f = (1/W) sum G e^{+2 pi i (...)/N}
 * (complex).  Its amplitude |I_f| gives peak (ties to the lowest y*N + x),
 * sigma = lower median of |I_f| / sqrt(2 ln 2) (the noise per quadrature of a
 * complex Gaussian image) and snr = peak / sigma; a candidate row is written
 * when snr > threshold.  Rows use rf_candidate with width_idx = -1 and
 * t_int = f; peak is the amplitude (the candidate window [t_begin, t_end)
 * does not apply).  d_stats (nullable) receives [ndm][nint/2] stats, row f-1.
 * *d_ncand is set to the true count (rows beyond cap dropped).  Widths are
 * not used.  Asynchronous on `stream`.  RF_EINVAL on NULL, RF_ERANGE if
 * nint is not a power of two in [2, 8192] or cap < 0, RF_EWORKSPACE if
 * ws_bytes is too small. */
rf_status rf_search_periodic(const rf_plan *plan, const void *d_vis, rf_candidate *d_cand,
                             int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats, void *d_ws,
                             size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Second-tier candidate products (section 3.1: candidates above a second,
 * higher threshold, typically 7 sigma, get visualisations; section 3.3: the
 * candidate's image and spectrum).
 * ------------------------------------------------------------------------ */

/* The second tier itself: copies, in order, the rows of h_in[0..n) whose
 * snr exceeds `threshold` (strictly; section 3.1 names about 7 sigma) to
 * h_out, at most cap of them; *nout receives the number of rows that pass
 * (which may exceed cap).  Host memory only; nothing runs on the device.
 * h_out may equal h_in (filtering in place).  RF_EINVAL on NULL (h_in and
 * h_out may be NULL when n, respectively cap, is 0), RF_ERANGE if n < 0,
 * cap < 0 or the threshold is not finite. */
rf_status rf_select_tier(const rf_candidate *h_in, int32_t n, float threshold,
                         rf_candidate *h_out, int32_t cap, int32_t *nout);

/* Workspace of rf_candidate_products for nspec spectrum rows: the gathered
 * rows (nspec x nbl x nchan x npol complex64), one grid, one image and the
 * imaging scratch of one image.  RF_ERANGE unless 1 <= nspec <= 4096. */
rf_status rf_products_workspace_bytes(const rf_plan *plan, int32_t nspec, size_t *bytes);

/* For each of h_cand[0..ncand) (host rows as the search returns them; the
 * caller picks the tier, e.g. snr > 7; read before the call returns), from
 * the segment d_vis the search ran on:
 *   d_cutout [ncand][2 half][2 half] float (nullable): the window of the
 *     candidate's image (DM trial dm_idx, width width_idx, resampled
 *     integration t_int / w) with the candidate pixel at (half, half),
 *     wrapping at the image edges;
 *   d_spec [ncand][nspec][nchan] float (nullable): the dedispersed dynamic
 *     spectrum toward the candidate pixel: row s is resampled integration
 *     t_int / w - nspec/2 + s (zero outside the segment), channel c the mean
 *     over its gridded baselines of Re(V_I exp(+2 pi i (iu (x - N/2) +
 *     iv (y - N/2)) / N)), zero for a channel with none.  Weighted by the
 *     channel's gridded baselines and divided by W a row sums to that row's
 *     image pixel.
 * Asynchronous on `stream`; d_ws (rf_products_workspace_bytes) is reused
 * candidate after candidate.  RF_EINVAL on NULL arguments or ncand < 0,
 * RF_ERANGE for half outside [1, N/2], nspec outside [1, 4096] or a row that
 * names no image of the plan (index, t_int not a multiple of the width, pixel
 * outside the image), RF_EWORKSPACE if ws_bytes is too small. */
rf_status rf_candidate_products(const rf_plan *plan, const void *d_vis, const rf_candidate *h_cand,
                                int32_t ncand, int32_t half, int32_t nspec, float *d_cutout,
                                float *d_spec, void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Tuning and batches.
 * ------------------------------------------------------------------------ */

/* Sets how the fused search schedules its work: `lanes` (1..4) concurrent
 * batch pipelines (streams) and `m_budget_mb` (16..4096) for the row-
 * transformed batches of all lanes together (image pairs per batch follow
 * from it).  Results do not depend on either (the same arithmetic per
 * image); speed does.  Defaults 2 and 240 (1920 for 2048^2 images).  Changes
 * rf_workspace_bytes(RF_OP_SEGMENT): call before sizing workspaces, and not
 * while the plan is in use.  RF_EINVAL on NULL, RF_ERANGE out of range. */
rf_status rf_plan_set_tuning(rf_plan *plan, int32_t lanes, int32_t m_budget_mb);

/* A batch: the fused searches of nseg segments (plans of any shapes) bound
 * once and run by one rf_batch_run call (section 3.2: segments are
 * independent units of work).  The segments run in order and share one
 * workspace. */
typedef struct rf_batch rf_batch;

/* Workspace of a batch over plans[0..nseg): the largest segment workspace
 * plus one fallback list per segment. */
rf_status rf_batch_workspace_bytes(const rf_plan *const *plans, int32_t nseg, size_t *bytes);

/* rf_batch_create flags. */
enum { RF_BATCH_GRAPH = 1 };

/* Binds the batch.  Every buffer is bound now and read or written by every
 * rf_batch_run: per segment i, d_vis[i] (the plan's segment layout),
 * d_cand[i] (cap[i] rows), d_ncand[i], d_stats[i] (d_stats may be NULL, or
 * entries NULL); d_ws of rf_batch_workspace_bytes.  All caller-owned and
 * kept alive until rf_batch_destroy; the plans must not be retuned meanwhile.
 * flags: 0.  RF_BATCH_GRAPH (capture every segment's search once into HIP
 * graphs, each run a few graph launches) is refused with RF_EUNSUPPORTED in
 * this build: its runs ended the host process with a segmentation fault
 * inside the capture, with no cause found in the capture sequence.  Nothing
 * runs on the device until rf_batch_run.  RF_EINVAL on NULL arguments,
 * nseg < 1 or unknown flags, RF_ERANGE on a negative cap, RF_EWORKSPACE if
 * ws is too small, RF_EHIP if the batch's streams cannot be created (nothing
 * is left allocated). */
rf_status rf_batch_create(const rf_plan *const *plans, int32_t nseg, const void *const *d_vis,
                          rf_candidate *const *d_cand, const int32_t *cap,
                          int32_t *const *d_ncand, rf_image_stats *const *d_stats, void *d_ws,
                          size_t ws_bytes, int32_t flags, rf_batch **out);

/* Nodes of the batch's captured graph (0 without RF_BATCH_GRAPH). */
rf_status rf_batch_graph_nodes(const rf_batch *batch, size_t *nodes);

/* Runs every segment's fused search, enqueued on `stream` and the batch's
 * lane streams, then recomputes exactly the images whose median left the
 * bracket (one synchronisation of `stream` per segment).  Results as
 * rf_search_segment on each segment, bit for bit. */
rf_status rf_batch_run(rf_batch *batch, void *stream);

rf_status rf_batch_destroy(rf_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* RF_H */
